"""Mutation checks of the oracle's pins (CPU only).

Each case plants one plausible mistake in the oracle (on the CPU, through
monkeypatch, restored afterwards) and asserts that at least one of the pins
named for it fails.  A pin that keeps passing on a planted mistake would not
protect the parity tests that trust the oracle.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from oracle import spectral_ns as ons

import test_oracle_mlp_pins as mlp_pins
import test_oracle_pins as pins

_orig = {
    "curl": ons.curl,
    "cross": ons.cross,
    "rhs": ons.rhs,
    "target": omlp.surrogate_target,
}


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


# ---------------------------------------------------------------------------
# the transform-based right-hand side and RK4 (Eq. NSfinal, Sec. 2)
# ---------------------------------------------------------------------------
def _mask_le(N, dealias="two_thirds"):
    kx, ky, kz = ons.wavenumbers(N)
    m = (3 * np.abs(kx) <= N) & (3 * np.abs(ky) <= N) & (3 * np.abs(kz) <= N)
    return np.broadcast_to(m, (N, N, N // 2 + 1)).copy()


def _rhs_no_projection(uh, nu, dealias="two_thirds"):
    N = uh.shape[1]
    M = ons.retained_mask(N, dealias)
    uh = uh * M
    c = ons.cross(ons.inverse(uh, N), ons.inverse(ons.curl(uh), N))
    Nh = ons.forward(c) * M
    kx, ky, kz = ons.wavenumbers(N)
    return Nh - nu * (kx * kx + ky * ky + kz * kz) * uh


def _rk4_equal_weights(uh, nu, dt, dealias="two_thirds"):
    N = uh.shape[1]
    uh = uh * ons.retained_mask(N, dealias)
    k1 = ons.rhs(uh, nu, dealias)
    k2 = ons.rhs(uh + 0.5 * dt * k1, nu, dealias)
    k3 = ons.rhs(uh + 0.5 * dt * k2, nu, dealias)
    k4 = ons.rhs(uh + dt * k3, nu, dealias)
    return uh + (dt / 4.0) * (k1 + k2 + k3 + k4)


def _set(monkeypatch, name, fn):
    """Replace a function both in its module and in the oracle package."""
    monkeypatch.setattr(ons, name, fn)
    monkeypatch.setattr(oracle, name, fn)


def test_curl_sign_is_caught(monkeypatch):
    _set(monkeypatch, "curl", lambda uh: -_orig["curl"](uh))
    assert _fails(pins.test_taylor_green_rhs_closed_form, 16)


def test_cross_product_order_is_caught(monkeypatch):
    _set(monkeypatch, "cross", lambda a, b: _orig["cross"](b, a))
    assert _fails(pins.test_taylor_green_rhs_closed_form, 16)
    assert _fails(pins.test_cross_matches_numpy_cross)


def test_non_strict_mask_is_caught(monkeypatch):
    _set(monkeypatch, "retained_mask", _mask_le)
    assert _fails(pins.test_mask_is_the_strict_two_thirds_rule, 18)


def test_viscous_sign_is_caught(monkeypatch):
    _set(monkeypatch, "rhs", lambda uh, nu, dealias="two_thirds": _orig["rhs"](uh, -nu, dealias))
    assert _fails(pins.test_taylor_green_rhs_closed_form, 16)
    assert _fails(pins.test_beltrami_exact_rk4_decay, 9, 16)


def test_missing_projection_is_caught(monkeypatch):
    _set(monkeypatch, "rhs", _rhs_no_projection)
    assert _fails(pins.test_taylor_green_rhs_closed_form, 16)


def test_rk4_weights_are_caught(monkeypatch):
    _set(monkeypatch, "rk4_step", _rk4_equal_weights)
    assert _fails(pins.test_beltrami_exact_rk4_decay, 9, 16)


# ---------------------------------------------------------------------------
# the surrogate's target, warm start and gradient (the integrator of Sec. 2
# is left open; the implicit step and its warm start are this library's)
# ---------------------------------------------------------------------------
def _set_mlp(monkeypatch, name, fn):
    monkeypatch.setattr(omlp, name, fn)
    monkeypatch.setattr(oracle, name, fn)


def _predict_mut(kind):
    def predict(theta, u, d1, d2, nu, dt, bf16=False, dealias="two_thirds"):
        N = u.shape[1]
        idx = np.nonzero(ons.retained_mask(N, dealias))
        F, s = omlp.surrogate_features(u, d1, d2, nu, dt, dealias)
        Y, _ = omlp.mlp_forward(theta, F, bf16)
        base = 2.0 * omlp._vec(d1, idx) - omlp._vec(d2, idx)
        rows = {"drop_s": base + Y, "sign": base - s[:, None] * Y, "s2": base + (s * s)[:, None] * Y}[kind]
        out = np.zeros_like(u)
        c = rows.reshape(-1, 3, 2)
        for comp in range(3):
            out[comp][idx] = c[:, comp, 0] + 1j * c[:, comp, 1]
        return out
    return predict


def _grad_without_tanh_derivative(theta, X, T, bf16=False):
    P = omlp.mlp_unpack(theta)
    Y, acts = omlp.mlp_forward(theta, X, bf16)
    R = Y - T
    loss = float(np.mean(R * R))
    dZ = 2.0 * R / R.size
    grads = {}
    for layer in (4, 3, 2, 1):
        grads[f"W{layer}"] = dZ.T @ acts[layer - 1]
        grads[f"b{layer}"] = dZ.sum(axis=0)
        if layer > 1:
            dZ = dZ @ P[f"W{layer}"]  # the factor 1 - h^2 of tanh is missing
    return loss, np.concatenate([grads[name].ravel() for name, _ in omlp.mlp_shapes()])


@pytest.mark.parametrize("kind", ["sign", "scale_s2", "drop_s", "extrapolation"])
def test_target_mutations_are_caught(monkeypatch, kind):
    orig = _orig["target"]

    def target(d, d1, d2, s, dealias="two_thirds"):
        safe = np.where(s > 0, s, 1.0)[:, None]
        if kind == "sign":
            return -orig(d, d1, d2, s, dealias)
        if kind == "scale_s2":
            return orig(d, d1, d2, s, dealias) / safe
        if kind == "drop_s":
            return orig(d, d1, d2, s, dealias) * s[:, None]
        return orig(d + d1 - d2, d1, d2, s, dealias)  # (d - d1)/s: extrapolation by d1 alone
    _set_mlp(monkeypatch, "surrogate_target", target)
    assert _fails(mlp_pins.test_target_by_hand_on_two_modes)


@pytest.mark.parametrize("kind", ["drop_s", "sign", "s2"])
def test_predict_mutations_are_caught(monkeypatch, kind):
    _set_mlp(monkeypatch, "surrogate_predict", _predict_mut(kind))
    assert _fails(mlp_pins.test_predict_adds_s_times_the_network_output)


def test_gradient_without_tanh_derivative_is_caught(monkeypatch):
    _set_mlp(monkeypatch, "mlp_loss_grad", _grad_without_tanh_derivative)
    assert _fails(mlp_pins.test_gradient_matches_central_differences)


def test_unmutated_pins_pass():
    # the same pin calls with nothing planted: the failures above come from
    # the mutations alone
    pins.test_taylor_green_rhs_closed_form(16)
    pins.test_cross_matches_numpy_cross()
    pins.test_mask_is_the_strict_two_thirds_rule(18)
    pins.test_beltrami_exact_rk4_decay(9, 16)
    mlp_pins.test_target_by_hand_on_two_modes()
    mlp_pins.test_predict_adds_s_times_the_network_output()
    mlp_pins.test_gradient_matches_central_differences()
