"""FP64 NumPy reference of the per-mode MLP surrogate (forward, loss,
backward, Adam) and of its input features.

TEST INFRASTRUCTURE.  Only the tests use this module; the GPU library shares
no code with it.

The surrogate warm-starts the Picard iteration of the implicit-midpoint step
(see implicit_midpoint.py).  It is not in the paper: Sec. 2 leaves the time
integrator open, and an iteration needs a starting guess.  Per retained mode
k it maps features of the state and of the two previous increments to a
correction of the plain predictor:

    d_pred = 2 D1 - D2 + s * y,   y = MLP(f),   s = ||D1_k||

with D1, D2 the increments of the two previous steps (newest first) and
||.|| the norm of the 3-component complex vector at mode k.

Features (32 per mode, in this order; zero when s = 0):
  f[0:6]    D1 / s              (re, im of components x, y, z)
  f[6:12]   D2 / s
  f[12:18]  dt F_NL^{n-1} / s, with dt F_NL^{n-1} = (1 - a) D1 + 2 a u^n,
            the nonlinear forcing of the previous step at its fixed point
  f[18:24]  u^n / ||u^n_k||     (0 where u^n_k = 0)
  f[24]     s / ||u^n_k||       (0 where u^n_k = 0)
  f[25:28]  k / N
  f[28]     a = dt nu |k|^2 / 2
  f[29:32]  0
Target: (D - (2 D1 - D2)) / s for the increment D of the step.

MLP: 32 -> 256 -> 256 -> 256 -> 6, tanh on the hidden layers, linear output.
Parameters, one flat FP32 vector in this order (weights W[out][in]):
  W1[256][32] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[6][256] b4[6].
Loss: mean over rows and outputs of (y - t)^2.

With bf16=True every matrix-product operand is rounded to bfloat16 (round to
nearest even, through float32) before the product, as the GPU kernels do
with their BF16 MFMA operands.  Products accumulate in FP64 here (FP32 on
the GPU).
"""
from __future__ import annotations

import numpy as np

from .spectral_ns import retained_mask, wavenumbers

__all__ = [
    "MLP_IN",
    "MLP_HIDDEN",
    "MLP_OUT",
    "mlp_shapes",
    "mlp_param_count",
    "mlp_unpack",
    "mlp_init",
    "bf16_round",
    "mlp_forward",
    "mlp_loss_grad",
    "adam_step",
    "surrogate_features",
    "surrogate_target",
    "surrogate_predict",
]

MLP_IN, MLP_HIDDEN, MLP_OUT = 32, 256, 6


def mlp_shapes():
    """(name, shape) of each parameter block, in storage order."""
    H = MLP_HIDDEN
    return [("W1", (H, MLP_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
            ("W4", (MLP_OUT, H)), ("b4", (MLP_OUT,))]


def mlp_param_count() -> int:
    return int(sum(np.prod(s) for _, s in mlp_shapes()))


def mlp_unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in mlp_shapes():
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def mlp_init(seed: int) -> np.ndarray:
    """Uniform +-1/sqrt(fan_in) weights and zero biases, as FP32 values."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in mlp_shapes():
        if name.startswith("W"):
            lim = 1.0 / np.sqrt(shape[1])
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via float32; returned as
    float64.  NaN and infinity are not expected here."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, bf16):
    return bf16_round(x) if bf16 else x


def mlp_forward(theta: np.ndarray, X: np.ndarray, bf16: bool = False):
    """Returns (Y, activations [X, H1, H2, H3])."""
    P = mlp_unpack(theta)
    acts = [X]
    h = X
    for layer in (1, 2, 3):
        W, b = P[f"W{layer}"], P[f"b{layer}"]
        h = np.tanh(_q(h, bf16) @ _q(W, bf16).T + b)
        if bf16:
            h = h.astype(np.float32).astype(np.float64)  # stored as FP32 on the GPU
        acts.append(h)
    Y = _q(h, bf16) @ _q(P["W4"], bf16).T + P["b4"]
    return Y, acts


def mlp_loss_grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray, bf16: bool = False):
    """Mean squared error and its gradient with respect to theta, by
    backpropagation through the layers of mlp_forward."""
    P = mlp_unpack(theta)
    Y, acts = mlp_forward(theta, X, bf16)
    rows = X.shape[0]
    R = Y - T
    loss = float(np.mean(R * R))
    dZ = 2.0 * R / R.size
    if bf16:
        dZ = dZ.astype(np.float32).astype(np.float64)
    grads = {}
    for layer in (4, 3, 2, 1):
        W = P[f"W{layer}"]
        A = acts[layer - 1]
        grads[f"W{layer}"] = _q(dZ, bf16).T @ _q(A, bf16)
        grads[f"b{layer}"] = dZ.sum(axis=0)
        if layer > 1:
            dH = _q(dZ, bf16) @ _q(W, bf16)
            dZ = dH * (1.0 - A * A)
            if bf16:
                dZ = dZ.astype(np.float32).astype(np.float64)
    g = np.concatenate([grads[name].ravel() for name, _ in mlp_shapes()])
    assert rows == X.shape[0]
    return loss, g


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015), bias-corrected; step counts
    from 1.  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def _modes(N, dealias):
    """Retained half-spectrum modes in canonical (kx, ky, kz) index order."""
    M = retained_mask(N, dealias)
    return np.nonzero(M)


def _vec(a, idx):
    """[rows, 6] real view (re, im per component) of a [3][N][N][N/2+1] field."""
    v = a[:, idx[0], idx[1], idx[2]].T  # rows x 3 complex
    return np.stack([v.real, v.imag], axis=-1).reshape(v.shape[0], 6)


def surrogate_features(u: np.ndarray, d1: np.ndarray, d2: np.ndarray, nu: float, dt: float,
                       dealias: str = "two_thirds"):
    """Features [rows, 32] and scales s [rows] of the retained modes of a
    state u^n with previous increments d1 (newest) and d2."""
    N = u.shape[1]
    idx = _modes(N, dealias)
    kx, ky, kz = (np.broadcast_to(k, (N, N, N // 2 + 1))[idx] for k in wavenumbers(N))
    a = 0.5 * dt * nu * (kx * kx + ky * ky + kz * kz)
    U, D1, D2 = _vec(u, idx), _vec(d1, idx), _vec(d2, idx)
    s = np.sqrt(np.sum(D1 * D1, axis=1))
    nu_ = np.sqrt(np.sum(U * U, axis=1))
    F = np.zeros((len(s), MLP_IN))
    live = s > 0
    inv = np.where(live, 1.0 / np.where(live, s, 1.0), 0.0)[:, None]
    F[:, 0:6] = D1 * inv
    F[:, 6:12] = D2 * inv
    F[:, 12:18] = ((1.0 - a)[:, None] * D1 + 2.0 * a[:, None] * U) * inv
    hasu = nu_ > 0
    invu = np.where(hasu, 1.0 / np.where(hasu, nu_, 1.0), 0.0)
    F[:, 18:24] = U * invu[:, None]
    F[:, 24] = s * invu
    F[:, 25] = kx / N
    F[:, 26] = ky / N
    F[:, 27] = kz / N
    F[:, 28] = a
    F[~live] = 0.0
    return F, s


def surrogate_target(d: np.ndarray, d1: np.ndarray, d2: np.ndarray, s: np.ndarray, dealias: str = "two_thirds"):
    """Target rows (d - (2 d1 - d2)) / s of the retained modes (0 where s = 0)."""
    N = d.shape[1]
    idx = _modes(N, dealias)
    R = _vec(d, idx) - (2.0 * _vec(d1, idx) - _vec(d2, idx))
    live = s > 0
    return np.where(live[:, None], R / np.where(live, s, 1.0)[:, None], 0.0)


def surrogate_predict(theta, u, d1, d2, nu, dt, bf16=False, dealias: str = "two_thirds"):
    """The warm-start increment 2 d1 - d2 + s MLP(f), as a half-spectrum
    field (zero outside the retained set)."""
    N = u.shape[1]
    idx = _modes(N, dealias)
    F, s = surrogate_features(u, d1, d2, nu, dt, dealias)
    Y, _ = mlp_forward(theta, F, bf16)
    base = 2.0 * _vec(d1, idx) - _vec(d2, idx)
    rows = base + s[:, None] * Y
    out = np.zeros_like(u)
    c = rows.reshape(-1, 3, 2)
    for comp in range(3):
        out[comp][idx] = c[:, comp, 0] + 1j * c[:, comp, 1]
    return out
