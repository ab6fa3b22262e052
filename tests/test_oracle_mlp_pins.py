"""Pins of the MLP reference (CPU): the analytic gradient against central
finite differences, the BF16 rounding against exactly known values, Adam
against its closed form on a quadratic, and the surrogate features against
their definitions on hand-made fields."""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import inputs


def test_param_count():
    assert oracle.mlp_param_count() == 256 * 32 + 256 + 2 * (256 * 256 + 256) + 6 * 256 + 6


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = oracle.mlp_init(1) * 3.0  # larger weights: the tanh curvature matters
    X = rng.standard_normal((7, 32))
    T = rng.standard_normal((7, 6))
    _, g = oracle.mlp_loss_grad(theta, X, T)
    # a sample of coordinates from every parameter block
    offs, o = [], 0
    for _, shape in oracle.mlp_shapes():
        n = int(np.prod(shape))
        offs += list(o + rng.choice(n, size=min(n, 6), replace=False))
        o += n
    h = 1e-6
    for i in offs:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (oracle.mlp_loss_grad(theta + e, X, T)[0] - oracle.mlp_loss_grad(theta - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-9, -3.0, 1.0 + 2.0**-7 + 2.0**-8, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0**-7, -3.0, 1.0 + 2.0**-6, 0.0])
    # 1 + 2^-8 is a tie below 1 + 2^-7: ties go to the even mantissa (1.0);
    # 1 + 2^-7 + 2^-8 is a tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    np.testing.assert_array_equal(oracle.bf16_round(x), want)
    r = np.random.default_rng(1).standard_normal(1000)
    q = oracle.bf16_round(r)
    assert np.all(np.abs(q - r) <= np.abs(r) * 2.0**-8)
    assert np.all(q.astype(np.float32).view(np.uint32) & 0xFFFF == 0)


def test_bf16_forward_stays_close_to_fp64():
    rng = np.random.default_rng(2)
    theta = oracle.mlp_init(3)
    X = rng.standard_normal((50, 32))
    y64, _ = oracle.mlp_forward(theta, X)
    y16, _ = oracle.mlp_forward(theta, X, bf16=True)
    assert np.linalg.norm(y16 - y64) <= 3e-2 * np.linalg.norm(y64)


def test_adam_closed_form_first_step_and_descent():
    # first step: m_hat = g, v_hat = g^2 -> update = -lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = oracle.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.1, eps=0.0)
    np.testing.assert_allclose(th, -0.1 * np.sign(g), rtol=1e-15)
    # minimising (x - 3)^2 converges
    x, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 2001):
        x, m, v = oracle.adam_step(x, 2 * (x - 3.0), m, v, t, 0.05)
    assert abs(x[0] - 3.0) < 1e-3


def test_features_on_a_single_mode():
    N, nu, dt = 16, 0.01, 0.02
    z = np.zeros((3, N, N, N // 2 + 1), complex)
    u, d1, d2 = z.copy(), z.copy(), z.copy()
    # mode k = (1, -2, 3): index (1, N-2, 3)
    u[:, 1, N - 2, 3] = [3 + 4j, 0, 0]          # |u_k| = 5
    d1[:, 1, N - 2, 3] = [0, 0.6j, 0.8]          # s = 1
    d2[:, 1, N - 2, 3] = [0.1, 0, 0]
    F, s = oracle.surrogate_features(u, d1, d2, nu, dt)
    M = oracle.retained_mask(N)
    rows = np.nonzero(M)
    r = [i for i in range(len(s)) if (rows[0][i], rows[1][i], rows[2][i]) == (1, N - 2, 3)][0]
    a = 0.5 * dt * nu * 14
    assert s[r] == pytest.approx(1.0)
    np.testing.assert_allclose(F[r, 0:6], [0, 0, 0, 0.6, 0.8, 0])
    np.testing.assert_allclose(F[r, 6:12], [0.1, 0, 0, 0, 0, 0])
    np.testing.assert_allclose(F[r, 12:18], [2 * a * 3, 2 * a * 4, 0, (1 - a) * 0.6, (1 - a) * 0.8, 0])
    np.testing.assert_allclose(F[r, 18:25], [0.6, 0.8, 0, 0, 0, 0, 0.2])
    np.testing.assert_allclose(F[r, 25:32], [1 / 16, -2 / 16, 3 / 16, a, 0, 0, 0])
    # every other row has s = 0 and is all zero
    assert np.all(s[np.arange(len(s)) != r] == 0) and np.all(F[np.arange(len(s)) != r] == 0)


def test_dtF_feature_is_the_nonlinear_forcing_at_the_fixed_point():
    # after a converged step, (1 - a) D1 + 2 a u^n = dt F_NL(midpoint of that step)
    N, nu, dt = 16, 0.05, 0.02
    u0 = inputs.smooth_random(N, 4) * 3
    u1, _, ok, fnl = oracle.implicit_midpoint_step(u0, nu, dt, 1e-13)
    assert ok
    F, s = oracle.surrogate_features(u1, u1 - u0, np.zeros_like(u0), nu, dt)
    idx = np.nonzero(oracle.retained_mask(N))
    v = (dt * fnl)[:, idx[0], idx[1], idx[2]].T
    want = np.stack([v.real, v.imag], axis=-1).reshape(-1, 6)
    live = s > 0
    np.testing.assert_allclose(F[live, 12:18] * s[live, None], want[live], rtol=0, atol=1e-10 * np.abs(want).max())


def test_zero_network_predicts_the_extrapolation():
    N = 16
    rng = np.random.default_rng(5)
    u, d1, d2 = (inputs.rough_random(N, int(sd)) for sd in rng.integers(0, 100, 3))
    theta = np.zeros(oracle.mlp_param_count())
    p = oracle.surrogate_predict(theta, u, d1, d2, 0.01, 0.01)
    M = oracle.retained_mask(N)
    np.testing.assert_allclose(p, (2 * d1 - d2) * M, rtol=0, atol=1e-12 * np.abs(d1).max())
