"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute-force
sums of the definitions, closed forms derived by hand, exact solutions of the
discrete scheme, library routines, and identities of the equations.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NU_TG = 1.0 / 1600.0


def _mesh(N):
    x = 2 * np.pi * np.arange(N) / N
    return np.meshgrid(x, x, x, indexing="ij")


def _signed(N):
    j = np.arange(N)
    return np.where(j <= N // 2, j, j - N)


def _dft_full_bruteforce(u):
    """sum_x u(x) exp(-i k.x) for every integer k of Eq. wavemesh, written as
    three explicit DFT-matrix contractions (no FFT)."""
    N = u.shape[-1]
    k = _signed(N)
    x = 2 * np.pi * np.arange(N) / N
    E = np.exp(-1j * np.outer(k, x))  # E[k, x]
    return np.einsum("ai,bj,ck,...ijk->...abc", E, E, E, u, optimize=True)


# -- P1: transforms (Eq. ffteq) ------------------------------------------------

@pytest.mark.parametrize("N", [4, 6, 8])
def test_forward_matches_bruteforce_dft(N):
    rng = np.random.default_rng(N)
    u = rng.standard_normal((3, N, N, N))
    full = _dft_full_bruteforce(u)
    half = oracle.forward(u)
    np.testing.assert_allclose(half, full[..., : N // 2 + 1], rtol=0, atol=1e-12 * np.abs(full).max())


@pytest.mark.parametrize("N", [4, 6, 8])
def test_inverse_matches_bruteforce_sum(N):
    rng = np.random.default_rng(100 + N)
    u = rng.standard_normal((2, N, N, N))
    full = _dft_full_bruteforce(u)
    # inverse of Eq. ffteq written as a direct sum over the full spectrum
    k = _signed(N)
    x = 2 * np.pi * np.arange(N) / N
    E = np.exp(1j * np.outer(x, k))
    direct = np.einsum("ia,jb,kc,...abc->...ijk", E, E, E, full, optimize=True).real / N**3
    np.testing.assert_allclose(direct, u, atol=1e-12)
    back = oracle.inverse(full[..., : N // 2 + 1], N)
    np.testing.assert_allclose(back, direct, atol=1e-12)


@pytest.mark.parametrize("N,P", [(8, 1), (8, 2), (12, 3), (16, 4), (16, 8)])
def test_slab_transform_equals_serial(N, P):
    """The slab algorithm with P virtual ranks and its all-to-all equals the
    serial transform: forward bit for bit (the same 1D transforms in the
    same order), inverse to rounding (x and y run in the other order)."""
    rng = np.random.default_rng(7 * N + P)
    u = rng.standard_normal((3, N, N, N))
    uh = oracle.forward(u)
    assert np.array_equal(oracle.forward_slab(u, P), uh)
    back = oracle.inverse_slab(uh, N, P)
    np.testing.assert_allclose(back, oracle.inverse(uh, N), rtol=0, atol=1e-14 * np.abs(u).max())
    np.testing.assert_allclose(back, u, rtol=0, atol=1e-13)


# -- component formulae ----------------------------------------------------------

def test_cross_matches_numpy_cross():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((3, 5, 6, 7))
    b = rng.standard_normal((3, 5, 6, 7))
    ref = np.cross(a, b, axis=0)
    np.testing.assert_allclose(oracle.cross(a, b), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", [8, 16])
def test_curl_of_taylor_green_closed_form(N):
    X, Y, Z = _mesh(N)
    w = oracle.inverse(oracle.curl(inputs.taylor_green(N)), N)
    ref = np.stack([
        -np.cos(X) * np.sin(Y) * np.sin(Z),
        -np.sin(X) * np.cos(Y) * np.sin(Z),
        2 * np.sin(X) * np.sin(Y) * np.cos(Z),
    ])
    np.testing.assert_allclose(w, ref, atol=1e-14)


# -- P2: worked example, Taylor-Green right-hand side at t = 0 (Sec. 4) ----------

@pytest.mark.parametrize("N", [8, 12, 16])
def test_taylor_green_rhs_closed_form(N):
    g = json.load(open(os.path.join(GOLDEN, "taylor_green.json")))
    nu = 1.0 / g["reynolds_number"]
    X, Y, Z = _mesh(N)
    du = oracle.inverse(oracle.rhs(inputs.taylor_green(N), nu), N)
    ref = np.stack([
        -0.125 * np.sin(2 * X) * np.cos(2 * Z) - 3 * nu * np.sin(X) * np.cos(Y) * np.cos(Z),
        -0.125 * np.sin(2 * Y) * np.cos(2 * Z) + 3 * nu * np.cos(X) * np.sin(Y) * np.cos(Z),
        0.125 * (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z),
    ])
    np.testing.assert_allclose(du, ref, atol=2e-15)


def test_taylor_green_scalars():
    g = json.load(open(os.path.join(GOLDEN, "taylor_green.json")))["derived_closed_forms"]
    N = 16
    uh = inputs.taylor_green(N)
    assert abs(oracle.energy(uh) - g["energy_t0"]) < 1e-15
    assert abs(oracle.dissipation_rate(uh, 1.0) - g["mean_enstrophy_t0"]) < 1e-14
    du = oracle.rhs(uh, NU_TG)
    w = np.full(N // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    dEdt = np.sum(w * np.sum(np.real(np.conj(uh) * du), axis=(0, 1, 2))) / N**6
    assert abs(dEdt / NU_TG - g["dEdt_t0_over_nu"]) < 1e-10


def test_taylor_green_generator_matches_transform():
    N = 8
    np.testing.assert_allclose(inputs.taylor_green(N), oracle.forward(inputs.taylor_green_physical(N)),
                               atol=1e-12)


# -- P3: exact decay of a Beltrami field under discrete RK4 ----------------------

@pytest.mark.parametrize("K2,N", [(9, 16), (5, 12), (2, 8)])
def test_beltrami_exact_rk4_decay(K2, N):
    nu, dt, n = 0.05, 0.01, 10
    u0 = inputs.beltrami(N, K2, seed=3)
    # the field is an eigenvector of the curl: omega = sqrt(K2) u
    w = oracle.inverse(oracle.curl(u0), N)
    np.testing.assert_allclose(w, np.sqrt(K2) * oracle.inverse(u0, N), atol=1e-13)
    z = -nu * K2 * dt
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    got = oracle.rk4(u0, nu, dt, n)
    ref = R**n * u0
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


# -- P4: dealiased product equals the Galerkin triad sum -------------------------

def _full_from_half(h, N):
    """Complete a Hermitian half-spectrum (..., N, N, N/2+1) to (..., N, N, N)."""
    full = np.zeros(h.shape[:-1] + (N,), dtype=complex)
    full[..., : N // 2 + 1] = h
    idx = (-np.arange(N)) % N
    for kz in range(N // 2 + 1, N):
        full[..., kz] = np.conj(h[..., idx, :, :][..., :, idx, :][..., (N - kz)])
    return full


@pytest.mark.parametrize("N", [8, 12])
def test_dealiased_product_equals_galerkin_triads(N):
    a = inputs.rough_random(N, seed=11)
    b = oracle.curl(a)
    M = oracle.retained_mask(N)
    got = oracle.forward(oracle.cross(oracle.inverse(a, N), oracle.inverse(b, N))) * M
    A = _full_from_half(a, N)
    B = _full_from_half(b, N)
    s = _signed(N)
    kept = [int(v) for v in s if 3 * abs(v) < N]
    ref = np.zeros_like(got)
    for kx in kept:
        for ky in kept:
            for kz in [v for v in kept if v >= 0]:
                acc = np.zeros(3, complex)
                for px in kept:
                    qx = kx - px
                    if 3 * abs(qx) >= N:
                        continue
                    for py in kept:
                        qy = ky - py
                        if 3 * abs(qy) >= N:
                            continue
                        for pz in kept:
                            qz = kz - pz
                            if 3 * abs(qz) >= N:
                                continue
                            acc += np.cross(A[:, px % N, py % N, pz % N], B[:, qx % N, qy % N, qz % N])
                ref[:, kx % N, ky % N, kz] = acc / N**3
    scale = np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)


# -- P5: identities of the semi-discrete equations -------------------------------

@pytest.mark.parametrize("gen,N", [("smooth", 16), ("rough", 12), ("rough", 16), ("smooth", 18)])
def test_rhs_invariants(gen, N):
    nu = 0.01
    uh = inputs.smooth_random(N, seed=5) if gen == "smooth" else inputs.rough_random(N, seed=5)
    du = oracle.rhs(uh, nu)
    kx, ky, kz = oracle.wavenumbers(N)
    k2 = kx * kx + ky * ky + kz * kz
    w = np.full(N // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    # energy budget: the nonlinear part does no work (u . (u x w) = 0 pointwise)
    lhs = np.sum(w * np.sum(np.real(np.conj(uh) * du), axis=(0, 1, 2)))
    rhs = -nu * np.sum(w * np.sum(k2 * np.sum(np.abs(uh) ** 2, axis=0), axis=(0, 1)))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    # divergence-free output, zero mean mode, zero outside the retained set
    div = kx * du[0] + ky * du[1] + kz * du[2]
    assert np.abs(div).max() <= 1e-12 * np.sqrt(k2.max()) * np.abs(du).max()
    assert np.abs(du[:, 0, 0, 0]).max() <= 1e-12 * np.abs(du).max()
    M = oracle.retained_mask(N)
    assert np.all(du[:, ~M] == 0)
    # kz = 0 plane stays Hermitian: du(-k) = conj(du(k))
    idx = (-np.arange(N)) % N
    p = du[:, :, :, 0]
    np.testing.assert_allclose(p[:, idx][:, :, idx], np.conj(p), atol=1e-12 * np.abs(du).max())


# -- P6: RK4 convergence order -------------------------------------------------

def test_rk4_fourth_order():
    N, nu, T = 16, 0.02, 0.08
    u0 = inputs.smooth_random(N, seed=2)
    ref = oracle.rk4(u0, nu, T / 64, 64)
    errs = []
    for n in (4, 8, 16):
        errs.append(np.linalg.norm(oracle.rk4(u0, nu, T / n, n) - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, (r1, r2)


# -- P7: integer parts ----------------------------------------------------------

@pytest.mark.parametrize("N", list(range(8, 66, 2)))
def test_mask_is_the_strict_two_thirds_rule(N):
    M = oracle.retained_mask(N)
    s = _signed(N)
    ref = np.zeros_like(M)
    for i in range(N):
        for j in range(N):
            for k in range(N // 2 + 1):
                ref[i, j, k] = 3 * abs(s[i]) < N and 3 * abs(s[j]) < N and 3 * k < N
    assert np.array_equal(M, ref)
    K = (N - 1) // 3
    assert M.sum() == (2 * K + 1) ** 2 * (K + 1)


def test_mask_none_drops_only_nyquist():
    N = 10
    M = oracle.retained_mask(N, "none")
    assert M.sum() == (N - 1) ** 2 * (N // 2)
    assert not M[N // 2].any() and not M[:, N // 2].any() and not M[..., N // 2].any()


# -- energy and generators -------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_energy_is_parseval(seed):
    N = 12
    uh = inputs.rough_random(N, seed)
    u = oracle.inverse(uh, N)
    assert abs(oracle.energy(uh) - 0.5 * np.mean(np.sum(u * u, axis=0))) < 1e-14
    assert abs(oracle.energy(uh) - 0.125) < 1e-14


@pytest.mark.parametrize("N", [6, 8])
def test_energy_is_parseval_with_nyquist_content(N):
    # an unmasked real field has content on the kz = N/2 plane, so the
    # half-spectrum weights (1 on kz = 0 and N/2, 2 elsewhere) all matter
    rng = np.random.default_rng(N)
    u = rng.standard_normal((3, N, N, N))
    uh = oracle.forward(u)
    assert np.abs(uh[..., N // 2]).max() > 1.0
    assert abs(oracle.energy(uh) - 0.5 * np.mean(np.sum(u * u, axis=0))) < 1e-13


@pytest.mark.parametrize("N", [8, 16, 18])
def test_generated_fields_are_real_and_solenoidal(N):
    for uh in (inputs.smooth_random(N, 1), inputs.rough_random(N, 1)):
        kx, ky, kz = oracle.wavenumbers(N)
        div = kx * uh[0] + ky * uh[1] + kz * uh[2]
        assert np.abs(div).max() < 1e-10 * np.abs(uh).max()
        # a real field round-trips through the real transform pair
        np.testing.assert_allclose(oracle.forward(oracle.inverse(uh, N)), uh, atol=1e-9 * np.abs(uh).max())


def test_smooth_random_independent_of_N():
    a = inputs.smooth_random(50, seed=4)
    b = inputs.smooth_random(64, seed=4)
    # same retained modes carry the same values (band |k_i| <= 16 fits both)
    for (kx, ky, kz) in [(1, 2, 3), (-5, 7, 0), (16, -16, 16), (3, -1, 2)]:
        np.testing.assert_allclose(a[:, kx % 50, ky % 50, kz] / 50**3, b[:, kx % 64, ky % 64, kz] / 64**3,
                                   rtol=1e-12)


# -- regression lock on the oracle (fixture written by tests/golden/make_oracle_fixture.py)

def test_oracle_matches_locked_fixture():
    path = os.path.join(GOLDEN, "oracle_rk4_n8.npz")
    d = np.load(path)
    got = oracle.rk4(d["u0"], float(d["nu"]), float(d["dt"]), int(d["nsteps"]))
    np.testing.assert_allclose(got, d["u1"], rtol=0, atol=1e-13 * np.abs(d["u1"]).max())
