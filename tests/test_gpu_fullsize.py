"""GPU parity at the benchmark size: N = 1024, FP32, one instance per call,
in the launch configuration bench.py times.

The oracle cannot run at 1024^3, so these tests use inputs whose exact
right-hand side the oracle computes at a small N:
  * Taylor-Green (Sec. 4): its right-hand side only has modes |k_i| <= 2, so
    the oracle at N = 16 is exact (alias-free, nothing truncated) and the
    1024^3 coefficients are the N = 16 ones times (1024/16)^3 (Eq. ffteq
    scaling); every other mode must vanish.
  * R1 band-limited to |k_i| <= 16: the product u x w only reaches
    |k_i| <= 32, which the 2/3 rule keeps and does not alias at N = 128, so
    the oracle at N = 128 gives every nonzero coefficient of the 1024^3
    right-hand side.
  * a few modes on the faces and corners of the retained box and spread over
    it (inputs.wide_sparse_modes): the triad-sum oracle gives the exact
    right-hand side at 1024^3, and the ragged last tiles and the 2/3 cut of
    every pass see nonzero data (FP32, untuned and tuned, and FP64).
  * a Beltrami field decays exactly as R(z)^n under RK4, on a mid shell and
    on the shell |k| = 341 that touches the faces of the retained box.
The comparison runs on the GPU (torch) to avoid copying 13 GB to the host.
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import fp32_tol, note

pytestmark = pytest.mark.gpu

N = 1024
NU = 1.0 / 1600.0


def _torch():
    import torch
    return torch


def _sparse_to_gpu(modes_idx, vals, scale=1.0):
    torch = _torch()
    x = torch.zeros((3, N, N, N // 2 + 1), dtype=torch.complex64, device="cuda")
    ix, iy, iz = [torch.from_numpy(np.asarray(a)).long().cuda() for a in modes_idx]
    x[:, ix, iy, iz] = torch.from_numpy(np.asarray(vals) * scale).to(torch.complex64).cuda()
    return x


def _small_to_big_index(n):
    """Signed wavenumbers of an n-grid half-spectrum mapped to 1024-grid indices."""
    j = np.arange(n)
    k = np.where(j <= n // 2, j, j - n)
    return k % N, k


def _run(op, x, nsteps=0, nu=NU, dt=1e-3, tune=False):
    """tune: autotune the plan first, as bench.py does before it times."""
    torch = _torch()
    h, wsb = binding.hot_plan(N, op, "f32", "two_thirds", nu, dt)
    try:
        y = torch.empty_like(x)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        if tune:
            binding.hot_tune(h, ws)
            print("tuned:", {k: binding.hot_tuned_width(h, 0, k) for k in ("x_inv_curl", "y_inv", "y_fwd", "x_fwd",
                                                                          "x_fwd_rk")}, flush=True)
        binding.hot_run(h, [x], [y], ws, nsteps)
        torch.cuda.synchronize()
        del ws
        return y
    finally:
        binding.hot_destroy(h)


def _compare_with_small_oracle(y, ref_small, n):
    """y: 1024^3 GPU result; ref_small: oracle half-spectrum at size n whose
    nonzero modes all fit the 1024 grid.  Returns relative L2 error over all
    modes (zero modes included)."""
    torch = _torch()
    big_idx, k = _small_to_big_index(n)
    kz = np.arange(n // 2 + 1)
    keep = np.abs(k) < n // 2
    ref = ref_small[:, keep][:, :, keep][:, :, :, kz < n // 2] * (N / n) ** 3
    bi = big_idx[keep]
    IX, IY, IZ = np.meshgrid(bi, bi, kz[kz < n // 2], indexing="ij")
    idx = [torch.from_numpy(a.ravel()).long().cuda() for a in (IX, IY, IZ)]
    expect = torch.zeros_like(y)
    expect[:, idx[0], idx[1], idx[2]] = torch.from_numpy(ref.reshape(3, -1)).to(torch.complex64).cuda()
    err = torch.linalg.vector_norm((y - expect).reshape(-1).to(torch.complex128))
    den = torch.linalg.vector_norm(expect.reshape(-1).to(torch.complex128))
    return note(float(err / den))


def test_taylor_green_rhs_1024_fp32():
    print("fullsize: TG rhs", flush=True)
    n = 16
    tg = inputs.taylor_green(n)
    nz = np.nonzero(np.abs(tg).sum(axis=0))
    big_idx, _ = _small_to_big_index(n)
    x = _sparse_to_gpu((big_idx[nz[0]], big_idx[nz[1]], nz[2]), tg[:, nz[0], nz[1], nz[2]], (N / n) ** 3)
    y = _run("rhs", x)
    ref = oracle.rhs(tg, NU)
    assert _compare_with_small_oracle(y, ref, n) < fp32_tol(N)


@pytest.mark.parametrize("tune", [False, True])
def test_band_limited_rhs_1024_fp32_matches_oracle_at_128(tune):
    print(f"fullsize: R1 rhs tune={tune}", flush=True)
    ix, iy, iz, vals = inputs.smooth_random_modes(N, seed=0)
    x = _sparse_to_gpu((ix, iy, iz), vals)
    y = _run("rhs", x, tune=tune)
    # the same field on a 128 grid: same wavenumbers, coefficients scaled by (128/1024)^3
    small = inputs.smooth_random(128, seed=0)
    # smooth_random normalises E = 1/8 on each grid, so the two fields are the same
    ref = oracle.rhs(small.astype(np.complex64).astype(np.complex128), NU)
    assert _compare_with_small_oracle(y, ref, 128) < fp32_tol(N)


@pytest.mark.parametrize("tune", [False, True])
def test_wide_sparse_rhs_1024_fp32_matches_triad_oracle(tune):
    print(f"fullsize: wide sparse rhs tune={tune}", flush=True)
    ix, iy, iz, vals = inputs.wide_sparse_modes(N, 128, seed=5)
    v32 = vals.astype(np.complex64)
    x = _sparse_to_gpu((ix, iy, iz), v32)
    y = _run("rhs", x, tune=tune)
    del x
    s = inputs.signed_index(N)
    kout, ref = oracle.rhs_triads(np.stack([s[ix], s[iy], iz], -1), v32.astype(np.complex128), N, NU)
    assert np.abs(kout).max() == (N - 1) // 3 and len(kout) > 5000
    expect = _sparse_to_gpu((kout[:, 0] % N, kout[:, 1] % N, kout[:, 2]), ref)
    torch = _torch()
    err = torch.linalg.vector_norm((y - expect).reshape(-1).to(torch.complex128))
    den = torch.linalg.vector_norm(expect.reshape(-1).to(torch.complex128))
    print(f"rel L2 {float(err / den):.3e} over {len(kout)} modes", flush=True)
    assert note(float(err / den)) < fp32_tol(N)


@pytest.mark.parametrize("K2", [10000, 341**2])
@pytest.mark.parametrize("tune", [False, True])
def test_beltrami_rk4_1024_fp32_exact_decay(tune, K2):
    # Explicit RK4 is stable for the viscous term only while dt nu |k|^2 stays
    # inside its real stability interval (|z| < 2.78); at N = 1024 the largest
    # retained |k|^2 is 3 * 341^2, so nu dt = 5e-6 gives |z| <= 1.75 there.  The
    # shells |k|^2 = 10^4 and 341^2 make the decay per step clearly visible;
    # the second reaches k_i = +-341 on every axis, the last retained index.
    print(f"fullsize: Beltrami rk4 K2={K2} tune={tune}", flush=True)
    nu, dt, n = 1e-3, 5e-3, 2
    assert nu * dt * 3 * 341**2 < 2.78
    ix, iy, iz, vals = inputs.beltrami_modes(N, K2, seed=4)
    x = _sparse_to_gpu((ix, iy, iz), vals)
    y = _run("rk4", x, nsteps=n, nu=nu, dt=dt, tune=tune)
    z = -nu * K2 * dt
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    torch = _torch()
    err = torch.linalg.vector_norm((y - x * R**n).reshape(-1).to(torch.complex128))
    den = torch.linalg.vector_norm((x * R**n).reshape(-1).to(torch.complex128))
    assert note(float(err / den)) < fp32_tol(N)


def test_band_limited_rhs_1024_fp64_matches_oracle_at_128():
    # the largest size in FP64 (workspace ~90 GB): FP64 bar of the parity tests
    print("fullsize: R1 rhs fp64", flush=True)
    torch = _torch()
    ix, iy, iz, vals = inputs.smooth_random_modes(N, seed=0)
    x = torch.zeros((3, N, N, N // 2 + 1), dtype=torch.complex128, device="cuda")
    idx = [torch.from_numpy(np.asarray(a)).long().cuda() for a in (ix, iy, iz)]
    x[:, idx[0], idx[1], idx[2]] = torch.from_numpy(np.asarray(vals)).cuda()
    h, wsb = binding.hot_plan(N, "rhs", "f64", "two_thirds", NU, 1e-3)
    try:
        y = torch.empty_like(x)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        binding.hot_run(h, [x], [y], ws, 0)
        torch.cuda.synchronize()
        del ws
    finally:
        binding.hot_destroy(h)
    ref = oracle.rhs(inputs.smooth_random(128, seed=0), NU)
    big_idx, k = _small_to_big_index(128)
    kz = np.arange(65)
    keep = np.abs(k) < 64
    r = ref[:, keep][:, :, keep][:, :, :, kz < 64] * (N / 128) ** 3
    bi = big_idx[keep]
    IX, IY, IZ = np.meshgrid(bi, bi, kz[kz < 64], indexing="ij")
    sel = [torch.from_numpy(a.ravel()).long().cuda() for a in (IX, IY, IZ)]
    got = y[:, sel[0], sel[1], sel[2]].cpu().numpy().reshape(r.shape)
    assert note(np.linalg.norm(got - r) / np.linalg.norm(r)) <= 1e-12
    # every other coefficient is zero: the norms agree
    assert float(torch.linalg.vector_norm(y)) == pytest.approx(float(np.linalg.norm(r)), rel=1e-12)


def test_wide_sparse_rhs_1024_fp64_matches_triad_oracle():
    # the FP64 kernels' tiles at the faces of the retained box, at the FP64 bar
    print("fullsize: wide sparse rhs fp64", flush=True)
    torch = _torch()
    ix, iy, iz, vals = inputs.wide_sparse_modes(N, 128, seed=6)
    x = torch.zeros((3, N, N, N // 2 + 1), dtype=torch.complex128, device="cuda")
    idx = [torch.from_numpy(np.asarray(a)).long().cuda() for a in (ix, iy, iz)]
    x[:, idx[0], idx[1], idx[2]] = torch.from_numpy(np.asarray(vals)).cuda()
    h, wsb = binding.hot_plan(N, "rhs", "f64", "two_thirds", NU, 1e-3)
    try:
        y = torch.empty_like(x)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        binding.hot_run(h, [x], [y], ws, 0)
        torch.cuda.synchronize()
        del ws, x
    finally:
        binding.hot_destroy(h)
    s = inputs.signed_index(N)
    kout, ref = oracle.rhs_triads(np.stack([s[ix], s[iy], iz], -1), vals, N, NU)
    sel = [torch.from_numpy(a).long().cuda() for a in (kout[:, 0] % N, kout[:, 1] % N, kout[:, 2])]
    got = y[:, sel[0], sel[1], sel[2]].cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"rel L2 {err:.3e} over {len(kout)} modes", flush=True)
    assert note(err) <= 1e-12
    # every other coefficient is zero to rounding: the norms agree
    assert float(torch.linalg.vector_norm(y)) == pytest.approx(float(np.linalg.norm(ref)), rel=1e-12)


def test_implicit_beltrami_1024_fp32_crank_nicolson_factor():
    # the implicit step at full size: a Beltrami field decays by (1 - a)/(1 + a) per step
    print("fullsize: Beltrami implicit", flush=True)
    torch = _torch()
    K2, nu, dt, n = 10000, 1e-3, 5e-3, 2
    ix, iy, iz, vals = inputs.beltrami_modes(N, K2, seed=4)
    x = _sparse_to_gpu((ix, iy, iz), vals)
    h, wsb = binding.hot_plan(N, "implicit", "f32", "two_thirds", nu, dt, 1e-5, 10)
    try:
        y = torch.empty_like(x)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        assert binding.hot_run(h, [x], [y], ws, n) == binding.HOT_OK
        torch.cuda.synchronize()
        sweeps, _ = binding.hot_implicit_stats(h, 1)
        del ws
    finally:
        binding.hot_destroy(h)
    a = 0.5 * dt * nu * K2
    R = ((1 - a) / (1 + a)) ** n
    err = torch.linalg.vector_norm((y - x * R).reshape(-1).to(torch.complex128))
    den = torch.linalg.vector_norm((x * R).reshape(-1).to(torch.complex128))
    assert note(float(err / den)) < fp32_tol(N)
    assert sweeps == [2 * n]
