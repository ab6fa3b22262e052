"""Dense fields on the long transform plans, FP32.

R2 fills every retained mode, so every tile, every twiddle and every stage
of the 256-, 512- and 1024-point plans carries data:
  * 256^3: one RK4 step of Eq. NSfinal against the FP64 oracle run here on
    the FP32-rounded input (about 30 s of host time).
  * 512^3: one RK4 step against the oracle's output at 8200 seeded modes
    and its whole-output norm (tests/golden/oracle_rk4_r2_512_f32in.npz,
    written by tests/golden/make_dense512_fixture.py, which calls only the
    oracle and the input generator).
  * 1024^3, where no oracle fits: the energy identity of the Galerkin
    nonlinear term, sum_half w Re(conj(u_k) . N_k) = 0 (u . (u x w) = 0 at
    every point), on a dense field with nu = 0, where the right-hand side is
    the projected N_k.  A wrong twiddle, index or sign in any pass breaks it.
Bar: the FP32 bound 10 u32 log2(N^3) of the other parity tests.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import fp32_tol, note, rel_l2, round32, run

pytestmark = pytest.mark.gpu

NU, DT = 1.0 / 1600.0, 1e-3
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_dense_rk4_256_fp32_matches_oracle():
    N = 256
    print(f"dense R2 rk4 N={N} f32", flush=True)
    uh = inputs.rough_random(N, N)
    (got,) = run("rk4", [uh], "f32", nu=NU, dt=DT, nsteps=1)
    ref = oracle.rk4(round32(uh), NU, DT, 1)
    assert rel_l2(got, ref) < fp32_tol(N)
    assert np.all(got[:, ~oracle.retained_mask(N)] == 0)


def test_dense_rk4_512_fp32_matches_sampled_oracle():
    import torch
    N = 512
    fx = np.load(os.path.join(GOLDEN, "oracle_rk4_r2_512_f32in.npz"))
    print(f"dense R2 rk4 N={N} f32 (sampled oracle)", flush=True)
    uh = inputs.rough_random(N, int(fx["seed"]))
    h, wsb = binding.hot_plan(N, "rk4", "f32", "two_thirds", float(fx["nu"]), float(fx["dt"]))
    try:
        x = torch.from_numpy(uh.astype(np.complex64)).cuda()
        del uh
        y = torch.empty_like(x)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        binding.hot_run(h, [x], [y], ws, 1)
        torch.cuda.synchronize()
        del ws, x
    finally:
        binding.hot_destroy(h)
    idx = [torch.from_numpy(fx[k].astype(np.int64)).cuda() for k in ("ix", "iy", "iz")]
    got = y[:, idx[0], idx[1], idx[2]].cpu().numpy()
    ref = fx["values"]
    assert rel_l2(got, ref) < fp32_tol(N)
    norm = float(torch.linalg.vector_norm(y.reshape(-1).to(torch.complex128)))
    assert note(abs(norm - float(fx["norm"])) / float(fx["norm"])) < fp32_tol(N)


def _dense_field_on_gpu(N, seed):
    """A dense random solenoidal field on the retained 2/3 modes of the N^3
    half spectrum, built on the GPU (a 1024^3 field is too slow to draw on
    the host): normal coefficients, projected perpendicular to k, the kz = 0
    plane made Hermitian, zero outside the retained set, E = 1/8."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    shape = (3, N, N, N // 2 + 1)
    x = torch.complex(torch.randn(shape, generator=g, device="cuda"), torch.randn(shape, generator=g, device="cuda"))
    j = torch.arange(N, device="cuda")
    k = torch.where(j <= N // 2, j, j - N).float()
    kz = torch.arange(N // 2 + 1, device="cuda").float()
    K = (N - 1) // 3
    keep = ((k.abs() <= K)[:, None, None] & (k.abs() <= K)[None, :, None] & (kz <= K)[None, None, :])
    kx, ky, kzz = k[:, None, None], k[None, :, None], kz[None, None, :]
    for c in range(3):
        x[c] *= keep
    k2 = (kx * kx + ky * ky + kzz * kzz).clamp(min=1.0)
    kd = (kx * x[0] + ky * x[1] + kzz * x[2]) / k2
    x[0] -= kx * kd
    x[1] -= ky * kd
    x[2] -= kzz * kd
    del kd
    x[:, 0, 0, 0] = 0
    # kz = 0 plane: u(-kx, -ky) = conj u(kx, ky)
    neg = (-j) % N
    p = x[:, :, :, 0]
    x[:, :, :, 0] = 0.5 * (p + p[:, neg][:, :, neg].conj())
    e = float((x.abs() ** 2).sum(dim=(0, 1, 2)).double()[1:].sum() * 2 + (x[:, :, :, 0].abs() ** 2).sum().double())
    return x * float(np.sqrt(0.125 * float(N) ** 6 * 2.0 / e))


@pytest.mark.parametrize("tune", [False, True])
def test_dense_rhs_1024_fp32_energy_identity(tune):
    import torch
    N = 1024
    print(f"dense rhs N={N} f32 energy identity tune={tune}", flush=True)
    x = _dense_field_on_gpu(N, 17)
    h, wsb = binding.hot_plan(N, "rhs", "f32", "two_thirds", 0.0, 1e-3)
    try:
        y = torch.empty_like(x)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        if tune:
            binding.hot_tune(h, ws)
        binding.hot_run(h, [x], [y], ws, 0)
        torch.cuda.synchronize()
        del ws
    finally:
        binding.hot_destroy(h)
    w = torch.full((N // 2 + 1,), 2.0, dtype=torch.float64, device="cuda")
    w[0] = 1.0
    # sum over the half spectrum with the real-field weights, per kz plane
    dot = torch.zeros(N // 2 + 1, dtype=torch.float64, device="cuda")
    mag = torch.zeros(N // 2 + 1, dtype=torch.float64, device="cuda")
    for c in range(3):
        prod = x[c].conj() * y[c]
        dot += prod.real.double().sum(dim=(0, 1))
        mag += prod.abs().double().sum(dim=(0, 1))
        del prod
    resid = float((w * dot).sum().abs() / (w * mag).sum())
    print(f"energy identity residual {resid:.3e}", flush=True)
    assert note(resid) < fp32_tol(N)
    # the right-hand side is not trivially zero, and is zero outside the retained set
    assert float((w * mag).sum()) > 0
    K = (N - 1) // 3
    assert float(y[:, :, :, K + 1:].abs().max()) == 0.0
    assert float(y[:, K + 1:N - K].abs().max()) == 0.0
