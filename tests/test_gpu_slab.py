"""z-slab shares of one field (hot_plan_slab / hot_slab_run), every share on
this one GPU with the all-to-all done by device copies (slab.exchange_local).

* Against the oracle: RK4 steps and right-hand sides, FP64 and FP32, with
  the tolerances of the single-field parity tests.
* Against the single-field path: bitwise equal.  Every column and z line is
  transformed by the same kernels with the same arithmetic; only the
  addresses differ.  At 512^3 FP32 over two shares (chunks of 86 retained
  kz at a 128-byte padded pitch of 96) and over eight (chunks of 22, the
  last share holding 17) this covers the blocked z-line loads and stores at
  a realistic size.
* Edge cases: one share (the phases alone), a last share with a single
  retained kz, dealias "none", a 3-smooth N.
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs, slab
from hotrun import CDT, fp32_tol, rel_l2, round32, run

pytestmark = pytest.mark.gpu

NU = 1.0 / 1600.0
DT = 1e-3


def _torch():
    import torch
    return torch


def run_shares(u, R, op, dtype, nsteps=1, dealias="two_thirds", nu=NU, dt=DT, on_device=False):
    """All R shares of the canonical field u ([3][N][N][N/2+1], numpy or a
    device tensor); returns the assembled canonical result (same kind)."""
    torch = _torch()
    N = u.shape[1]
    plans, lays, wss, ins, outs = [], [], [], [], []
    try:
        for r in range(R):
            h, wsb = binding.hot_plan_slab(N, op, R, r, dtype, dealias, nu, dt)
            plans.append(h)
            lay = binding.hot_slab_layout_of(h)
            lays.append(lay)
            wss.append(torch.zeros(wsb, dtype=torch.uint8, device="cuda"))
            part = u[..., lay.kz0:lay.kz0 + lay.nkz]
            if on_device:
                ins.append(part.contiguous())
            else:
                ins.append(torch.from_numpy(np.ascontiguousarray(part.astype(CDT[dtype]))).cuda())
            outs.append(torch.empty_like(ins[-1]))
        for r in range(R):
            binding.hot_slab_run(plans[r], binding.HOT_SLAB_GATHER, wss[r], inp=ins[r])
        stages = [4] if op == "rhs" else [s for _ in range(nsteps) for s in range(4)]
        for st in stages:
            for r in range(R):
                binding.hot_slab_run(plans[r], binding.HOT_SLAB_INVERSE, wss[r], stage=st)
            slab.exchange_local(wss, lays, forward=True)
            for r in range(R):
                binding.hot_slab_run(plans[r], binding.HOT_SLAB_CROSS, wss[r], stage=st)
            slab.exchange_local(wss, lays, forward=False)
            for r in range(R):
                binding.hot_slab_run(plans[r], binding.HOT_SLAB_FORWARD, wss[r], stage=st)
        for r in range(R):
            binding.hot_slab_run(plans[r], binding.HOT_SLAB_SCATTER, wss[r], out=outs[r])
        res = torch.cat(outs, dim=3)
        torch.cuda.synchronize()
        return res if on_device else res.cpu().numpy()
    finally:
        for h in plans:
            binding.hot_destroy(h)


CASES = [  # N, R, dtype, op, steps
    (32, 2, "f64", "rk4", 1),
    (48, 3, "f64", "rk4", 2),
    (64, 4, "f64", "rhs", 0),
    (64, 8, "f32", "rk4", 1),  # last share: one retained kz
    (54, 2, "f32", "rhs", 0),  # 3-smooth N
    (24, 1, "f64", "rk4", 1),  # one share: the phases alone
]


@pytest.mark.parametrize("N,R,dtype,op,steps", CASES)
def test_shares_match_oracle_and_single_field(N, R, dtype, op, steps):
    print(f"slab N={N} R={R} {dtype} {op} steps={steps}", flush=True)
    u = inputs.rough_random(N, 40 + N)
    got = run_shares(u, R, op, dtype, steps)
    x = round32(u) if dtype == "f32" else u
    ref = oracle.rhs(x, NU) if op == "rhs" else oracle.rk4(x, NU, DT, steps)
    assert rel_l2(got, ref) < (1e-12 if dtype == "f64" else fp32_tol(N))
    assert np.all(got[:, ~oracle.retained_mask(N)] == 0)
    (single,) = run(op, [u], dtype, nu=NU, dt=DT, nsteps=steps)
    assert np.array_equal(got, single)


def test_shares_dealias_none():
    N, R = 32, 4
    u = inputs.rough_random(N, 3, dealias="none")
    got = run_shares(u, R, "rhs", "f64", dealias="none", nu=0.01)
    assert rel_l2(got, oracle.rhs(u, 0.01, dealias="none")) < 1e-12
    (single,) = run("rhs", [u], "f64", dealias="none", nu=0.01)
    assert np.array_equal(got, single)


@pytest.mark.parametrize("R", [2, 8])
def test_shares_512_fp32_equal_the_single_field(R):
    torch = _torch()
    N = 512
    print(f"slab N={N} R={R} f32 rk4", flush=True)
    u = torch.from_numpy(inputs.smooth_random(N, 11).astype(np.complex64)).cuda()
    got = run_shares(u, R, "rk4", "f32", 1, on_device=True)
    h, wsb = binding.hot_plan(N, "rk4", "f32", "two_thirds", NU, DT)
    try:
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        single = torch.empty_like(u)
        binding.hot_run(h, [u], [single], ws, 1)
        torch.cuda.synchronize()
    finally:
        binding.hot_destroy(h)
    del ws
    assert torch.equal(got, single)
    assert float(torch.linalg.vector_norm(single)) > 0
