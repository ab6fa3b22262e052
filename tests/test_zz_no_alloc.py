"""hot_run_noalloc: the RK4 and right-hand-side ops on the library's static
scratch, for callers that cannot allocate, against hot_run with a caller
workspace (the same kernels, so bit for bit) and against the oracle, on two
calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import fp32_tol, rel_l2, round32, to_dev, workspace

pytestmark = pytest.mark.gpu

NU, DT = 1.0 / 1600.0, 1e-3


def _both(sizes, op, dtype, nsteps, fields):
    """Outputs of hot_run (workspace) and hot_run_noalloc (static scratch)."""
    import torch
    h, wsb = binding.hot_plan(sizes, op, dtype, nu=NU, dt=DT)
    try:
        assert wsb <= 16 << 20
        ins = [to_dev(f, dtype) for f in fields]
        ref = [torch.empty_like(x) for x in ins]
        got = [torch.full_like(x, float("nan")) for x in ins]
        binding.hot_run(h, ins, ref, workspace(wsb), nsteps)
        torch.cuda.synchronize()
        assert binding.hot_run_noalloc(h, ins, got, nsteps) == binding.HOT_OK
        torch.cuda.synchronize()
        return [r.cpu().numpy() for r in ref], [g.cpu().numpy() for g in got]
    finally:
        binding.hot_destroy(h)


def test_noalloc_matches_the_workspace_path_on_two_calls():
    # first call: an uneven FP32 batch, one RK4 step
    sizes = [32, 24, 32, 64]
    fields = [inputs.rough_random(N, 40 + i) for i, N in enumerate(sizes)]
    print(f"noalloc rk4 f32 {sizes}", flush=True)
    ref, got = _both(sizes, "rk4", "f32", 1, fields)
    for f, r, g in zip(fields, ref, got):
        assert np.array_equal(r.view(np.uint8), g.view(np.uint8))
        assert rel_l2(g, oracle.rk4(round32(f), NU, DT, 1)) < fp32_tol(f.shape[1])
    # second call, smaller: one FP64 instance of N = 16, right-hand side
    f = inputs.rough_random(16, 77)
    print("noalloc rhs f64 [16]", flush=True)
    ref, got = _both([16], "rhs", "f64", 0, [f])
    assert np.array_equal(ref[0].view(np.uint8), got[0].view(np.uint8))
    assert rel_l2(got[0], oracle.rhs(f, NU)) < 1e-12
    # and a third, larger again: whatever the second call left in the scratch
    # does not leak into the result
    f = inputs.smooth_random(48, 5)
    ref, got = _both([48], "rk4", "f64", 2, [f])
    assert np.array_equal(ref[0].view(np.uint8), got[0].view(np.uint8))
    assert rel_l2(got[0], oracle.rk4(f, NU, DT, 2)) < 1e-12


def test_noalloc_rejects_plans_beyond_the_scratch():
    lib = binding.library()
    h, wsb = binding.hot_plan(128, "rk4", "f64", nu=NU, dt=DT)
    try:
        assert wsb > 16 << 20
        arr = (ctypes.c_void_p * 1)(256 * 1000)
        assert lib.hot_run_noalloc(h, arr, arr, 1, None, None) == binding.HOT_E_TOOBIG
    finally:
        binding.hot_destroy(h)
