"""The per-call statistics (hot_stats through stats_dev), graph replays of the
implicit step, and RK4 calls resumed from their own output.

  * stats_dev: E and eps of every instance's state against the oracle's
    energy() and dissipation_rate() of the same state (FP64, 1e-12), and the
    implicit step's sweep and max_iter counters against hot_implicit_stats.
  * An implicit step captured into a graph and replayed (with eager work
    between replays) equals the eager call bit for bit, statistics included:
    the host never waits for the stopping test, so the whole call records.
  * RK4: n steps, then n more steps from that output, equal 2n steps in one
    call bit for bit (the step is a function of the state alone).
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import to_dev, workspace

pytestmark = pytest.mark.gpu

NU = 1.0 / 1600.0
SIZES = [16, 24, 16, 32, 18]


def _fields():
    return [inputs.rough_random(N, 500 + i) * (1.0 + 0.25 * i) for i, N in enumerate(SIZES)]


@pytest.mark.parametrize("op", ["rhs", "rk4", "implicit"])
def test_stats_match_the_oracle(op):
    import torch
    print(f"stats {op}", flush=True)
    fields = _fields()
    kw = dict(tol=1e-10, max_iter=30) if op == "implicit" else {}
    h, wsb = binding.hot_plan(SIZES, op, "f64", nu=NU, dt=0.01, **kw)
    try:
        ins = [to_dev(f, "f64") for f in fields]
        outs = [torch.empty_like(x) for x in ins]
        st = binding.stats_buffer(len(fields))
        binding.hot_run(h, ins, outs, workspace(wsb), 2, stats=st)
        torch.cuda.synchronize()
        E, eps, sw, nc = binding.stats_view(st)
        if op == "implicit":
            sw_h, nc_h = binding.hot_implicit_stats(h, len(fields))
            assert list(sw) == sw_h and list(nc) == nc_h and min(sw) > 0
        else:
            assert not sw.any() and not nc.any()
        for i, f in enumerate(fields):
            # the state: the right-hand side's input, the time steppers' result
            state = f * oracle.retained_mask(f.shape[1]) if op == "rhs" else outs[i].cpu().numpy()
            assert abs(E[i] - oracle.energy(state)) <= 1e-12 * oracle.energy(state)
            d = oracle.dissipation_rate(state, NU)
            assert abs(eps[i] - d) <= 1e-12 * d
    finally:
        binding.hot_destroy(h)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_implicit_graph_replay_equals_eager(dtype):
    import torch
    print(f"implicit graph {dtype}", flush=True)
    fields = _fields()
    tol = 1e-10 if dtype == "f64" else 1e-5
    h, wsb = binding.hot_plan(SIZES, "implicit", dtype, nu=NU, dt=0.02, tol=tol, max_iter=12)
    try:
        ws = workspace(wsb)
        s = torch.cuda.Stream()
        ins = [to_dev(f, dtype) for f in fields]
        outs = [torch.empty_like(x) for x in ins]
        st = binding.stats_buffer(len(fields))
        torch.cuda.synchronize()
        binding.hot_run(h, ins, outs, ws, 3, s, stats=st)
        torch.cuda.synchronize()
        eager = [o.cpu().numpy() for o in outs]
        eager_stats = st.cpu().numpy().copy()
        sw_eager = binding.hot_implicit_stats(h, len(fields))
        g = binding.hot_graph_create(h, ins, outs, ws, 3, s, stats=st)
        try:
            for _ in range(3):
                for o in outs:
                    o.zero_()
                st.zero_()
                binding.hot_run(h, ins, [torch.empty_like(x) for x in ins], ws, 1, s)  # eager work between
                torch.cuda.synchronize()
                binding.hot_graph_launch(g, s)
                torch.cuda.synchronize()
                for a, o in zip(eager, outs):
                    assert np.array_equal(a.view(np.uint8), o.cpu().numpy().view(np.uint8))
                assert np.array_equal(eager_stats, st.cpu().numpy())
        finally:
            binding.hot_graph_destroy(g)
        assert sum(sw_eager[0]) > 0
    finally:
        binding.hot_destroy(h)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rk4_resumed_equals_one_longer_call(dtype):
    import torch
    print(f"rk4 resume {dtype}", flush=True)
    fields = _fields()
    h, wsb = binding.hot_plan(SIZES, "rk4", dtype, nu=NU, dt=1e-3)
    try:
        ws = workspace(wsb)
        ins = [to_dev(f, dtype) for f in fields]
        mid = [torch.empty_like(x) for x in ins]
        two = [torch.empty_like(x) for x in ins]
        one = [torch.empty_like(x) for x in ins]
        binding.hot_run(h, ins, mid, ws, 3)
        binding.hot_run(h, mid, two, ws, 3)
        binding.hot_run(h, ins, one, ws, 6)
        torch.cuda.synchronize()
        for a, b in zip(two, one):
            assert np.array_equal(a.cpu().numpy().view(np.uint8), b.cpu().numpy().view(np.uint8))
    finally:
        binding.hot_destroy(h)
