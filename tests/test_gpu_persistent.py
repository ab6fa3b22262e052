"""The persistent batch kernel (the "graph" schedule 2): a whole RK4 call over
a batch of uneven FP32 instances in one launch, its passes taken from a work
queue with per-size completion counters.  Checked per instance against the
oracle, against the launch-per-pass schedule with the same fused passes,
for zero steps (the masked input), through graph replays, on a batch of a
few hundred instances, and on its error path (the bound of its waits forced
down from the host)."""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import fp32_tol, rel_l2, round32, to_dev, workspace

pytestmark = pytest.mark.gpu

NU, DT = 1.0 / 1600.0, 1e-3
SIZES = [16, 18, 24, 16, 32, 36, 48, 24, 54, 64, 16, 32]
# the launch-per-pass schedule with the passes the persistent kernel runs
FUSED = {"yz_fused": 0, "x_fwd_rk": 1}


def _fields(sizes, seed0=300):
    return [inputs.rough_random(int(N), seed0 + i) for i, N in enumerate(sizes)]


def _run(fields, nsteps, variants, stream=None, graph_reps=0):
    import torch
    h, wsb = binding.hot_plan([f.shape[1] for f in fields], "rk4", "f32", "two_thirds", NU, DT)
    try:
        for name, v in variants.items():
            binding.hot_set_variant(h, name, v)
        ws = workspace(wsb)
        ins = [to_dev(f, "f32") for f in fields]
        outs = [torch.empty_like(x) for x in ins]
        binding.hot_run(h, ins, outs, ws, nsteps, stream)
        torch.cuda.synchronize()
        eager = [o.cpu().numpy() for o in outs]
        replays = []
        if graph_reps:
            g = binding.hot_graph_create(h, ins, outs, ws, nsteps, stream)
            try:
                for _ in range(graph_reps):
                    for o in outs:
                        o.zero_()  # eager work between replays
                    torch.cuda.synchronize()
                    binding.hot_graph_launch(g, stream)
                    torch.cuda.synchronize()
                    replays.append([o.cpu().numpy() for o in outs])
            finally:
                binding.hot_graph_destroy(g)
        return eager, replays
    finally:
        binding.hot_destroy(h)


@pytest.mark.parametrize("nsteps", [1, 2])
def test_persistent_rk4_matches_oracle_per_instance(nsteps):
    print(f"persistent rk4, {nsteps} steps, sizes {SIZES}", flush=True)
    fields = _fields(SIZES)
    got, _ = _run(fields, nsteps, {"graph": 2})
    for f, g in zip(fields, got):
        N = f.shape[1]
        ref = oracle.rk4(round32(f), NU, DT, nsteps)
        assert rel_l2(g, ref) < fp32_tol(N), N


def test_persistent_equals_launch_per_pass():
    """Same passes, plans and arithmetic as the per-pass launches of the fused
    schedule; only the tile widths and the compiler's contraction choices in
    the two kernels may differ, so the results agree to a few ulps."""
    print("persistent against the fused per-pass schedule", flush=True)
    fields = _fields(SIZES)
    per, _ = _run(fields, 2, FUSED)
    pk, _ = _run(fields, 2, {"graph": 2})
    same = 0
    for a, b, f in zip(pk, per, fields):
        same += int(np.array_equal(a.view(np.uint32), b.view(np.uint32)))
        assert rel_l2(a, b) < 1e-6, f.shape[1]
    print(f"bitwise equal: {same} of {len(fields)} instances", flush=True)


def test_persistent_zero_steps_is_the_masked_input():
    print("persistent, zero steps", flush=True)
    fields = _fields(SIZES)
    per, _ = _run(fields, 0, FUSED)
    pk, _ = _run(fields, 0, {"graph": 2})
    for a, b in zip(pk, per):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_persistent_graph_replays_equal_eager_run():
    import torch
    print("persistent, graph replays", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager, replays = _run(_fields(SIZES), 1, {"graph": 2}, stream=s, graph_reps=3)
    assert len(replays) == 3
    for rep in replays:
        for a, b in zip(rep, eager):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_persistent_large_batch():
    """A few hundred instances (sizes drawn as in the batch workload): every
    instance against the per-pass schedule, sampled ones against the oracle."""
    sizes = inputs.batch_sizes(320, 7)
    print(f"persistent, {len(sizes)} instances", flush=True)
    fields = _fields(sizes, seed0=5000)
    per, _ = _run(fields, 1, FUSED)
    pk, _ = _run(fields, 1, {"graph": 2})
    for a, b, f in zip(pk, per, fields):
        assert rel_l2(a, b) < 1e-6, f.shape[1]
    for i in (0, 101, 202, 319):
        N = fields[i].shape[1]
        assert rel_l2(pk[i], oracle.rk4(round32(fields[i]), NU, DT, 1)) < fp32_tol(N), N


def test_persistent_wait_bound_ends_the_call():
    """The error path, forced from the host: with the waits bounded to one
    poll, the first wait not met at once raises the error flag, no wait
    follows and the kernel drains (no hang); the scatter items from then on
    write NaN.  The next call with the default bound is correct again (every
    call starts from a zeroed control block)."""
    import torch
    sizes = inputs.batch_sizes(320, 7)
    print(f"persistent, waits bounded to one poll, {len(sizes)} instances", flush=True)
    fields = _fields(sizes, seed0=5000)
    h, wsb = binding.hot_plan([f.shape[1] for f in fields], "rk4", "f32", "two_thirds", NU, DT)
    try:
        binding.hot_set_variant(h, "graph", 2)
        binding.hot_set_variant(h, "persistent", 1)
        assert binding.hot_tuned_width(h, 0, "persistent") == 1
        ws = workspace(wsb)
        ins = [to_dev(f, "f32") for f in fields]
        outs = [torch.empty_like(x) for x in ins]
        binding.hot_run(h, ins, outs, ws, 1)
        torch.cuda.synchronize()
        nan = sum(int(torch.isnan(o).any().item()) for o in outs)
        print(f"instances with NaN output: {nan} of {len(outs)}", flush=True)
        assert nan > 0
        binding.hot_set_variant(h, "persistent", 0)
        binding.hot_run(h, ins, outs, ws, 1)
        torch.cuda.synchronize()
        for i in (0, 150, 319):
            N = fields[i].shape[1]
            got = outs[i].cpu().numpy()
            assert rel_l2(got, oracle.rk4(round32(fields[i]), NU, DT, 1)) < fp32_tol(N), N
    finally:
        binding.hot_destroy(h)


def test_persistent_stats_match_the_per_pass_schedule():
    """stats_dev after a persistent call: E and eps of every instance's state
    equal those after the per-pass schedule to rounding (the states agree to
    a few ulps)."""
    import torch
    print("persistent, stats_dev", flush=True)
    fields = _fields(SIZES)
    res = {}
    for name, variants in (("per_pass", FUSED), ("persistent", {"graph": 2})):
        h, wsb = binding.hot_plan([f.shape[1] for f in fields], "rk4", "f32", "two_thirds", NU, DT)
        try:
            for k, v in variants.items():
                binding.hot_set_variant(h, k, v)
            ins = [to_dev(f, "f32") for f in fields]
            outs = [torch.empty_like(x) for x in ins]
            st = binding.stats_buffer(len(fields))
            binding.hot_run(h, ins, outs, workspace(wsb), 2, stats=st)
            torch.cuda.synchronize()
            res[name] = binding.stats_view(st)
        finally:
            binding.hot_destroy(h)
    E0, eps0, _, _ = res["per_pass"]
    E1, eps1, sw, nc = res["persistent"]
    assert np.all(E0 > 0) and np.all(eps0 > 0)
    np.testing.assert_allclose(E1, E0, rtol=1e-6)
    np.testing.assert_allclose(eps1, eps0, rtol=1e-6)
    assert not np.any(sw) and not np.any(nc)
