"""Batched instances of uneven N in one plan: each pass runs as one launch per
distinct N over all its instances.  Checked per instance against the oracle,
bit for bit against the same instance run alone, through a captured HIP
graph replayed several times, after autotuning, and after the pointer
tables change."""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import fp32_tol, rel_l2, round32, to_dev, workspace

pytestmark = pytest.mark.gpu

NU, DT = 1.0 / 1600.0, 1e-3
SIZES = [16, 18, 24, 16, 32, 36, 48, 24, 54, 64, 16, 32]


def _fields(dtype):
    return [inputs.rough_random(N, 300 + i) for i, N in enumerate(SIZES)]


def _plan_run(fields, dtype, nsteps, op="rk4", stream=None, tune=False, graph_reps=0, variants=None):
    import torch
    h, wsb = binding.hot_plan([f.shape[1] for f in fields], op, dtype, "two_thirds", NU, DT)
    try:
        ws = workspace(wsb)
        ins = [to_dev(f, dtype) for f in fields]
        outs = [torch.empty_like(x) for x in ins]
        if tune:
            binding.hot_tune(h, ws, stream)
        for name, v in (variants or {}).items():
            binding.hot_set_variant(h, name, v)
        binding.hot_run(h, ins, outs, ws, nsteps, stream)
        torch.cuda.synchronize()
        eager = [o.cpu().numpy() for o in outs]
        replays = []
        if graph_reps:
            g = binding.hot_graph_create(h, ins, outs, ws, nsteps, stream)
            try:
                for r in range(graph_reps):
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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_rk4_matches_oracle_per_instance(dtype):
    print(f"batch rk4 {dtype}", flush=True)
    fields = _fields(dtype)
    got, _ = _plan_run(fields, dtype, 1)
    for f, g in zip(fields, got):
        N = f.shape[1]
        ref = oracle.rk4(round32(f) if dtype == "f32" else f, NU, DT, 1)
        assert rel_l2(g, ref) < (1e-12 if dtype == "f64" else fp32_tol(N)), N


def test_batched_rhs_matches_oracle_per_instance():
    fields = _fields("f64")
    got, _ = _plan_run(fields, "f64", 0, op="rhs")
    for f, g in zip(fields, got):
        assert rel_l2(g, oracle.rhs(f, NU)) < 1e-12


def test_batched_instance_equals_its_single_run_bitwise():
    fields = _fields("f32")
    batch, _ = _plan_run(fields, "f32", 2)
    for i in (0, 2, 5, 9):
        single, _ = _plan_run([fields[i]], "f32", 2)
        assert np.array_equal(batch[i].view(np.uint32), single[0].view(np.uint32)), SIZES[i]


@pytest.mark.parametrize("branches", [1, 0])
def test_graph_replays_equal_eager_run(branches):
    # branches = 1: one graph branch per size (the default); 0: one chain
    import torch
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager, replays = _plan_run(_fields("f32"), "f32", 1, stream=s, graph_reps=3, variants={"graph": branches})
    assert len(replays) == 3
    for rep in replays:
        for a, b in zip(rep, eager):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_graph_replays_with_fused_passes_equal_eager_run():
    """The fused y-z pass (small sizes) and the fused x pass inside a captured
    graph: every replay equals the eager run bit for bit."""
    import torch
    s = torch.cuda.Stream()
    fused = {"yz_fused": 0, "x_fwd_rk": 1}
    with torch.cuda.stream(s):
        eager, replays = _plan_run(_fields("f32"), "f32", 1, stream=s, graph_reps=3, variants=fused)
    assert len(replays) == 3
    for rep in replays:
        for a, b in zip(rep, eager):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    for f, g in zip(_fields("f32"), eager):
        assert rel_l2(g, oracle.rk4(round32(f), NU, DT, 1)) < fp32_tol(f.shape[1])


def test_autotuned_plan_stays_correct():
    fields = _fields("f32")
    got, _ = _plan_run(fields, "f32", 1, tune=True)
    for f, g in zip(fields, got):
        assert rel_l2(g, oracle.rk4(round32(f), NU, DT, 1)) < fp32_tol(f.shape[1])


def test_pointer_tables_follow_new_arrays():
    import torch
    fields = _fields("f64")[:5]
    h, wsb = binding.hot_plan([f.shape[1] for f in fields], "rhs", "f64", "two_thirds", NU, DT)
    try:
        ws = workspace(wsb)
        ins = [to_dev(f, "f64") for f in fields]
        outs = [torch.empty_like(x) for x in ins]
        binding.hot_run(h, ins, outs, ws)
        ins2 = [to_dev(f * 2.0, "f64") for f in fields]  # new arrays, new pointers
        outs2 = [torch.empty_like(x) for x in ins2]
        binding.hot_run(h, ins2, outs2, ws)
        torch.cuda.synchronize()
        for f, o1, o2 in zip(fields, outs, outs2):
            assert rel_l2(o1.cpu().numpy(), oracle.rhs(f, NU)) < 1e-12
            assert rel_l2(o2.cpu().numpy(), oracle.rhs(2.0 * f, NU)) < 1e-12
    finally:
        binding.hot_destroy(h)


def test_graph_keeps_its_pointers_after_a_run_on_other_arrays():
    # a graph made on arrays A, then an eager call on arrays B over the same
    # workspace, then a replay: the replay must read and write A only
    import torch
    fields = _fields("f32")[:6]
    h, wsb = binding.hot_plan([f.shape[1] for f in fields], "rk4", "f32", "two_thirds", NU, DT)
    try:
        ws = workspace(wsb)
        ins_a = [to_dev(f, "f32") for f in fields]
        outs_a = [torch.zeros_like(x) for x in ins_a]
        ins_b = [to_dev(inputs.rough_random(f.shape[1], 900 + i), "f32") for i, f in enumerate(fields)]
        outs_b = [torch.zeros_like(x) for x in ins_b]
        s = torch.cuda.Stream()  # graphs are captured on a non-default stream
        torch.cuda.synchronize()
        g = binding.hot_graph_create(h, ins_a, outs_a, ws, 1, s)
        try:
            binding.hot_run(h, ins_b, outs_b, ws, 1, s)
            torch.cuda.synchronize()
            want_b = [o.cpu().numpy() for o in outs_b]
            for o in outs_b:
                o.fill_(7.0)
            torch.cuda.synchronize()
            binding.hot_graph_launch(g, s)
            torch.cuda.synchronize()
        finally:
            binding.hot_graph_destroy(g)
        for o in outs_b:  # B untouched by the replay
            assert bool((o == 7.0).all())
        for f, o in zip(fields, outs_a):
            assert rel_l2(o.cpu().numpy(), oracle.rk4(round32(f), NU, DT, 1)) < fp32_tol(f.shape[1])
        for f, w in zip(ins_b, want_b):
            ref = oracle.rk4(f.cpu().numpy().astype(np.complex128), NU, DT, 1)
            assert rel_l2(w, ref) < fp32_tol(f.shape[1])
    finally:
        binding.hot_destroy(h)
