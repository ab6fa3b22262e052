"""Benchmark: classical RK4 steps of the pseudo-spectral Navier-Stokes
right-hand side (Eq. NSfinal) on one 1024^3 field in FP32, through libhot.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 1024] [--dtype f32]

Prints ONE JSON line.  A "step" is one RK4 step (four right-hand sides: curl,
6 inverse and 3 forward real 3D FFTs, cross product, 2/3 dealiasing,
projection, viscous term, stage update) of one N^3 field; the W warm-up and
K timed steps each run as one hot_run call (inputs resident in HBM).

Extra fields:
  roofline      dominant pass: algorithmic bytes per launch / mean launch
                time (HIP events on the run stream) against 8 TB/s HBM;
                traffic from the committed rocprofv3 counter summary when its
                source hash matches the kernels built now, else null.
  cpu_baseline  the CPU oracle timed on a bounded sample (RK4 steps at a
                smaller N on one core, then on every allowed core at once,
                up to 16), scaled to this workload's unit.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NU = 1.0 / 1600.0  # Re = 1600 (Sec. 4)
DT = 1e-3          # Sec. 4


def source_hash():
    """Hash of the sources of the right-hand-side and RK4 kernels."""
    h = hashlib.sha256()
    for name in ("fft_core.hpp", "kernels.hpp", "impl.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1607_00850_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def load_counters(kernel, workload):
    """HBM traffic per launch from profiles/counters.json, if it was taken
    with the kernels that are built now."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    rec = d.get(workload, {}).get(kernel)
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


COPY_KERNEL = "__amd_rocclr_copyBuffer"


def ingest_counters(fetch_csv, write_csv, calib_mib, workload, command):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch) of `bench.py --steps 1 --warmup 0 --calibrate-copy MIB` into
    profiles/counters.json: mean HBM bytes per launch for each libhot kernel,
    each counter scaled by what it reads for the plain copy kernel of known
    size (MIB MiB read and MIB MiB written)."""
    import csv
    import re
    from collections import defaultdict

    def per_kernel(path, counter):
        # (dispatch id, KiB) per kernel, in dispatch order
        vals = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            m = re.search(r"hot::(k_\w+)", r["Kernel_Name"])
            name = m.group(1) if m else r["Kernel_Name"]
            if name.startswith("k_strided"):
                m2 = re.search(r"LinePlan<[^>]*>, (-?1), \d+, (true|false), (true|false)", r["Kernel_Name"])
                name = {("1", "true", "false"): "y_inv", ("-1", "false", "true"): "y_or_x_fwd"}.get(
                    m2.groups() if m2 else None, "k_strided")
            vals[name].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        return vals

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    true_bytes = float(calib_mib) * 2**20
    fs = true_bytes / (fetch[COPY_KERNEL][0][1] * 1024.0)
    ws = true_bytes / (write[COPY_KERNEL][0][1] * 1024.0)
    # kernel -> pass; several kernels can serve one pass (the row forms, the
    # x inverse variants); k_strided forward with compact output rows is the
    # y forward pass when the x forward pass is fused with the stage update
    names = {"k_z_cross": "z_cross", "k_z_cross_packed": "z_cross", "k_x_inv_curl": "x_inv_curl",
             "k_x_inv_curl3": "x_inv_curl", "k_rk_stage": "rk_stage", "k_gather": "gather", "k_gather_t": "gather",
             "k_scatter": "scatter", "y_inv": "y_inv", "k_y_inv_pack": "y_inv", "k_x_fwd_rk": "x_fwd_rk",
             "y_or_x_fwd": "y_fwd", "k_y_fwd_unpack": "y_fwd", "k_y_fwd_unpack3": "y_fwd"}
    out = {"fetch_scale": fs, "write_scale": ws, "command": command}
    # only the dispatches of the timed call (its last launches of each pass:
    # one gather and scatter, four of every other pass for the one RK4 step
    # of `--steps 1 --warmup 0`), not the autotuner's timing launches of other
    # variants before it
    last = {"gather": 1, "scatter": 1}
    for pname in sorted(set(names.values())):
        n = last.get(pname, 4)
        fv = [v for _, v in sorted(d for k, nm in names.items() if nm == pname and k in fetch for d in fetch[k])][-n:]
        wv = [v for _, v in sorted(d for k, nm in names.items() if nm == pname and k in write for d in write[k])][-n:]
        if fv and wv:
            f = sum(fv) / len(fv) * 1024.0 * fs
            w = sum(wv) / len(wv) * 1024.0 * ws
            out[pname] = {"fetch_bytes": f, "write_bytes": w, "hbm_bytes_per_launch": f + w,
                          "dispatches": len(fv), "source_hash": source_hash()}
    path = os.path.join(ROOT, "profiles", "counters.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d[workload] = out
    json.dump(d, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


def calibrate_copy(mib):
    """One plain device-to-device copy of `mib` MiB: a kernel of known
    traffic for scaling the HBM byte counters."""
    import torch
    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def device_field(N, dtype, seed=0):
    """R1 (smooth random solenoidal field, E = 1/8) scattered on the GPU."""
    import torch
    from paper_1607_00850_amd import inputs

    ix, iy, iz, vals = inputs.smooth_random_modes(N, seed)
    cdt = torch.complex64 if dtype == "f32" else torch.complex128
    x = torch.zeros((3, N, N, N // 2 + 1), dtype=cdt, device="cuda")
    idx = [torch.from_numpy(a).long().cuda() for a in (ix, iy, iz)]
    x[:, idx[0], idx[1], idx[2]] = torch.from_numpy(vals).to(cdt).cuda()
    return x


def _r1_modes(args):
    from paper_1607_00850_amd import inputs
    N, seed = args
    return inputs.smooth_random_modes(N, seed)


GEN_WORKERS = 16  # host processes generating the batch fields (--gen-workers)


def batch_modes(sizes, first_seed=1000):
    """R1 modes (seed first_seed + i) of every instance, generated by a
    process pool (forked: call before the process touches the GPU), or in
    this process with one worker."""
    import concurrent.futures

    jobs = [(int(N), first_seed + i) for i, N in enumerate(sizes)]
    if GEN_WORKERS <= 1:
        return [_r1_modes(j) for j in jobs]
    with concurrent.futures.ProcessPoolExecutor(min(GEN_WORKERS, os.cpu_count() or 1)) as ex:
        return list(ex.map(_r1_modes, jobs, chunksize=64))


def batch_fields(sizes, dtype, first_seed=1000, modes=None):
    """R1 (seed first_seed + i) for every instance, laid out per size in one
    device buffer with 256-byte aligned instance slices."""
    import numpy as np
    import torch

    esz = 8 if dtype == "f32" else 16
    if modes is None:
        modes = batch_modes(sizes, first_seed)
    ins, outs, keep = [None] * len(sizes), [None] * len(sizes), []
    for N in sorted(set(int(v) for v in sizes)):
        idx = [i for i, v in enumerate(sizes) if int(v) == N]
        n = 3 * N * N * (N // 2 + 1)
        stride = -(-n * esz // 256) * 256 // esz
        host = np.zeros((len(idx), stride), dtype=np.complex64 if dtype == "f32" else np.complex128)
        for b, i in enumerate(idx):
            ix, iy, iz, vals = modes[i]
            for c in range(3):
                host[b, ((c * N + ix) * N + iy) * (N // 2 + 1) + iz] = vals[c]
        dev_in = torch.from_numpy(host).to("cuda")
        dev_out = torch.empty_like(dev_in)
        keep += [dev_in, dev_out]
        for b, i in enumerate(idx):
            ins[i] = dev_in[b, :n]
            outs[i] = dev_out[b, :n]
    return ins, outs, keep


def batch_cpu_baseline(sizes, per_size=2):
    """The CPU oracle on the batch: one RK4 step of `per_size` instances of
    every size (R1, the batch's seeds) on one pinned core, the mean time per
    size summed over the batch's size counts (one core)."""
    import numpy as np

    import oracle
    from paper_1607_00850_amd import inputs

    allowed = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    if allowed:
        os.sched_setaffinity(0, {allowed[0]})
    try:
        per = {}
        for N in sorted(set(int(v) for v in sizes)):
            first = [i for i, v in enumerate(sizes) if int(v) == N][:per_size]
            fields = [inputs.smooth_random(N, 1000 + i) for i in first]
            t0 = time.perf_counter()
            for uh in fields:
                oracle.rk4(uh, NU, DT, 1)
            per[N] = (time.perf_counter() - t0) / len(fields)
    finally:
        if allowed:
            os.sched_setaffinity(0, set(allowed))
    counts = {int(k): int(v) for k, v in zip(*np.unique(sizes, return_counts=True))}
    total = sum(per[N] * c for N, c in counts.items())
    return {
        "value": len(sizes) / total,
        "unit": "instances/s",
        "cores": 1,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": f"one FP64 oracle RK4 step of {per_size} instances per size, {sum(per.values()) * per_size:.1f} s; "
                  f"mean seconds per instance by size {({N: round(t, 4) for N, t in per.items()})}, weighted by the "
                  f"batch's size counts: {total:.1f} s per batch step on 1 core",
    }


# batch schedules (hot_set_variant "graph"): one graph branch per size, the
# sizes chained, or the persistent kernel (one launch for every pass)
GRAPH_LAYOUTS = {"branches": 1, "chain": 0, "persistent": 2}


def bench_batch(a):
    """Many uneven instances: one RK4 step of every instance per call."""
    import numpy as np
    import torch

    from paper_1607_00850_amd import binding, inputs

    sizes = inputs.batch_sizes(a.batch, 0)
    cpu = None if (a.no_cpu_baseline or a.replays_only) else batch_cpu_baseline(sizes)
    t_gen = time.perf_counter()
    ins, outs, keep = batch_fields(sizes, a.dtype)
    t_gen = time.perf_counter() - t_gen
    plan, wsb = binding.hot_plan([int(v) for v in sizes], "rk4", a.dtype, "two_thirds", NU, DT)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    res = {}
    if a.replays_only:
        # for kernel traces of the graph alone: tune, capture, pause half a
        # second (it marks the start of the replays in a trace), replay
        try:
            with torch.cuda.stream(s):
                binding.hot_tune(plan, ws, s)
                binding.hot_set_variant(plan, "graph", GRAPH_LAYOUTS[a.graph_layout])
                g = binding.hot_graph_create(plan, ins, outs, ws, 1, s)
                binding.hot_graph_launch(g, s)
                torch.cuda.synchronize()
                time.sleep(0.5)
                t0 = time.perf_counter()
                for _ in range(a.replays_only):
                    binding.hot_graph_launch(g, s)
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / a.replays_only
                binding.hot_graph_destroy(g)
        finally:
            binding.hot_destroy(plan)
        print(json.dumps({"replays": a.replays_only, "ms_per_replay": t * 1e3, "instances_per_sec": len(sizes) / t}),
              flush=True)
        return None
    try:
        with torch.cuda.stream(s):
            binding.hot_tune(plan, ws, s)
            for _ in range(a.warmup):
                binding.hot_run(plan, ins, outs, ws, 1, s)
            torch.cuda.synchronize()
            # eager: one hot_run per batch step, per-pass events on
            binding.hot_profile_enable(plan, True)
            t0 = time.perf_counter()
            for _ in range(a.steps):
                binding.hot_run(plan, ins, outs, ws, 1, s)
            torch.cuda.synchronize()
            t_eager = (time.perf_counter() - t0) / a.steps
            prof = binding.hot_profile_read(plan)
            binding.hot_profile_enable(plan, False)
            # graph: the whole batch step as one replayed HIP graph
            binding.hot_set_variant(plan, "graph", GRAPH_LAYOUTS[a.graph_layout])
            g = binding.hot_graph_create(plan, ins, outs, ws, 1, s)
            binding.hot_graph_launch(g, s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.steps):
                binding.hot_graph_launch(g, s)
            torch.cuda.synchronize()
            t_graph = (time.perf_counter() - t0) / a.steps
            binding.hot_graph_destroy(g)
        pass_bytes = {}
        for k in prof:
            pass_bytes[k] = sum(binding.hot_pass_bytes(plan, i, k) for i in range(len(sizes)))
        widths = {int(N): binding.hot_tuned_width(plan, int(np.argmax(sizes == N)), "y_inv") for N in set(sizes)}
        yz_sizes = sorted(int(N) for N in set(sizes)
                          if binding.hot_tuned_width(plan, int(np.argmax(sizes == N)), "yz_fused") > 0)
    finally:
        binding.hot_destroy(plan)
    del ws
    # one instance per call: a plan per size, every instance run alone
    plans = {}
    try:
        for N in set(int(v) for v in sizes):
            h, w = binding.hot_plan(N, "rk4", a.dtype, "two_thirds", NU, DT)
            plans[N] = (h, torch.empty(w, dtype=torch.uint8, device="cuda"))
        with torch.cuda.stream(s):
            for i, N in enumerate(sizes[:64]):  # warm-up
                h, w = plans[int(N)]
                binding.hot_run(h, [ins[i]], [outs[i]], w, 1, s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i, N in enumerate(sizes):
                h, w = plans[int(N)]
                binding.hot_run(h, [ins[i]], [outs[i]], w, 1, s)
            torch.cuda.synchronize()
            t_single = time.perf_counter() - t0
    finally:
        for h, _ in plans.values():
            binding.hot_destroy(h)
    B = len(sizes)
    dom = max(prof, key=lambda k: prof[k][0])
    step_bytes = sum(pass_bytes[k] * prof[k][1] for k in prof) / a.steps / 1.0
    # launches per call of a pass = (#sizes) x (uses per call); bytes summed over instances per call
    uses = {k: prof[k][1] / a.steps / len(set(sizes)) for k in prof}
    call_bytes = {k: pass_bytes[k] * uses[k] for k in prof}
    dom_time = prof[dom][0] / a.steps / 1e3
    achieved = call_bytes[dom] / dom_time / 1e9
    step_bytes = sum(call_bytes.values())
    line = {
        "metric": "instances/sec",
        "value": B / t_graph,
        "unit": "instances/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": t_graph * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.dtype,
        "data": "synthetic (R1 per instance, seeds 1000+i; sizes log-uniform over [16, 64], seed 0)",
        "config": {"workload": f"rk4_batch_{B}_uneven_16-64_{a.dtype}", "instances": B, "graph": a.graph_layout,
                   "sizes": {int(k): int(v) for k, v in zip(*np.unique(sizes, return_counts=True))},
                   "points": int((sizes.astype(np.int64) ** 3).sum()), "nu": NU, "dt": DT,
                   "launch": ("one HIP graph replay per batch step (the pointer tables, a setup kernel and one "
                              "persistent kernel for every pass inside)" if a.graph_layout == "persistent" else
                              "one HIP graph replay per batch step (one launch per pass per size inside)")},
        "elements_per_sec": float((sizes.astype(np.float64) ** 3).sum()) / t_graph,
        "eager_instances_per_sec": B / t_eager,
        "one_instance_per_call_instances_per_sec": B / t_single,
        "tuned_y_inv_columns": widths,
        "fused_yz_sizes": yz_sizes,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "step_roofline": {"model_bytes_per_step": step_bytes, "achieved_GBps": step_bytes / t_graph / 1e9,
                          "frac": step_bytes / t_graph / 1e9 / HBM_PEAK_GBS},
        "setup_seconds": {"fields": t_gen},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)
    del keep


IMP_DT = 1e-2  # implicit step: 10x the RK4 step of Sec. 4
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_ROW = 2 * (32 * 256 + 2 * 256 * 256 + 256 * 6)  # the six real outputs (not the padded tile)


def bench_surrogate(a):
    """MLP surrogate for the implicit step: train it on input/output pairs
    of FP64 oracle trajectories at N = 64 (a file written beforehand by
    `python -m oracle.surrogate_data`; this script does not run the oracle),
    then compare plain and surrogate-assisted implicit steps on a batch of
    uneven instances at the same tolerance."""
    import numpy as np
    import torch

    from paper_1607_00850_amd import binding, inputs

    nu, dt, tol = NU, IMP_DT, 1e-5
    sizes = inputs.batch_sizes(a.surrogate_batch, 0)
    modes = batch_modes(sizes)  # host work first: the pool forks before any GPU call
    # ---- training data: input/output pairs of FP64 oracle trajectories at
    # N = 64, written beforehand by `python -m oracle.surrogate_data` (rows
    # drawn with probability ~ s^2 within each field); held out: every
    # retained mode of other oracle trajectories
    t0 = time.perf_counter()
    if not a.train_data or not a.val_data:
        raise SystemExit("--workload surrogate needs --train-data and --val-data (files written by "
                         "`python -m oracle.surrogate_data`)")
    tr = np.load(a.train_data)
    va = np.load(a.val_data)
    X = torch.from_numpy(tr["x"]).cuda()
    T = torch.from_numpy(tr["t"]).cuda()
    Xv = torch.from_numpy(va["x"]).cuda()
    Tv = torch.from_numpy(va["t"]).cuda()
    Sv = torch.from_numpy(va["s"].astype(np.float32)).cuda()
    train = [int(v) for v in tr["seeds"]]
    t_data = time.perf_counter() - t0
    rows = X.shape[0]
    # ---- training (FP32 master weights, BF16 MFMA products, Adam)
    P = binding.hot_mlp_param_count()
    rng = np.random.default_rng(0)
    blocks = []
    for fo, fi in ((256, 32), (256, 256), (256, 256), (6, 256)):  # W uniform +-1/sqrt(fan_in), b zero
        blocks += [rng.uniform(-1 / np.sqrt(fi), 1 / np.sqrt(fi), size=fo * fi), np.zeros(fo)]
    theta = np.concatenate(blocks).astype(np.float32)
    assert theta.size == P
    th = torch.from_numpy(theta).cuda()
    grad = torch.empty(P, dtype=torch.float32, device="cuda")
    m = torch.zeros(P, dtype=torch.float32, device="cuda")
    v = torch.zeros(P, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    mb = a.minibatch
    tws = torch.empty(binding.hot_mlp_train_bytes(mb), dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(0)
    xb = torch.empty((mb, 32), dtype=torch.float32, device="cuda")
    tb = torch.empty((mb, 6), dtype=torch.float32, device="cuda")
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    grad_ms = 0.0
    for step in range(1, a.train_steps + 1):
        idx = torch.randint(0, rows, (mb,), device="cuda", generator=gen)
        torch.index_select(X, 0, idx, out=xb)
        torch.index_select(T, 0, idx, out=tb)
        lr = 1e-3 * (0.5 * (1 + np.cos(np.pi * (step - 1) / a.train_steps)))  # cosine decay
        if step == a.train_steps // 2:
            ev0.record()
        binding.hot_mlp_grad(th, xb, tb, mb, grad, loss, tws)
        if step == a.train_steps // 2:
            ev1.record()
        binding.hot_mlp_adam(th, grad, m, v, step, max(lr, 1e-5))
        if step % max(1, a.train_steps // 10) == 0:
            losses.append(float(loss.item()))
            print(f"train step {step}: loss {losses[-1]:.4g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    grad_ms = ev0.elapsed_time(ev1)
    pk = torch.empty(binding.hot_mlp_packed_bytes(), dtype=torch.uint8, device="cuda")
    binding.hot_mlp_pack(th, pk)
    # validation: error of the predicted correction relative to the plain
    # extrapolation's error (1.0 = no better than the extrapolation)
    val = {"note": "||s (y - t)|| / ||s t||: the increment error of the warm start relative to that of the "
                   "plain extrapolation (1.0 = no better), over the held-out rows"}
    for name, xv, tv, sv in (("held_out_oracle_N64", Xv, Tv, Sv),):
        yv = torch.empty_like(tv)
        binding.hot_mlp_forward(pk, xv, yv, xv.shape[0])
        torch.cuda.synchronize()
        w = sv[:, None]
        val[name] = {"rows": int(xv.shape[0]),
                     "rel_l2": float(torch.linalg.vector_norm(w * (yv - tv)) / torch.linalg.vector_norm(w * tv))}
    # ---- batched comparison (one implicit step per instance, FP32, tol 1e-5)
    ins, mids, keep = batch_fields(sizes, "f32", modes=modes)  # mids: the states advanced in place
    B = len(sizes)
    sample = list(range(0, B, max(1, B // 64)))
    res = {}
    ws = None
    # plain and assisted: the third step (two increments of history: the
    # linear extrapolation, or the surrogate's correction of it); plain_h3,
    # plain_h4: the fourth and fifth steps, whose plain predictor extrapolates
    # three and four increments
    for mode in ("plain", "assisted", "plain_h3", "plain_h4"):
        plan, wsb = binding.hot_plan([int(x) for x in sizes], "implicit", "f32", "two_thirds", nu, dt, tol, 50,
                                     keep_history=True)
        if ws is None:
            ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        try:
            for i in range(B):
                mids[i].copy_(ins[i])
            binding.hot_tune(plan, ws)
            hist = {"plain_h3": 3, "plain_h4": 4}.get(mode, 2)
            binding.hot_run(plan, mids, mids, ws, hist)  # history: plain steps
            if mode == "assisted":
                binding.hot_set_surrogate(plan, pk)
            pre = [mids[i].clone() for i in sample]
            torch.cuda.synchronize()
            binding.hot_profile_enable(plan, True)
            t0 = time.perf_counter()
            rc = binding.hot_run(plan, mids, mids, ws, 1)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            prof = binding.hot_profile_read(plan)
            binding.hot_profile_enable(plan, False)
            sweeps, nonconv = binding.hot_implicit_stats(plan, B)
            res[mode] = {"seconds": el, "instances_per_sec": B / el, "mean_sweeps": float(np.mean(sweeps)),
                         "max_sweeps": int(np.max(sweeps)), "nonconverged": int(np.sum(nonconv)), "rc": rc,
                         "predict_ms": prof.get("imp_predict", (0.0, 0))[0],
                         "sweep_ms": sum(v[0] for k, v in prof.items() if k not in ("imp_predict", "gather",
                                                                                     "scatter", "imp_advance")),
                         "state": [mids[i].clone() for i in sample], "pre": pre}
        finally:
            binding.hot_destroy(plan)
    pre = res["plain"].pop("pre")
    res["assisted"].pop("pre")
    for mode in ("plain_h3", "plain_h4"):
        res[mode].pop("pre")
        res[mode].pop("state")
    diffs = [float(torch.linalg.vector_norm(p - q) / max(float(torch.linalg.vector_norm(p - u)), 1e-300))
             for p, q, u in zip(res["plain"].pop("state"), res["assisted"].pop("state"), pre)]
    # rows the fused MLP kernel runs: every compact slot (no row padding for N <= 64 in FP32)
    mlp_rows = int(sum(binding.hot_mlp_dataset_rows(int(n)) for n in sizes))
    pred_s = res["assisted"]["predict_ms"] / 1e3
    mlp_tflops = mlp_rows * MLP_FLOP_PER_ROW / pred_s / 1e12 if pred_s > 0 else None
    grad_tflops = 3 * mb * MLP_FLOP_PER_ROW / (grad_ms / 1e3) / 1e12 if grad_ms > 0 else None
    line = {
        "metric": "instances/sec",
        "value": res["assisted"]["instances_per_sec"],
        "unit": "instances/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 2,
        "ms_per_step": res["assisted"]["seconds"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (state) / bf16 x bf16 -> f32 (MLP)",
        "data": "synthetic (R1 per instance, seeds 1000+i; sizes log-uniform over [16, 64], seed 0)",
        "config": {"workload": f"implicit_surrogate_batch_{B}_uneven_16-64_f32", "instances": B, "nu": nu,
                   "dt": dt, "tol": tol, "points": int((sizes.astype(np.int64) ** 3).sum()),
                   "timed": "one implicit step per instance after two plain steps of history"},
        "plain": res["plain"],
        "assisted": res["assisted"],
        "plain_h3": res["plain_h3"],
        "plain_h4": res["plain_h4"],
        "speedup_assisted_over_plain": res["plain"]["seconds"] / res["assisted"]["seconds"],
        "speedup_plain_h3_over_plain": res["plain"]["seconds"] / res["plain_h3"]["seconds"],
        "speedup_plain_h4_over_plain": res["plain"]["seconds"] / res["plain_h4"]["seconds"],
        "sweeps_saved_per_instance": res["plain"]["mean_sweeps"] - res["assisted"]["mean_sweeps"],
        "assisted_vs_plain_diff_rel_to_increment": {"max": max(diffs), "mean": float(np.mean(diffs)),
                                                    "sampled_instances": len(diffs)},
        "roofline": {"bound": "mfma", "kernel": "mlp_fused (imp_predict)", "achieved": mlp_tflops,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (mlp_tflops / BF16_PEAK_TFLOPS) if mlp_tflops else None, "traffic": None},
        "training": {"data": "FP64 oracle implicit-midpoint trajectories at N = 64 (oracle.surrogate_data)",
                     "fields": len(train), "train_rows": rows, "steps": a.train_steps,
                     "minibatch": mb, "seconds": t_train, "data_seconds": t_data, "loss_trace": losses,
                     "grad_call_ms": grad_ms, "grad_gemm_tflops": grad_tflops,
                     "grad_mfma_frac": (grad_tflops / BF16_PEAK_TFLOPS) if grad_tflops else None},
        "validation": val,
    }
    print(json.dumps(line), flush=True)


def bench_tg(a):
    """Taylor-Green vortex at Re = 1600 (Sec. 4), one long RK4 run: the
    kinetic energy E(t), the dissipation rate eps(t) = nu <|omega|^2> after
    every step, and the residual of the energy budget dE/dt = -eps of the
    dealiased Galerkin system (trapezoid rule between steps).  There is no
    reference solution to compare with, so the run checks itself."""
    import numpy as np
    import torch

    from paper_1607_00850_amd import binding, inputs

    N, steps, dtype = a.tg_n, a.tg_steps, a.dtype
    cdt = torch.complex64 if dtype == "f32" else torch.complex128
    u = torch.from_numpy(inputs.taylor_green(N)).to(cdt).cuda()
    plan, wsb = binding.hot_plan(N, "rk4", dtype, "two_thirds", NU, DT)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    diag = torch.empty((steps + 1, 2), dtype=torch.float64, device="cuda")
    try:
        binding.hot_tune(plan, ws)
        binding.hot_diagnostics(plan, [u], ws, diag[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in range(steps):
            binding.hot_run(plan, [u], [u], ws, 1)
            binding.hot_diagnostics(plan, [u], ws, diag[n + 1])
            if (n + 1) % 2000 == 0:
                torch.cuda.synchronize()
                print(f"tg step {n + 1}: E {float(diag[n + 1, 0]):.6f} eps {float(diag[n + 1, 1]):.6g}",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        binding.hot_destroy(plan)
    d = diag.cpu().numpy()
    E, eps = d[:, 0], d[:, 1]
    t = DT * np.arange(steps + 1)
    resid = (E[1:] - E[:-1]) / DT + 0.5 * (eps[1:] + eps[:-1])
    k = int(np.argmax(eps))
    every = max(1, steps // 40)
    line = {
        "metric": "instances/sec",
        "value": steps / el,
        "unit": "RK4 steps/s of one field (diagnostics after every step included)",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": el * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "Taylor-Green initial field (Sec. 4), Re = 1600",
        "config": {"workload": f"taylor_green_re1600_{N}^3_{dtype}", "N": N, "nu": NU, "dt": DT, "t_end": DT * steps},
        "E0": float(E[0]),
        "eps0": float(eps[0]),
        "E_end": float(E[-1]),
        "eps_peak": {"t": float(t[k]), "value": float(eps[k])},
        "budget_residual": {"max_abs_over_peak_eps": float(np.max(np.abs(resid)) / eps[k]),
                            "rms_over_peak_eps": float(np.sqrt(np.mean(resid ** 2)) / eps[k])},
        "series": [[float(t[i]), float(E[i]), float(eps[i])] for i in range(0, steps + 1, every)],
    }
    print(json.dumps(line), flush=True)


def _oracle_rk4_rate(seconds, core=None, n=128):
    """RK4 steps of the FP64 oracle at N = n on one core for about `seconds`:
    (steps, elapsed s).  Pins the calling process to `core` (default: its
    lowest allowed core)."""
    import oracle
    from paper_1607_00850_amd import inputs

    try:
        os.sched_setaffinity(0, {min(os.sched_getaffinity(0)) if core is None else core})
    except (AttributeError, OSError):
        pass
    uh = inputs.smooth_random(n, 0)
    steps, t0 = 0, time.perf_counter()
    while True:
        uh = oracle.rk4_step(uh, NU, DT)
        steps += 1
        if time.perf_counter() - t0 > seconds:
            break
    return steps, time.perf_counter() - t0


def bench_slab(a):
    """One share of a z-slab decomposed field at its real shape: share
    `rank` of `ranks` of an N^3 field (2048^3 over 8 shares by default, the
    paper's largest mesh, which one MI355X cannot hold whole).  Times RK4
    steps of the share's local passes (per stage: inverse x and y passes,
    z passes with u x omega, forward y and x passes with the stage update).
    The two all-to-alls per stage belong to the multi-GPU collective and are
    not run: on one GPU there is no peer to exchange with, so the z pass
    transforms whatever its receive buffer holds (the timing of every pass
    is independent of the values).  The exchanged bytes are reported."""
    import torch

    from paper_1607_00850_amd import binding, inputs

    N, R, rank, dtype = a.n, a.ranks, a.rank, a.dtype
    cdt = torch.complex64 if dtype == "f32" else torch.complex128
    if a.calibrate_copy > 0:
        calibrate_copy(a.calibrate_copy)
    plan, wsb = binding.hot_plan_slab(N, "rk4", R, rank, dtype, "two_thirds", NU, DT)
    try:
        lay = binding.hot_slab_layout_of(plan)
        ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda")
        # R1 (seed 0), the part of it in this share's kz slab
        ix, iy, iz, vals = inputs.smooth_random_modes(N, 0)
        keep = (iz >= lay.kz0) & (iz < lay.kz0 + lay.nkz)
        x = torch.zeros((3, N, N, lay.nkz), dtype=cdt, device="cuda")
        idx = [torch.from_numpy(v[keep]).long().cuda() for v in (ix, iy, iz - lay.kz0)]
        x[:, idx[0], idx[1], idx[2]] = torch.from_numpy(vals[:, keep]).to(cdt).cuda()
        y = torch.empty_like(x)
        stream = torch.cuda.current_stream()
        widths = {}
        if not a.no_tune:
            binding.hot_tune(plan, ws, stream)
            widths = {k: binding.hot_tuned_width(plan, 0, k) for k in ("x_inv_curl", "y_inv", "y_fwd", "x_fwd",
                                                                       "x_fwd_rk")}

        def steps(k):
            for _ in range(k):
                for st in range(4):
                    for ph in (binding.HOT_SLAB_INVERSE, binding.HOT_SLAB_CROSS, binding.HOT_SLAB_FORWARD):
                        binding.hot_slab_run(plan, ph, ws, stage=st, stream=stream)

        binding.hot_slab_run(plan, binding.HOT_SLAB_GATHER, ws, inp=x, stream=stream)
        steps(a.warmup)
        torch.cuda.synchronize()
        binding.hot_profile_enable(plan, True)
        t0 = time.perf_counter()
        steps(a.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = binding.hot_profile_read(plan)
        binding.hot_profile_enable(plan, False)
        binding.hot_slab_run(plan, binding.HOT_SLAB_SCATTER, ws, out=y, stream=stream)
        torch.cuda.synchronize()
        pass_bytes = {k: binding.hot_pass_bytes(plan, 0, k) for k in prof}
    finally:
        binding.hot_destroy(plan)
    ms_step = (t1 - t0) * 1e3 / a.steps
    dom = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches = prof[dom]
    achieved = pass_bytes[dom] / (tot_ms / launches / 1e3) / 1e9
    passes = {k: {"ms_per_launch": prof[k][0] / prof[k][1], "launches": prof[k][1],
                  "GBps": pass_bytes[k] / (prof[k][0] / prof[k][1] / 1e3) / 1e9,
                  "model_bytes_per_launch": pass_bytes[k]} for k in sorted(prof)}
    step_bytes = sum(pass_bytes[k] * prof[k][1] for k in prof) / a.steps
    # per stage: six components out and three back, one block per peer each
    exch = 4 * (6 + 3) * (R - 1) * lay.block_bytes
    workload = f"rk4_step_share_{rank}_of_{R}_{N}^3_{dtype}"
    line = {
        "metric": "instances/sec",
        "value": 1e3 / ms_step,
        "unit": "RK4 steps/s of one share's local passes",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (R1 seed 0: the part in this share's kz slab)",
        "config": {"workload": workload, "N": N, "shares": R, "share": rank,
                   "x_planes": lay.nx, "kz0": lay.kz0, "retained_kz": lay.mz, "z_pitch": lay.pitch,
                   "nu": NU, "dt": DT, "exchange": "not run (one GPU)"},
        "elements_per_sec": float(N) ** 3 / R * 1e3 / ms_step,
        "exchange_bytes_per_step": {"sent": exch, "received": exch},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": load_counters(dom, workload)},
        "step_roofline": {"model_bytes_per_step": step_bytes, "achieved_GBps": step_bytes / (ms_step / 1e3) / 1e9,
                          "frac": step_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        "passes": passes,
        "tuned_columns": widths,
        "workspace_GB": wsb / 1e9,
    }
    print(json.dumps(line), flush=True)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), and its core count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} logical cores"


def cpu_baseline(N_work, seconds=12.0, max_procs=16):
    """Time the CPU oracle on RK4 steps at N = 128 and scale to instances/s of
    an N_work^3 step by the FFT cost N^3 log2 N: once on one pinned core (the
    reported value), then as one pinned single-threaded process per allowed
    core (at most max_procs), all at once (all_cores).  Runs before the GPU is
    touched: the worker processes are forked."""
    import concurrent.futures

    import numpy as np

    n = 128
    scale = np.log2(N_work) / np.log2(n)
    allowed = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    steps, el = _oracle_rk4_rate(seconds, n=n)
    if allowed:
        os.sched_setaffinity(0, set(allowed))
    pps = n**3 * steps / el
    out = {
        "value": pps / scale / float(N_work) ** 3,
        "unit": "instances/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} RK4 steps of the FP64 oracle at N={n} (R1 seed 0) in {el:.1f} s on 1 core = "
                  f"{pps:.3g} point-steps/s; scaled to N={N_work} by log2(N) ({scale:.3f}x per point)",
    }
    out["cpu_model"] = cpu_model()
    # one measured step at 256^3 beside the extrapolation from 128^3
    s256, el256 = _oracle_rk4_rate(0.0, n=256)
    out["measured_256"] = {
        "seconds_per_rk4_step": el256 / s256,
        "point_steps_per_s": 256**3 * s256 / el256,
        "scaled_from_128": pps * np.log2(128) / np.log2(256),
    }
    cores = allowed[:max_procs]
    if len(cores) > 1:
        with concurrent.futures.ProcessPoolExecutor(len(cores)) as ex:
            runs = list(ex.map(_oracle_rk4_rate, [seconds] * len(cores), cores))
        agg = sum(n**3 * st / t for st, t in runs)
        out["all_cores"] = {
            "value": agg / scale / float(N_work) ** 3,
            "unit": "instances/s",
            "cores": len(cores),
            "sample": f"{len(cores)} pinned single-threaded oracle processes at once, each RK4 steps at N={n} for "
                      f"about {seconds:.0f} s ({sum(st for st, _ in runs)} steps in all) = {agg:.3g} point-steps/s; "
                      f"scaled as above",
        }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default column widths (no hot_tune)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (a known-size kernel "
                         "for scaling HBM byte counters)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/counters.json from two rocprofv3 --pmc counter_collection.csv files "
                         "(no GPU needed); use with --calibrate-copy MIB and --pmc-command")
    ap.add_argument("--pmc-command", default="", help="the profiled command, recorded with the counters")
    ap.add_argument("--ingest-workload", default="",
                    help="workload key for --ingest-counters (default: the single-field key of --n and --dtype)")
    ap.add_argument("--gen-workers", type=int, default=16, help="batch workloads: field generation processes")
    ap.add_argument("--tg-n", type=int, default=256, help="tg: points per axis")
    ap.add_argument("--tg-steps", type=int, default=20000, help="tg: RK4 steps (dt = 1e-3)")
    ap.add_argument("--train-data", default="", help="surrogate: training pairs (python -m oracle.surrogate_data)")
    ap.add_argument("--val-data", default="", help="surrogate: held-out pairs (python -m oracle.surrogate_data)")
    ap.add_argument("--train-steps", type=int, default=3000, help="surrogate: Adam steps")
    ap.add_argument("--minibatch", type=int, default=4096, help="surrogate: rows per Adam step")
    ap.add_argument("--surrogate-batch", type=int, default=16384, help="surrogate: instances compared")
    ap.add_argument("--workload", default="single", choices=["single", "batch", "surrogate", "tg", "slab"],
                    help="single: one N^3 field (default); batch: many uneven instances, one RK4 step each; "
                         "slab: one share of a z-slab decomposed field (use with --n 2048)")
    ap.add_argument("--ranks", type=int, default=8, help="slab: shares of the field")
    ap.add_argument("--rank", type=int, default=0, help="slab: the share timed")
    ap.add_argument("--batch", type=int, default=4096, help="instances of the batch workload")
    ap.add_argument("--graph-layout", default="branches", choices=["branches", "chain", "persistent"],
                    help="batch: one graph branch per size (default), the sizes one after another, or the "
                         "persistent kernel (every pass of the call in one launch)")
    ap.add_argument("--replays-only", type=int, default=0, metavar="K",
                    help="batch: tune, capture, pause 0.5 s, replay the graph K times and print only that "
                         "(for kernel traces of the replays)")
    a = ap.parse_args()
    global GEN_WORKERS
    GEN_WORKERS = a.gen_workers

    if a.ingest_counters:
        ingest_counters(a.ingest_counters[0], a.ingest_counters[1], a.calibrate_copy,
                        a.ingest_workload or f"rk4_step_{a.n}^3_{a.dtype}", a.pmc_command)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(f"bench.py: libhot runs on one GPU (asked for --gpus {a.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU slab decomposition is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    # the CPU oracle first: its worker processes are forked before the GPU is touched
    cpu = None
    if a.workload == "single" and not a.no_cpu_baseline:
        cpu = cpu_baseline(a.n, a.cpu_seconds)

    import torch

    from paper_1607_00850_amd import binding

    if a.workload == "batch":
        bench_batch(a)
        return
    if a.workload == "surrogate":
        bench_surrogate(a)
        return
    if a.workload == "tg":
        bench_tg(a)
        return
    if a.workload == "slab":
        bench_slab(a)
        return

    if a.calibrate_copy > 0:
        calibrate_copy(a.calibrate_copy)

    N, dtype = a.n, a.dtype
    x = device_field(N, dtype)
    y = torch.empty_like(x)
    plan, wsb = binding.hot_plan(N, "rk4", dtype, "two_thirds", NU, DT)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    try:
        widths = {}
        if not a.no_tune:
            binding.hot_tune(plan, ws, stream)
            widths = {k: binding.hot_tuned_width(plan, 0, k) for k in ("x_inv_curl", "y_inv", "y_fwd", "x_fwd")}
        binding.hot_run(plan, [x], [y], ws, a.warmup, stream)
        torch.cuda.synchronize()
        binding.hot_profile_enable(plan, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binding.hot_run(plan, [x], [y], ws, a.steps, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = binding.hot_profile_read(plan)
        binding.hot_profile_enable(plan, False)
        pass_bytes = {k: binding.hot_pass_bytes(plan, 0, k) for k in prof}
    finally:
        binding.hot_destroy(plan)

    ms_step = (t1 - t0) * 1e3 / a.steps
    inst_s = 1e3 / ms_step
    dom = max(prof, key=lambda k: prof[k][0])
    tot_ms, launches = prof[dom]
    avg_s = tot_ms / launches / 1e3
    achieved = pass_bytes[dom] / avg_s / 1e9
    workload = f"rk4_step_{N}^3_{dtype}"
    traffic = load_counters(dom, workload)
    passes = {k: {"ms_per_launch": prof[k][0] / prof[k][1], "launches": prof[k][1],
                  "GBps": pass_bytes[k] / (prof[k][0] / prof[k][1] / 1e3) / 1e9,
                  "model_bytes_per_launch": pass_bytes[k]} for k in sorted(prof)}
    step_bytes = sum(pass_bytes[k] * prof[k][1] for k in prof) / a.steps
    line = {
        "metric": "instances/sec",
        "value": inst_s,
        "unit": "instances/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (R1: seeded smooth random solenoidal field, E=1/8)",
        "config": {"workload": workload, "N": N, "instances_per_launch": 1, "nu": NU, "dt": DT,
                   "dealias": "two_thirds", "steps_per_call": a.steps},
        "elements_per_sec": float(N) ** 3 * inst_s,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "step_roofline": {"model_bytes_per_step": step_bytes, "achieved_GBps": step_bytes / (ms_step / 1e3) / 1e9,
                          "frac": step_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        "passes": passes,
        "tuned_columns": widths,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
