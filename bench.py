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
                smaller N on one core), scaled to this workload's unit.
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
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1607_00850_amd", "csrc", "*"))):
        h.update(open(p, "rb").read())
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
            vals[name].append(float(r["Counter_Value"]))
        return vals

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    true_bytes = float(calib_mib) * 2**20
    fs = true_bytes / (fetch[COPY_KERNEL][0] * 1024.0)
    ws = true_bytes / (write[COPY_KERNEL][0] * 1024.0)
    names = {"k_z_cross": "z_cross", "k_x_inv_curl": "x_inv_curl", "k_rk_stage": "rk_stage",
             "k_gather": "gather", "k_scatter": "scatter", "y_inv": "y_inv"}
    out = {"fetch_scale": fs, "write_scale": ws, "command": command}
    for k, pname in names.items():
        if k in fetch and k in write:
            f = sum(fetch[k]) / len(fetch[k]) * 1024.0 * fs
            w = sum(write[k]) / len(write[k]) * 1024.0 * ws
            out[pname] = {"fetch_bytes": f, "write_bytes": w, "hbm_bytes_per_launch": f + w,
                          "dispatches": len(fetch[k]), "source_hash": source_hash()}
    path = os.path.join(ROOT, "profiles", "counters.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d[workload] = out
    json.dump(d, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


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


def batch_fields(sizes, dtype, first_seed=1000):
    """R1 (seed first_seed + i) for every instance, laid out per size in one
    device buffer with 256-byte aligned instance slices."""
    import concurrent.futures

    import numpy as np
    import torch

    cdt = torch.complex64 if dtype == "f32" else torch.complex128
    esz = 8 if dtype == "f32" else 16
    with concurrent.futures.ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        modes = list(ex.map(_r1_modes, [(int(N), first_seed + i) for i, N in enumerate(sizes)], chunksize=64))
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


def bench_batch(a):
    """Many uneven instances: one RK4 step of every instance per call."""
    import numpy as np
    import torch

    from paper_1607_00850_amd import binding, inputs

    sizes = inputs.batch_sizes(a.batch, 0)
    t_gen = time.perf_counter()
    ins, outs, keep = batch_fields(sizes, a.dtype)
    t_gen = time.perf_counter() - t_gen
    plan, wsb = binding.hot_plan([int(v) for v in sizes], "rk4", a.dtype, "two_thirds", NU, DT)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    res = {}
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
        "config": {"workload": f"rk4_batch_{B}_uneven_16-64_{a.dtype}", "instances": B,
                   "sizes": {int(k): int(v) for k, v in zip(*np.unique(sizes, return_counts=True))},
                   "points": int((sizes.astype(np.int64) ** 3).sum()), "nu": NU, "dt": DT,
                   "launch": "one HIP graph replay per batch step (one launch per pass per size inside)"},
        "elements_per_sec": float((sizes.astype(np.float64) ** 3).sum()) / t_graph,
        "eager_instances_per_sec": B / t_eager,
        "one_instance_per_call_instances_per_sec": B / t_single,
        "tuned_y_inv_columns": widths,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "step_roofline": {"model_bytes_per_step": step_bytes, "achieved_GBps": step_bytes / t_graph / 1e9,
                          "frac": step_bytes / t_graph / 1e9 / HBM_PEAK_GBS},
        "setup_seconds": {"fields": t_gen},
    }
    print(json.dumps(line), flush=True)
    del keep


def cpu_baseline(N_work, seconds=12.0):
    """Time the CPU oracle (one core) on RK4 steps at N = 128 and scale to
    instances/s of an N_work^3 step by the FFT cost N^3 log2 N."""
    import numpy as np

    import oracle
    from paper_1607_00850_amd import inputs

    try:
        os.sched_setaffinity(0, {min(os.sched_getaffinity(0))})
    except (AttributeError, OSError):
        pass
    n = 128
    uh = inputs.smooth_random(n, 0)
    steps, t0 = 0, time.perf_counter()
    while True:
        uh = oracle.rk4_step(uh, NU, DT)
        steps += 1
        if time.perf_counter() - t0 > seconds:
            break
    el = time.perf_counter() - t0
    pps = n**3 * steps / el
    scale = (np.log2(N_work) / np.log2(n))
    inst = pps / scale / float(N_work) ** 3
    return {
        "value": inst,
        "unit": "instances/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} RK4 steps of the FP64 oracle at N={n} (R1 seed 0) in {el:.1f} s on 1 core = "
                  f"{pps:.3g} point-steps/s; scaled to N={N_work} by log2(N) ({scale:.3f}x per point)",
    }


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
    ap.add_argument("--workload", default="single", choices=["single", "batch"],
                    help="single: one N^3 field (default); batch: many uneven instances, one RK4 step each")
    ap.add_argument("--batch", type=int, default=4096, help="instances of the batch workload")
    a = ap.parse_args()

    if a.ingest_counters:
        ingest_counters(a.ingest_counters[0], a.ingest_counters[1], a.calibrate_copy,
                        f"rk4_step_{a.n}^3_{a.dtype}", a.pmc_command)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU slab decomposition is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1607_00850_amd import binding

    if a.workload == "batch":
        bench_batch(a)
        return

    if a.calibrate_copy > 0:
        nbytes = a.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

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
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(N, a.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
