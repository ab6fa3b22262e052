"""Test helpers: run one libhot operation on the GPU through the C ABI.

Only marshalling lives here: numpy arrays go to device tensors, the C ABI is
called, results come back to numpy.
"""
import json
import os

import numpy as np

from paper_1607_00850_amd import binding

CDT = {"f64": "complex128", "f32": "complex64"}
RDT = {"f64": "float64", "f32": "float32"}


def _torch():
    import torch
    return torch


def to_dev(x, dtype):
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(x.astype(CDT[dtype] if np.iscomplexobj(x) else RDT[dtype])))
    return t.to("cuda")


def empty_spectral(N, dtype):
    torch = _torch()
    return torch.empty((3, N, N, N // 2 + 1), dtype=getattr(torch, CDT[dtype]), device="cuda")


def empty_physical(N, dtype):
    torch = _torch()
    return torch.empty((3, N, N, N), dtype=getattr(torch, RDT[dtype]), device="cuda")


def workspace(nbytes):
    torch = _torch()
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
    assert ws.data_ptr() % 256 == 0
    return ws


def run(op, arrays, dtype="f64", dealias="two_thirds", nu=0.0, dt=0.0, nsteps=0, inplace=False, variants=None):
    """arrays: list of numpy inputs (one per instance).  Returns numpy outputs.
    variants: {pass name: variant} forced on the plan before the run."""
    torch = _torch()
    ns = [a.shape[1] for a in arrays]
    h, wsb = binding.hot_plan(ns, op, dtype, dealias, nu, dt)
    try:
        for name, v in (variants or {}).items():
            binding.hot_set_variant(h, name, v)
        ins = [to_dev(a, dtype) for a in arrays]
        if inplace:
            outs = ins
        elif op == "c2r":
            outs = [empty_physical(N, dtype) for N in ns]
        else:
            outs = [empty_spectral(N, dtype) for N in ns]
        ws = workspace(wsb)
        binding.hot_run(h, ins, outs, ws, nsteps)
        torch.cuda.synchronize()
        return [o.cpu().numpy() for o in outs]
    finally:
        binding.hot_destroy(h)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    den = np.linalg.norm(b)
    return note(float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a)))


def note(err):
    """Record an observed relative error under the running test's id when
    HOT_ERRLOG names a file (the per-family error tables); returns err."""
    log = os.environ.get("HOT_ERRLOG")
    if log:
        with open(log, "a") as f:
            f.write(json.dumps({"test": os.environ.get("PYTEST_CURRENT_TEST", "?"), "err": float(err)}) + "\n")
    return err


# unit roundoff of FP32 (round to nearest): 2^-24
U32 = 2.0**-24


def fp32_tol(N, C=10.0):
    """Tolerance for the FP32 path: C * u32 * log2(N^3), u32 = 2^-24 the unit
    roundoff (1.07e-5 at N = 64, 1.79e-5 at N = 1024)."""
    return C * U32 * np.log2(float(N) ** 3)


def round32(x):
    """The FP32-rounded input, upcast back to FP64 (what the FP32 path sees)."""
    return x.astype(np.complex64).astype(np.complex128) if np.iscomplexobj(x) else x.astype(np.float32).astype(np.float64)


def run_implicit(arrays, dtype="f64", nu=0.0, dt=1e-3, nsteps=1, tol=1e-10, max_iter=50, inplace=False,
                 dealias="two_thirds", variants=None):
    """The implicit step through the C ABI.  Returns (outputs, sweeps per
    instance, max_iter stops per instance, return code)."""
    torch = _torch()
    ns = [a.shape[1] for a in arrays]
    h, wsb = binding.hot_plan(ns, "implicit", dtype, dealias, nu, dt, tol, max_iter)
    try:
        for name, v in (variants or {}).items():
            binding.hot_set_variant(h, name, v)
        ins = [to_dev(a, dtype) for a in arrays]
        outs = ins if inplace else [empty_spectral(N, dtype) for N in ns]
        ws = workspace(wsb)
        rc = binding.hot_run(h, ins, outs, ws, nsteps)
        torch.cuda.synchronize()
        sweeps, nonconv = binding.hot_implicit_stats(h, len(arrays))
        if rc == binding.HOT_OK and any(nonconv):
            rc = binding.HOT_E_NOCONVERGE  # as hot_implicit_stats reports it
        return [o.cpu().numpy() for o in outs], sweeps, nonconv, rc
    finally:
        binding.hot_destroy(h)
