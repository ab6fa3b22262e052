"""ctypes binding of libhot (include/hot.h): argument marshalling only.

Every computation runs in the HIP kernels of libhot.so; this module converts
Python values and torch tensors into the C ABI's plain pointers and sizes.
The first call fails loudly if the library has not been built.  The
environment variable HOT_LIBRARY may name another build of the same library.
"""
from __future__ import annotations

import ctypes
import os

from .build import LIB

HOT_ABI_VERSION = 3
HOT_OK = 0
HOT_E_INVALID = -1
HOT_E_UNSUPPORTED = -2
HOT_E_WORKSPACE = -3
HOT_E_HIP = -4
HOT_E_NONFINITE = -5
HOT_E_NOCONVERGE = -6
HOT_E_TOOBIG = -7

HOT_F64, HOT_F32 = 0, 1
HOT_DEALIAS_TWO_THIRDS, HOT_DEALIAS_NONE = 0, 1
HOT_OP_R2C, HOT_OP_C2R, HOT_OP_RHS, HOT_OP_RK4, HOT_OP_IMPLICIT = 0, 1, 2, 3, 4

HOT_FLAG_KEEP_HISTORY = 1
HOT_FLAG_CHECK_FINITE = 2
HOT_SLAB_GATHER, HOT_SLAB_INVERSE, HOT_SLAB_CROSS, HOT_SLAB_FORWARD, HOT_SLAB_SCATTER = 0, 1, 2, 3, 4

DTYPES = {"f64": HOT_F64, "f32": HOT_F32}
DEALIAS = {"two_thirds": HOT_DEALIAS_TWO_THIRDS, "none": HOT_DEALIAS_NONE}
OPS = {"r2c": HOT_OP_R2C, "c2r": HOT_OP_C2R, "rhs": HOT_OP_RHS, "rk4": HOT_OP_RK4, "implicit": HOT_OP_IMPLICIT}


class HotDesc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("n", ctypes.POINTER(ctypes.c_int32)),
        ("nu", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("dtype", ctypes.c_int32),
        ("dealias", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class HotSlabLayout(ctypes.Structure):
    _fields_ = [
        ("nranks", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("kz0", ctypes.c_int32),
        ("nkz", ctypes.c_int32),
        ("mz", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("pitch", ctypes.c_int32),
        ("send_offset", ctypes.c_size_t),
        ("recv_offset", ctypes.c_size_t),
        ("comp_bytes", ctypes.c_size_t),
        ("block_bytes", ctypes.c_size_t),
    ]


class HotError(RuntimeError):
    def __init__(self, code, where, hip=0):
        self.code = code
        self.hip = hip
        msg = f"{where}: {_lib().hot_error_string(code).decode()} ({code})"
        if hip:
            msg += f", HIP error {hip}"
        super().__init__(msg)


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("HOT_LIBRARY", LIB)
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_1607_00850_amd.build`")
        lib = ctypes.CDLL(path)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        lib.hot_plan.argtypes = [ctypes.POINTER(HotDesc), ctypes.POINTER(vp), ctypes.POINTER(sz)]
        lib.hot_plan.restype = ctypes.c_int
        lib.hot_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, i32, vp, vp]
        lib.hot_run.restype = ctypes.c_int
        lib.hot_run_noalloc.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp, vp]
        lib.hot_run_noalloc.restype = ctypes.c_int
        lib.hot_destroy.argtypes = [vp]
        lib.hot_destroy.restype = ctypes.c_int
        lib.hot_error_string.argtypes = [ctypes.c_int]
        lib.hot_error_string.restype = ctypes.c_char_p
        lib.hot_last_hip_error.argtypes = [vp]
        lib.hot_last_hip_error.restype = ctypes.c_int
        lib.hot_profile_enable.argtypes = [vp, ctypes.c_int]
        lib.hot_profile_enable.restype = ctypes.c_int
        lib.hot_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        lib.hot_profile_read.restype = ctypes.c_int
        lib.hot_pass_name.argtypes = [i32]
        lib.hot_pass_name.restype = ctypes.c_char_p
        lib.hot_pass_bytes.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double)]
        lib.hot_pass_bytes.restype = ctypes.c_int
        lib.hot_graph_create.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, i32, vp, vp,
                                         ctypes.POINTER(vp)]
        lib.hot_graph_create.restype = ctypes.c_int
        lib.hot_graph_launch.argtypes = [vp, vp]
        lib.hot_graph_launch.restype = ctypes.c_int
        lib.hot_graph_destroy.argtypes = [vp]
        lib.hot_graph_destroy.restype = ctypes.c_int
        lib.hot_tune.argtypes = [vp, vp, vp, i32]
        lib.hot_tune.restype = ctypes.c_int
        lib.hot_tuned_width.argtypes = [vp, i32, i32]
        lib.hot_tuned_width.restype = ctypes.c_int
        lib.hot_diagnostics.argtypes = [vp, ctypes.POINTER(vp), vp, vp, vp]
        lib.hot_diagnostics.restype = ctypes.c_int
        lib.hot_set_variant.argtypes = [vp, i32, i32]
        lib.hot_set_variant.restype = ctypes.c_int
        lib.hot_implicit_stats.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.hot_implicit_stats.restype = ctypes.c_int
        lib.hot_set_surrogate.argtypes = [vp, vp]
        lib.hot_set_surrogate.restype = ctypes.c_int
        lib.hot_mlp_param_count.argtypes = []
        lib.hot_mlp_param_count.restype = i32
        lib.hot_mlp_packed_bytes.argtypes = []
        lib.hot_mlp_packed_bytes.restype = sz
        lib.hot_mlp_pack.argtypes = [vp, vp, vp]
        lib.hot_mlp_pack.restype = ctypes.c_int
        lib.hot_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
        lib.hot_mlp_forward.restype = ctypes.c_int
        lib.hot_mlp_train_bytes.argtypes = [i32]
        lib.hot_mlp_train_bytes.restype = sz
        lib.hot_mlp_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
        lib.hot_mlp_grad.restype = ctypes.c_int
        lib.hot_mlp_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, vp]
        lib.hot_mlp_adam.restype = ctypes.c_int
        lib.hot_mlp_dataset_rows.argtypes = [i32]
        lib.hot_mlp_dataset_rows.restype = ctypes.c_int64
        lib.hot_mlp_dataset.argtypes = [i32, i32, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp]
        lib.hot_mlp_dataset.restype = ctypes.c_int
        lib.hot_plan_slab.argtypes = [ctypes.POINTER(HotDesc), i32, i32, ctypes.POINTER(vp), ctypes.POINTER(sz)]
        lib.hot_plan_slab.restype = ctypes.c_int
        lib.hot_slab_layout_of.argtypes = [vp, ctypes.POINTER(HotSlabLayout)]
        lib.hot_slab_layout_of.restype = ctypes.c_int
        lib.hot_slab_run.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        lib.hot_slab_run.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library object."""
    return _lib()


def hot_plan(n, op, dtype="f64", dealias="two_thirds", nu=0.0, dt=0.0, tol=1e-10, max_iter=50,
             keep_history=False, check_finite=False):
    """Plan an operation; returns (handle, workspace_bytes).  n: int or list.
    tol, max_iter, keep_history: the implicit step (ignored otherwise);
    check_finite: hot_run scans its results for NaN and infinity."""
    ns = [int(n)] if isinstance(n, int) else [int(v) for v in n]
    arr = (ctypes.c_int32 * len(ns))(*ns)
    flags = (HOT_FLAG_KEEP_HISTORY if keep_history else 0) | (HOT_FLAG_CHECK_FINITE if check_finite else 0)
    d = HotDesc(HOT_ABI_VERSION, len(ns), arr, float(nu), float(dt), DTYPES[dtype], DEALIAS[dealias], OPS[op],
                flags, float(tol), int(max_iter), 0)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    rc = _lib().hot_plan(ctypes.byref(d), ctypes.byref(h), ctypes.byref(ws))
    if rc != HOT_OK:
        raise HotError(rc, "hot_plan")
    return h, ws.value


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def hot_run(plan, ins, outs, workspace, nsteps=0, stream=None, stats=None):
    """Enqueue the planned op.  ins/outs: sequences of device tensors (or raw
    pointers), one per instance; workspace: device tensor or pointer;
    stream: a torch.cuda.Stream, a raw hipStream_t, or None for torch's
    current stream; stats: None, or a device buffer of batch hot_stats
    records (24 bytes each, see stats_view).  Returns HOT_OK, or for a plan
    with check_finite HOT_E_NONFINITE (a NaN or infinity) or
    HOT_E_NOCONVERGE (an implicit step stopped at max_iter); raises
    otherwise."""
    stream = _stream(stream)
    n = len(ins)
    pin = (ctypes.c_void_p * n)(*[_ptr(t) for t in ins])
    pout = (ctypes.c_void_p * n)(*[_ptr(t) for t in outs])
    rc = _lib().hot_run(plan, pin, pout, _ptr(workspace), int(nsteps), _ptr(stats), stream)
    if rc not in (HOT_OK, HOT_E_NOCONVERGE, HOT_E_NONFINITE):
        raise HotError(rc, "hot_run", _lib().hot_last_hip_error(plan))
    return rc


def hot_run_noalloc(plan, ins, outs, nsteps=0, stream=None, stats=None):
    """hot_run on the library's static 16 MiB scratch instead of a workspace
    (for callers that cannot allocate).  Returns as hot_run; raises HotError
    (code HOT_E_TOOBIG) for plans whose workspace does not fit."""
    stream = _stream(stream)
    n = len(ins)
    pin = (ctypes.c_void_p * n)(*[_ptr(t) for t in ins])
    pout = (ctypes.c_void_p * n)(*[_ptr(t) for t in outs])
    rc = _lib().hot_run_noalloc(plan, pin, pout, int(nsteps), _ptr(stats), stream)
    if rc not in (HOT_OK, HOT_E_NOCONVERGE, HOT_E_NONFINITE):
        raise HotError(rc, "hot_run_noalloc", _lib().hot_last_hip_error(plan))
    return rc


def hot_destroy(plan):
    _lib().hot_destroy(plan)
    _KEEP.pop(plan.value, None)


def hot_profile_enable(plan, enable=True):
    rc = _lib().hot_profile_enable(plan, 1 if enable else 0)
    if rc != HOT_OK:
        raise HotError(rc, "hot_profile_enable")


def hot_profile_read(plan, max_passes=32):
    """Returns {pass_name: (total_ms, launches)} for passes that ran."""
    ms = (ctypes.c_double * max_passes)()
    cnt = (ctypes.c_int64 * max_passes)()
    n = _lib().hot_profile_read(plan, max_passes, ms, cnt)
    if n < 0:
        raise HotError(n, "hot_profile_read", _lib().hot_last_hip_error(plan))
    out = {}
    for i in range(min(n, max_passes)):
        if cnt[i]:
            out[_lib().hot_pass_name(i).decode()] = (ms[i], cnt[i])
    return out


def hot_pass_bytes(plan, instance, pass_name):
    lib = _lib()
    for i in range(64):
        name = lib.hot_pass_name(i).decode()
        if not name:
            break
        if name == pass_name:
            b = ctypes.c_double()
            rc = lib.hot_pass_bytes(plan, instance, i, ctypes.byref(b))
            if rc != HOT_OK:
                raise HotError(rc, "hot_pass_bytes")
            return b.value
    raise KeyError(pass_name)


def pass_names():
    lib = _lib()
    names = []
    for i in range(64):
        s = lib.hot_pass_name(i).decode()
        if not s:
            break
        names.append(s)
    return names


def hot_graph_create(plan, ins, outs, workspace, nsteps=0, stream=None, stats=None):
    """Capture the whole operation into a HIP graph; returns a graph handle.
    stream must be a non-default stream (torch.cuda.Stream or hipStream_t);
    stats as for hot_run."""
    stream = _stream(stream)
    n = len(ins)
    pin = (ctypes.c_void_p * n)(*[_ptr(t) for t in ins])
    pout = (ctypes.c_void_p * n)(*[_ptr(t) for t in outs])
    g = ctypes.c_void_p()
    rc = _lib().hot_graph_create(plan, pin, pout, _ptr(workspace), int(nsteps), _ptr(stats), stream,
                                 ctypes.byref(g))
    if rc != HOT_OK:
        raise HotError(rc, "hot_graph_create", _lib().hot_last_hip_error(plan))
    return g


def hot_graph_launch(graph, stream=None):
    rc = _lib().hot_graph_launch(graph, _stream(stream))
    if rc != HOT_OK:
        raise HotError(rc, "hot_graph_launch")


def hot_graph_destroy(graph):
    _lib().hot_graph_destroy(graph)


def hot_tune(plan, workspace, stream=None, reps=3):
    """Autotune the strided column widths of every size in the plan."""
    rc = _lib().hot_tune(plan, _ptr(workspace), _stream(stream), int(reps))
    if rc != HOT_OK:
        raise HotError(rc, "hot_tune", _lib().hot_last_hip_error(plan))


def hot_set_variant(plan, pass_name, variant):
    """Override the autotuner's choice for a pass (see include/hot.h)."""
    _check(_lib().hot_set_variant(plan, pass_names().index(pass_name), int(variant)), "hot_set_variant")


def hot_tuned_width(plan, instance, pass_name):
    lib = _lib()
    idx = pass_names().index(pass_name)
    w = lib.hot_tuned_width(plan, int(instance), idx)
    if w < 0:
        raise HotError(w, "hot_tuned_width")
    return w


def hot_implicit_stats(plan, batch):
    """Per instance of the last implicit call: (sweeps summed over its steps,
    steps that stopped at max_iter), as two lists.  Waits for that call."""
    sw = (ctypes.c_int32 * batch)()
    nc = (ctypes.c_int32 * batch)()
    rc = _lib().hot_implicit_stats(plan, sw, nc)
    if rc not in (HOT_OK, HOT_E_NOCONVERGE):
        raise HotError(rc, "hot_implicit_stats", _lib().hot_last_hip_error(plan))
    return list(sw), list(nc)


STATS_BYTES = 24  # sizeof(hot_stats)


def stats_buffer(batch):
    """A device buffer for batch hot_stats records."""
    import torch
    return torch.zeros(batch * STATS_BYTES, dtype=torch.uint8, device="cuda")


def stats_view(buf):
    """(energy, dissipation, sweeps, nonconv) per instance of a stats buffer
    read back to the host (numpy arrays)."""
    import numpy as np
    raw = buf.cpu().numpy().view(np.uint8)
    rec = np.dtype([("energy", "<f8"), ("dissipation", "<f8"), ("sweeps", "<i4"), ("nonconv", "<i4")])
    r = raw.view(rec)
    return r["energy"].copy(), r["dissipation"].copy(), r["sweeps"].copy(), r["nonconv"].copy()


_KEEP = {}  # plan handle -> packed surrogate tensor the plan points to


def hot_set_surrogate(plan, packed):
    """Warm-start an implicit plan with a packed MLP (device tensor or
    pointer; None for the plain extrapolation).  The plan keeps only the
    pointer, so a tensor passed here is held until the plan is destroyed or
    given another surrogate."""
    rc = _lib().hot_set_surrogate(plan, _ptr(packed))
    if rc != HOT_OK:
        raise HotError(rc, "hot_set_surrogate")
    _KEEP[plan.value] = packed


def hot_mlp_param_count():
    return int(_lib().hot_mlp_param_count())


def hot_mlp_packed_bytes():
    return int(_lib().hot_mlp_packed_bytes())


def hot_mlp_train_bytes(rows):
    return int(_lib().hot_mlp_train_bytes(int(rows)))


def _check(rc, where):
    if rc != HOT_OK:
        raise HotError(rc, where)


def hot_mlp_pack(params, packed, stream=None):
    _check(_lib().hot_mlp_pack(_ptr(params), _ptr(packed), _stream(stream)), "hot_mlp_pack")


def hot_mlp_forward(packed, x, y, rows, stream=None):
    _check(_lib().hot_mlp_forward(_ptr(packed), _ptr(x), _ptr(y), int(rows), _stream(stream)), "hot_mlp_forward")


def hot_mlp_grad(params, x, t, rows, grad, loss, workspace, stream=None):
    _check(_lib().hot_mlp_grad(_ptr(params), _ptr(x), _ptr(t), int(rows), _ptr(grad), _ptr(loss), _ptr(workspace),
                               _stream(stream)), "hot_mlp_grad")


def hot_mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib().hot_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                               float(beta2), float(eps), _stream(stream)), "hot_mlp_adam")


def hot_mlp_dataset_rows(N):
    r = int(_lib().hot_mlp_dataset_rows(int(N)))
    if r < 0:
        raise HotError(r, "hot_mlp_dataset_rows")
    return r


def hot_mlp_dataset(N, dtype, u, d1, d2, d, nu, dt, x, t=None, s=None, stream=None):
    """Training features (targets when d is given, scales when s is given)
    of one field."""
    _check(_lib().hot_mlp_dataset(int(N), DTYPES[dtype], _ptr(u), _ptr(d1), _ptr(d2), _ptr(d), float(nu), float(dt),
                                  _ptr(x), _ptr(t), _ptr(s), _stream(stream)), "hot_mlp_dataset")


def hot_diagnostics(plan, ins, workspace, out, stream=None):
    """Energy and dissipation rate of each instance into the device double
    tensor out[batch][2] (see include/hot.h)."""
    n = len(ins)
    pin = (ctypes.c_void_p * n)(*[_ptr(t) for t in ins])
    rc = _lib().hot_diagnostics(plan, pin, _ptr(workspace), _ptr(out), _stream(stream))
    if rc != HOT_OK:
        raise HotError(rc, "hot_diagnostics", _lib().hot_last_hip_error(plan))


def hot_plan_slab(n, op, nranks, rank, dtype="f64", dealias="two_thirds", nu=0.0, dt=0.0):
    """Plan share `rank` of `nranks` of one N^3 field (op "rhs" or "rk4");
    returns (handle, workspace_bytes)."""
    arr = (ctypes.c_int32 * 1)(int(n))
    d = HotDesc(HOT_ABI_VERSION, 1, arr, float(nu), float(dt), DTYPES[dtype], DEALIAS[dealias], OPS[op], 0, 1e-10, 50,
                0)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    rc = _lib().hot_plan_slab(ctypes.byref(d), int(nranks), int(rank), ctypes.byref(h), ctypes.byref(ws))
    if rc != HOT_OK:
        raise HotError(rc, "hot_plan_slab")
    return h, ws.value


def hot_slab_layout_of(plan):
    """The share's HotSlabLayout (geometry and exchange buffer offsets)."""
    lay = HotSlabLayout()
    _check(_lib().hot_slab_layout_of(plan, ctypes.byref(lay)), "hot_slab_layout_of")
    return lay


def hot_slab_run(plan, phase, workspace, stage=0, inp=None, out=None, stream=None):
    """Enqueue one phase (HOT_SLAB_*) of a share; see include/hot.h."""
    rc = _lib().hot_slab_run(plan, int(phase), int(stage), _ptr(inp), _ptr(out), _ptr(workspace), _stream(stream))
    if rc != HOT_OK:
        raise HotError(rc, "hot_slab_run", _lib().hot_last_hip_error(plan))
