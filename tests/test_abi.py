"""The C-ABI library loads, exports every symbol include/hot.h declares, and
validates its arguments on the host (no GPU calls)."""
import ctypes
import os
import re

import pytest

from paper_1607_00850_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hot.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hot_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("hot_plan", "hot_run", "hot_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = binding.library()
    for s in declared_symbols():
        assert hasattr(lib, s), s
        assert ctypes.cast(getattr(lib, s), ctypes.c_void_p).value


def test_header_compiles_as_c():
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        open(src, "w").write('#include "hot.h"\nint main(void){hot_desc d; (void)d; return 0;}\n')
        r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-c", src,
                            "-o", os.path.join(d, "t.o")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def _expect(code, **kw):
    args = dict(n=64, op="rk4", dtype="f64", dealias="two_thirds", nu=0.01, dt=0.001)
    args.update(kw)
    with pytest.raises(binding.HotError) as e:
        binding.hot_plan(**args)
    assert e.value.code == code


def test_plan_rejects_bad_arguments():
    _expect(binding.HOT_E_INVALID, n=63)         # odd
    _expect(binding.HOT_E_INVALID, n=6)          # below 8
    _expect(binding.HOT_E_INVALID, nu=-1.0)
    _expect(binding.HOT_E_INVALID, nu=float("nan"))
    _expect(binding.HOT_E_INVALID, dt=0.0)
    _expect(binding.HOT_E_INVALID, dt=-1e-3)
    _expect(binding.HOT_E_UNSUPPORTED, n=4096)   # even, but no kernels for it
    _expect(binding.HOT_E_UNSUPPORTED, n=[64, 100])


def test_plan_rejects_bad_descriptor_fields():
    lib = binding.library()
    n = (ctypes.c_int32 * 1)(64)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    good = dict(abi_version=2, batch=1, n=n, nu=0.0, dt=1e-3, dtype=0, dealias=0, op=3, flags=0, tol=1e-6,
                max_iter=10, reserved=0)
    for field, bad in [("abi_version", 1), ("batch", 0), ("dtype", 7), ("dealias", 5), ("op", 9), ("flags", 1),
                       ("flags", 4), ("reserved", 1)]:
        kw = dict(good)
        kw[field] = bad
        d = binding.HotDesc(**kw)
        assert lib.hot_plan(ctypes.byref(d), ctypes.byref(h), ctypes.byref(ws)) == binding.HOT_E_INVALID
        assert not h.value
    assert lib.hot_plan(None, ctypes.byref(h), ctypes.byref(ws)) == binding.HOT_E_INVALID


def test_run_rejects_bad_pointers_without_touching_the_gpu():
    h, wsb = binding.hot_plan(16, "rhs", "f64", nu=0.01)
    lib = binding.library()
    try:
        arr = (ctypes.c_void_p * 1)(256 * 1000)
        nul = (ctypes.c_void_p * 1)(None)
        assert lib.hot_run(h, arr, arr, None, 0, None, None) == binding.HOT_E_WORKSPACE
        assert lib.hot_run(h, arr, arr, ctypes.c_void_p(256 * 7 + 3), 0, None, None) == binding.HOT_E_WORKSPACE
        assert lib.hot_run(h, nul, arr, ctypes.c_void_p(256 * 9), 0, None, None) == binding.HOT_E_INVALID
        mis = (ctypes.c_void_p * 1)(256 * 1000 + 8)
        assert lib.hot_run(h, mis, arr, ctypes.c_void_p(256 * 9), 0, None, None) == binding.HOT_E_INVALID
        assert lib.hot_run(h, arr, arr, ctypes.c_void_p(256 * 9), -1, None, None) == binding.HOT_E_INVALID
        assert lib.hot_run(None, arr, arr, ctypes.c_void_p(256 * 9), 0, None, None) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    assert lib.hot_destroy(None) == 0


def _align(v):
    return (v + 255) // 256 * 256


@pytest.mark.parametrize("dtype,elem", [("f64", 16), ("f32", 8)])
@pytest.mark.parametrize("N", [8, 32, 64, 1024])
def test_workspace_size_formula(N, dtype, elem):
    if N not in (8, 16, 32, 64, 128, 256, 512, 1024):
        pytest.skip("size not built")
    K = (N - 1) // 3
    M, Mz = 2 * K + 1, K + 1
    seg = 128 // elem  # rows padded to whole 128-byte segments once Mz >= 4 segments
    P = -(-Mz // seg) * seg if Mz >= 4 * seg else Mz
    C, D1, D2 = M * M * P, N * M * P, N * N * P
    h, ws = binding.hot_plan(N, "rk4", dtype, nu=0.01, dt=1e-3)
    binding.hot_destroy(h)
    # + the partial sums of the per-instance statistics: 64 blocks x (E, eps) in FP64,
    # + for FP32 the persistent batch kernel's control block and arguments (4096 bytes)
    persist = 4096 if dtype == "f32" else 0
    assert ws == (4 * _align(3 * C * elem) + _align(6 * D1 * elem) + _align(6 * D2 * elem) + _align(64 * 2 * 8)
                  + persist)
    h, ws = binding.hot_plan(N, "r2c", dtype)
    binding.hot_destroy(h)
    assert ws == 2 * _align(3 * N * N * (N // 2 + 1) * elem)


def test_pass_byte_model_rk4_1024_f32():
    h, _ = binding.hot_plan(1024, "rk4", "f32", nu=1 / 1600, dt=1e-3)
    try:
        K = 341
        M, Mz, N = 683, 342, 1024
        C, D1, D2 = M * M * Mz, N * M * Mz, N * N * Mz
        assert binding.hot_pass_bytes(h, 0, "y_inv") == 8.0 * (6 * D1 + 6 * D2)
        assert binding.hot_pass_bytes(h, 0, "z_cross") == 8.0 * (9 * D2)
        assert binding.hot_pass_bytes(h, 0, "x_inv_curl") == 8.0 * (3 * C + 6 * D1)
        assert K == (N - 1) // 3
    finally:
        binding.hot_destroy(h)


def test_error_strings():
    lib = binding.library()
    for code in (0, -1, -2, -3, -4, -99):
        assert lib.hot_error_string(code)


def test_graph_and_tune_reject_bad_arguments_without_the_gpu():
    lib = binding.library()
    h, wsb = binding.hot_plan([16, 24, 16], "rk4", "f32", nu=0.01, dt=1e-3)
    try:
        arr = (ctypes.c_void_p * 3)(256 * 1000, 256 * 2000, 256 * 3000)
        g = ctypes.c_void_p()
        # the legacy default stream cannot be captured
        assert lib.hot_graph_create(h, arr, arr, ctypes.c_void_p(256 * 9), 1, None, None, ctypes.byref(g)) == \
            binding.HOT_E_INVALID
        assert not g.value
        assert lib.hot_tune(h, ctypes.c_void_p(256 * 9), None, 0) == binding.HOT_E_INVALID
        assert lib.hot_tune(h, None, None, 1) == binding.HOT_E_WORKSPACE
        assert lib.hot_graph_launch(None, None) == binding.HOT_E_INVALID
        assert lib.hot_graph_destroy(None) == 0
    finally:
        binding.hot_destroy(h)


def test_batched_workspace_is_the_sum_over_sizes():
    # instances of equal N share one batch-major region; different N add up
    _, w16 = binding.hot_plan([16], "rk4", "f32", nu=0.01, dt=1e-3)
    _, w24 = binding.hot_plan([24], "rk4", "f32", nu=0.01, dt=1e-3)
    _, wb = binding.hot_plan([16, 24, 16, 16], "rk4", "f32", nu=0.01, dt=1e-3)
    # every FP32 RK4 plan holds one persistent-kernel area (4096 bytes) once
    per = 4096
    w16, w24, wb = w16 - per, w24 - per, wb - per
    assert wb >= 3 * w16 + w24 - 4 * 256 * 8 and wb <= 3 * w16 + w24 + 2 * 256 * 8


def test_implicit_plan_validation_and_workspace():
    _expect(binding.HOT_E_INVALID, op="implicit", tol=0.0)
    _expect(binding.HOT_E_INVALID, op="implicit", tol=float("nan"))
    _expect(binding.HOT_E_INVALID, op="implicit", max_iter=0)
    _expect(binding.HOT_E_INVALID, op="implicit", dt=0.0)
    N, elem = 32, 16
    K = (N - 1) // 3
    M, Mz = 2 * K + 1, K + 1
    C, D1, D2 = M * M * Mz, N * M * Mz, N * N * Mz
    h, ws = binding.hot_plan(N, "implicit", "f64", nu=0.01, dt=1e-3, tol=1e-8, max_iter=20)
    binding.hot_destroy(h)
    nparts = -(-C // 256)
    base = 4 * _align(3 * C * elem) + _align(6 * D1 * elem) + _align(6 * D2 * elem) + _align(64 * 2 * 8)
    # + four histories, the flag, the partial sums and the two counters
    assert ws == base + 4 * _align(3 * C * elem) + _align(4) + _align(nparts * 16) + _align(2 * 4)


def test_implicit_stats_and_graph_rules_without_the_gpu():
    lib = binding.library()
    h, _ = binding.hot_plan(16, "rk4", "f64", nu=0.01, dt=1e-3)
    try:
        assert lib.hot_implicit_stats(h, None, None) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan([16, 32], "implicit", "f32", nu=0.01, dt=1e-3, tol=1e-5, max_iter=8)
    try:
        # nothing ran yet: zero sweeps
        assert binding.hot_implicit_stats(h, 2) == ([0, 0], [0, 0])
    finally:
        binding.hot_destroy(h)
    # a kept history continues from the calls before: no graph capture
    h, _ = binding.hot_plan([16, 32], "implicit", "f32", nu=0.01, dt=1e-3, tol=1e-5, max_iter=8, keep_history=True)
    try:
        arr = (ctypes.c_void_p * 2)(256 * 1000, 256 * 2000)
        g = ctypes.c_void_p()
        rc = lib.hot_graph_create(h, arr, arr, ctypes.c_void_p(256 * 9), 1, None, ctypes.c_void_p(256), ctypes.byref(g))
        assert rc == binding.HOT_E_UNSUPPORTED and not g.value
        # statistics only for the ops with a state, and 8-byte aligned
        assert lib.hot_run(h, arr, arr, ctypes.c_void_p(256 * 9), 1, ctypes.c_void_p(256 + 4), None) == \
            binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan(16, "r2c", "f32")
    try:
        arr = (ctypes.c_void_p * 1)(256 * 1000)
        assert lib.hot_run(h, arr, arr, ctypes.c_void_p(256 * 9), 0, ctypes.c_void_p(256), None) == \
            binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    assert lib.hot_error_string(binding.HOT_E_NOCONVERGE) != lib.hot_error_string(-99)


def test_check_finite_flag_rules_without_the_gpu():
    lib = binding.library()
    # allowed on the three time-stepping/right-hand-side ops; costs one 256-byte slot
    for op in ("rhs", "rk4", "implicit"):
        _, w0 = binding.hot_plan([16, 24], op, "f32", nu=0.01, dt=1e-3)
        h, w1 = binding.hot_plan([16, 24], op, "f32", nu=0.01, dt=1e-3, check_finite=True)
        binding.hot_destroy(h)
        assert w1 == w0 + 256
    h, _ = binding.hot_plan(16, "implicit", "f64", nu=0.01, dt=1e-3, keep_history=True, check_finite=True)
    binding.hot_destroy(h)
    _expect(binding.HOT_E_INVALID, op="r2c", check_finite=True)
    _expect(binding.HOT_E_INVALID, op="c2r", check_finite=True)
    # the check synchronises on the host: no graph capture
    h, _ = binding.hot_plan(16, "rk4", "f64", nu=0.01, dt=1e-3, check_finite=True)
    try:
        arr = (ctypes.c_void_p * 1)(256 * 1000)
        g = ctypes.c_void_p()
        rc = lib.hot_graph_create(h, arr, arr, ctypes.c_void_p(256 * 9), 1, None, ctypes.c_void_p(256), ctypes.byref(g))
        assert rc == binding.HOT_E_UNSUPPORTED and not g.value
    finally:
        binding.hot_destroy(h)
    msg = lib.hot_error_string(binding.HOT_E_NONFINITE)
    assert msg and msg != lib.hot_error_string(-99)


def test_mlp_sizes_and_surrogate_rules_without_the_gpu():
    import oracle
    lib = binding.library()
    assert binding.hot_mlp_param_count() == oracle.mlp_param_count()
    # BF16 weights (the output layer padded to 16 rows) and FP32 biases (b4 padded to 16)
    assert binding.hot_mlp_packed_bytes() == 2 * (256 * 32 + 2 * 256 * 256 + 16 * 256) + 4 * (3 * 256 + 16)
    assert binding.hot_mlp_train_bytes(0) == 0
    assert binding.hot_mlp_train_bytes(1000) > 5 * 1000 * 256 * 4
    h, _ = binding.hot_plan(16, "rk4", "f64", nu=0.01, dt=1e-3)
    try:
        assert lib.hot_set_surrogate(h, ctypes.c_void_p(256)) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan(16, "implicit", "f64", nu=0.01, dt=1e-3, keep_history=True)
    try:
        assert lib.hot_set_surrogate(h, ctypes.c_void_p(256 + 8)) == binding.HOT_E_INVALID
        assert lib.hot_set_surrogate(h, ctypes.c_void_p(256)) == binding.HOT_OK
        assert lib.hot_set_surrogate(h, None) == binding.HOT_OK
    finally:
        binding.hot_destroy(h)
    _expect(binding.HOT_E_INVALID, op="rk4", keep_history=True)
    assert lib.hot_mlp_forward(None, None, None, 1, None) == binding.HOT_E_INVALID
    assert lib.hot_mlp_adam(None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-8, None) == binding.HOT_E_INVALID


def test_set_variant_rules_without_the_gpu():
    lib = binding.library()
    names = binding.pass_names()
    h, _ = binding.hot_plan(32, "rk4", "f32", nu=0.01, dt=1e-3)
    try:
        for v in (-1, 0, 1, 2):
            binding.hot_set_variant(h, "x_fwd_rk", v)
            assert (binding.hot_tuned_width(h, 0, "x_fwd_rk") == 0) == (v < 0)
        assert lib.hot_set_variant(h, names.index("x_fwd_rk"), 3) == binding.HOT_E_INVALID
        assert lib.hot_set_variant(h, names.index("y_inv"), 3) == binding.HOT_E_INVALID
        assert lib.hot_set_variant(h, names.index("z_cross"), 4) == binding.HOT_E_INVALID
        assert binding.hot_tuned_width(h, 0, "z_cross") == 1  # packed pair rows by default
        binding.hot_set_variant(h, "z_cross", 0)
        assert binding.hot_tuned_width(h, 0, "z_cross") == 0
        binding.hot_set_variant(h, "z_cross", 1)
        binding.hot_set_variant(h, "y_inv", 0)
        binding.hot_set_variant(h, "x_fwd_rk", -1)
        assert binding.hot_tuned_width(h, 0, "x_fwd_rk") == 0
        binding.hot_set_variant(h, "x_fwd_rk", 1)
        assert binding.hot_tuned_width(h, 0, "x_fwd_rk") == binding.hot_tuned_width(h, 0, "x_fwd") > 0
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan(32, "implicit", "f32", nu=0.01, dt=1e-3)
    try:
        assert lib.hot_set_variant(h, names.index("x_fwd_rk"), 0) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)


def test_implicit_flag_check_rules_without_the_gpu():
    lib = binding.library()
    names = binding.pass_names()
    h, _ = binding.hot_plan(16, "implicit", "f32", nu=0.01, dt=1e-3)
    try:
        assert binding.hot_tuned_width(h, 0, "imp_decide") == 2  # default: look every 2 sweeps
        for k in (0, 1, 7):
            binding.hot_set_variant(h, "imp_decide", k)
            assert binding.hot_tuned_width(h, 0, "imp_decide") == k
        assert lib.hot_set_variant(h, names.index("imp_decide"), -1) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan(16, "rk4", "f32", nu=0.01, dt=1e-3)
    try:
        assert lib.hot_set_variant(h, names.index("imp_decide"), 2) == binding.HOT_E_INVALID
        assert lib.hot_tuned_width(h, 0, names.index("imp_decide")) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)


def test_fused_yz_variant_rules_without_the_gpu():
    lib = binding.library()
    names = binding.pass_names()
    yz = names.index("yz_fused")
    assert names[-5:] == ["yz_fused", "tables", "stats", "graph", "persistent"]
    # the fused y-z pass exists for small N only: a batch switches the sizes that have it
    h, _ = binding.hot_plan([16, 64, 128, 1024], "rk4", "f32", nu=0.01, dt=1e-3)
    try:
        assert [binding.hot_tuned_width(h, i, "yz_fused") for i in range(4)] == [0, 0, 0, 0]
        binding.hot_set_variant(h, "yz_fused", 0)
        assert [binding.hot_tuned_width(h, i, "yz_fused") for i in range(4)] == [1, 1, 0, 0]
        binding.hot_set_variant(h, "yz_fused", -1)
        assert binding.hot_tuned_width(h, 0, "yz_fused") == 0
        assert lib.hot_set_variant(h, yz, 1) == binding.HOT_E_INVALID
        assert lib.hot_set_variant(h, yz, -2) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    # FP64: the six planes of N = 64 do not fit in LDS, those of N = 48 do
    h, _ = binding.hot_plan([48, 64], "implicit", "f64", nu=0.01, dt=1e-3)
    try:
        binding.hot_set_variant(h, "yz_fused", 0)
        assert [binding.hot_tuned_width(h, i, "yz_fused") for i in range(2)] == [1, 0]
    finally:
        binding.hot_destroy(h)
    for op in ("r2c", "c2r"):
        h, _ = binding.hot_plan(32, op, "f32")
        try:
            assert lib.hot_set_variant(h, yz, 0) == binding.HOT_E_INVALID
        finally:
            binding.hot_destroy(h)
    h, _ = binding.hot_plan_slab(32, "rk4", 2, 0, "f32", nu=0.01, dt=1e-3)
    try:
        assert lib.hot_set_variant(h, yz, 0) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan(64, "rk4", "f32", nu=0.01, dt=1e-3)
    try:
        K = 21
        M, Mz = 2 * K + 1, K + 1
        assert binding.hot_pass_bytes(h, 0, "yz_fused") == 9 * 64 * M * Mz * 8
    finally:
        binding.hot_destroy(h)


def test_diagnostics_argument_checks_without_the_gpu():
    lib = binding.library()
    h, _ = binding.hot_plan(16, "rk4", "f64", nu=0.01, dt=1e-3)
    try:
        arr = (ctypes.c_void_p * 1)(256 * 1000)
        assert lib.hot_diagnostics(h, arr, ctypes.c_void_p(256), None, None) == binding.HOT_E_INVALID
        assert lib.hot_diagnostics(h, arr, None, ctypes.c_void_p(256), None) == binding.HOT_E_WORKSPACE
        assert lib.hot_diagnostics(h, arr, ctypes.c_void_p(256 + 8), ctypes.c_void_p(256), None) == \
            binding.HOT_E_WORKSPACE
        nul = (ctypes.c_void_p * 1)(None)
        assert lib.hot_diagnostics(h, nul, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == binding.HOT_E_INVALID
        assert lib.hot_diagnostics(None, arr, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == \
            binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)


def _slab_expect(code, **kw):
    args = dict(n=64, op="rk4", nranks=4, rank=0, dtype="f64", nu=0.01, dt=1e-3)
    args.update(kw)
    with pytest.raises(binding.HotError) as e:
        binding.hot_plan_slab(**args)
    assert e.value.code == code


def test_slab_share_geometry_and_workspace():
    # N = 64, 2/3 rule: Mz = 22 retained kz in chunks of 6 over 4 shares
    N, R, e = 64, 4, 16
    lays, wss = [], []
    for r in range(R):
        h, ws = binding.hot_plan_slab(N, "rk4", R, r, "f64", nu=0.01, dt=1e-3)
        lays.append(binding.hot_slab_layout_of(h))
        wss.append(ws)
        binding.hot_destroy(h)
    assert [(l.kz0, l.mz, l.nkz) for l in lays] == [(0, 6, 6), (6, 6, 6), (12, 6, 6), (18, 4, 33 - 18)]
    for r, l in enumerate(lays):
        assert (l.nranks, l.rank, l.nx, l.chunk, l.pitch) == (R, r, N // R, 6, 6)
        assert l.block_bytes == (N // R) * N * 6 * e and l.comp_bytes == R * l.block_bytes
        assert l.send_offset % 256 == 0 and l.recv_offset % 256 == 0
        assert l.recv_offset >= l.send_offset + 6 * l.comp_bytes
    # compact state of a share: M x M x pitch per component
    K = (N - 1) // 3
    M, C = 2 * K + 1, (2 * K + 1) ** 2 * 6
    D1, D2 = N * M * 6, N * N * 6
    assert wss[0] == 4 * _align(3 * C * e) + _align(6 * D1 * e) + 2 * _align(6 * D2 * e) + _align(64 * 2 * 8)
    # 128-byte pitch once chunks are long enough: N = 1024 FP32 over 4 shares
    h, _ = binding.hot_plan_slab(1024, "rk4", 4, 3, "f32", nu=0.01, dt=1e-3)
    l = binding.hot_slab_layout_of(h)
    binding.hot_destroy(h)
    assert (l.chunk, l.pitch, l.kz0, l.mz, l.nkz) == (86, 96, 258, 342 - 258, 513 - 258)


def test_slab_pass_bytes():
    h, _ = binding.hot_plan_slab(64, "rk4", 4, 1, "f32", nu=0.01, dt=1e-3)
    try:
        assert binding.hot_pass_bytes(h, 0, "z_cross") == 9 * 16 * 64 * 22 * 8
        assert binding.hot_pass_bytes(h, 0, "scatter") == (3 * 43 * 43 * 6 + 3 * 64 * 64 * 6) * 8
    finally:
        binding.hot_destroy(h)


def test_slab_plan_and_run_rules_without_the_gpu():
    lib = binding.library()
    _slab_expect(binding.HOT_E_UNSUPPORTED, nranks=5)     # 64 % 5 != 0
    _slab_expect(binding.HOT_E_UNSUPPORTED, nranks=32)    # chunk 1: shares beyond kz 21 hold nothing
    _slab_expect(binding.HOT_E_INVALID, rank=4)
    _slab_expect(binding.HOT_E_INVALID, rank=-1)
    _slab_expect(binding.HOT_E_INVALID, nranks=0)
    _slab_expect(binding.HOT_E_INVALID, op="implicit")
    _slab_expect(binding.HOT_E_INVALID, op="r2c")
    h, _ = binding.hot_plan_slab(64, "rk4", 2, 0, "f64", nu=0.01, dt=1e-3)
    try:
        arr = (ctypes.c_void_p * 1)(256 * 1000)
        ws = ctypes.c_void_p(256 * 9)
        assert lib.hot_run(h, arr, arr, ws, 1, None, None) == binding.HOT_E_UNSUPPORTED
        g = ctypes.c_void_p()
        assert lib.hot_graph_create(h, arr, arr, ws, 1, None, ctypes.c_void_p(256), ctypes.byref(g)) == \
            binding.HOT_E_UNSUPPORTED
        assert lib.hot_diagnostics(h, arr, ws, ctypes.c_void_p(256), None) == binding.HOT_E_UNSUPPORTED
        run = lib.hot_slab_run
        assert run(h, 7, 0, None, None, ws, None) == binding.HOT_E_INVALID
        assert run(h, binding.HOT_SLAB_INVERSE, 4, None, None, ws, None) == binding.HOT_E_INVALID
        assert run(h, binding.HOT_SLAB_FORWARD, -1, None, None, ws, None) == binding.HOT_E_INVALID
        assert run(h, binding.HOT_SLAB_GATHER, 0, None, None, ws, None) == binding.HOT_E_INVALID
        assert run(h, binding.HOT_SLAB_SCATTER, 0, None, ctypes.c_void_p(257), ws, None) == binding.HOT_E_INVALID
        assert run(h, binding.HOT_SLAB_CROSS, 0, None, None, ctypes.c_void_p(257), None) == binding.HOT_E_WORKSPACE
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan_slab(64, "rhs", 2, 1, "f64", nu=0.01)
    try:
        assert lib.hot_slab_run(h, binding.HOT_SLAB_INVERSE, 0, None, None, ctypes.c_void_p(256), None) == \
            binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    # a plain plan has no slab layout
    h, _ = binding.hot_plan(32, "rk4", "f64", nu=0.01, dt=1e-3)
    try:
        lay = binding.HotSlabLayout()
        assert lib.hot_slab_layout_of(h, ctypes.byref(lay)) == binding.HOT_E_INVALID
        assert lib.hot_slab_run(h, 0, 0, None, None, ctypes.c_void_p(256), None) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)


def test_persistent_schedule_rules_without_the_gpu():
    """The persistent batch kernel (graph variant 2) takes FP32 RK4 plans with
    the 2/3 rule whose sizes all have its bodies (N <= 64 of the batch sizes),
    at most eight sizes; everything else is refused on the host."""
    lib = binding.library()
    names = binding.pass_names()
    graph = names.index("graph")
    ok = [([16, 18, 24, 32, 36, 48, 54, 64], "rk4", "f32", "two_thirds"), ([32], "rk4", "f32", "two_thirds")]
    bad = [([16, 128], "rk4", "f32", "two_thirds"), ([16, 8], "rk4", "f32", "two_thirds"),
           ([16, 32], "rk4", "f64", "two_thirds"), ([16, 32], "rhs", "f32", "two_thirds"),
           ([16, 32], "implicit", "f32", "two_thirds"), ([16, 32], "rk4", "f32", "none")]
    for n, op, dt, de in ok + bad:
        h, _ = binding.hot_plan(n, op, dt, de, nu=0.01, dt=1e-3)
        try:
            rc = lib.hot_set_variant(h, graph, 2)
            if (n, op, dt, de) in ok:
                assert rc == binding.HOT_OK
                assert binding.hot_tuned_width(h, 0, "graph") == 2
                binding.hot_set_variant(h, "graph", 1)
                assert binding.hot_tuned_width(h, 0, "graph") == 1
            else:
                assert rc == binding.HOT_E_INVALID, (n, op, dt, de)
                assert binding.hot_tuned_width(h, 0, "graph") == 1
        finally:
            binding.hot_destroy(h)
    assert lib.hot_set_variant(None, graph, 2) == binding.HOT_E_INVALID
    # the bound of the persistent kernel's waits: plans of schedule 2 only, >= 0
    pers = names.index("persistent")
    h, _ = binding.hot_plan([16, 32], "rk4", "f32", nu=0.01, dt=1e-3)
    try:
        assert binding.hot_tuned_width(h, 0, "persistent") == 0
        binding.hot_set_variant(h, "persistent", 5)
        assert binding.hot_tuned_width(h, 0, "persistent") == 5
        assert lib.hot_set_variant(h, pers, -1) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
    h, _ = binding.hot_plan([16, 32], "rk4", "f64", nu=0.01, dt=1e-3)
    try:
        assert lib.hot_set_variant(h, pers, 1) == binding.HOT_E_INVALID
    finally:
        binding.hot_destroy(h)
