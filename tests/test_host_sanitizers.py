"""The host side of libhot (planning, workspace layout, argument checks,
variants, error paths) under AddressSanitizer and UndefinedBehaviorSanitizer.

hot.hip, mlp.hip and persist.hip are compiled again with the sanitizers on
their host pass only (device code is built as usual), linked with the kernel objects of
the last in-tree build, and tests/test_abi.py runs against that library in a
child process with the ASan runtime preloaded.  Any report fails the test:
UBSan does not recover, ASan halts on the first error.  Leak detection is off
(the Python interpreter itself does not free everything at exit).  No GPU is
needed: test_abi makes no compute calls.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1607_00850_amd import build  # noqa: E402

SAN_FLAGS = ["-O1", "-g",
             "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]
HOST_UNITS = ("hot.hip", "mlp.hip", "persist.hip")


def _asan_runtime():
    r = subprocess.run([build.hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def _kernel_objects():
    """The kernel objects of the in-tree build, rebuilt where older than a
    source they include."""
    units = [u for u in build._units() if os.path.basename(u) not in HOST_UNITS]
    newest = max(os.path.getmtime(os.path.join(build.CSRC, f)) for f in os.listdir(build.CSRC))
    objs = []
    for u in units:
        obj = os.path.join(build.BUILD, os.path.basename(u).replace(".hip", ".o"))
        if not os.path.exists(obj) or os.path.getmtime(obj) < max(newest, os.path.getmtime(u)):
            obj = build._compile(u, [], False)
        objs.append(obj)
    return objs


@pytest.fixture(scope="module")
def sanitized_library(tmp_path_factory):
    try:
        build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc is not available")
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("the compiler's ASan runtime is not available")
    out = tmp_path_factory.mktemp("san")
    objs = []
    for name in HOST_UNITS:
        obj = str(out / name.replace(".hip", ".o"))
        cmd = [build.hipcc(), *build.HIPCC_FLAGS, *SAN_FLAGS, "-c", "-o", obj, os.path.join(build.CSRC, name)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
        objs.append(obj)
    lib = str(out / "libhot_san.so")
    r = subprocess.run([build.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs, *_kernel_objects()],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return lib, rt


def test_library_is_instrumented(sanitized_library):
    lib, _ = sanitized_library
    r = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True)
    assert r.returncode == 0
    assert "__asan_report_load8" in r.stdout and "__ubsan_handle_" in r.stdout


def test_abi_suite_is_clean_under_asan_and_ubsan(sanitized_library):
    lib, rt = sanitized_library
    env = dict(os.environ, HOT_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q", "-x",
                        "-p", "no:cacheprovider", "-m", "not gpu"],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
