"""Build libhot.so (gfx950) in-tree with hipcc.

    python -m paper_1607_00850_amd.build

The kernels of each (element type, N) live in their own translation unit,
generated into _build/ and compiled in parallel; hot.hip holds the host side
and the C ABI.  Always rebuilds.
"""
import concurrent.futures
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhot.so")

HIPCC_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; libhot needs ROCm to build")
    return exe


def sizes():
    """The N list of HOT_SIZES in csrc/impl.hpp."""
    text = open(os.path.join(CSRC, "impl.hpp")).read()
    m = re.search(r"#define HOT_SIZES\(X\)((?: X\(\d+\))+)", text)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _units():
    os.makedirs(BUILD, exist_ok=True)
    units = [os.path.join(CSRC, "hot.hip"), os.path.join(CSRC, "mlp.hip"), os.path.join(CSRC, "persist.hip")]
    for t, ty in (("f32", "float"), ("f64", "double")):
        for n in sizes():
            path = os.path.join(BUILD, f"ops_{t}_{n}.hip")
            src = (f'#include "../csrc/impl.hpp"\n'
                   f"namespace hot {{\nOps make_ops_{t}_{n}() {{ return Impl<{ty}, {n}>::ops(); }}\n}}\n")
            if not os.path.exists(path) or open(path).read() != src:
                open(path, "w").write(src)
            units.append(path)
    return units


def _compile(src, extra, verbose):
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}{r.stderr}")
    return obj


def build_library(verbose=False, extra_flags=(), out=LIB, jobs=None):
    """Compile every translation unit and link libhot.so next to this file."""
    units = _units()
    jobs = jobs or min(16, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra_flags), verbose), units))
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"link failed with exit code {r.returncode}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
