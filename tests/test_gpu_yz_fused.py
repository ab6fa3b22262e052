"""The fused y-z pass for small N (k_yz_fused) against the separate y_inv,
z_cross and y_fwd passes and against the oracle.

The fused kernel runs the same transforms with the same plans and twiddles
as the three separate passes, only with the (x, y, kz) intermediate in LDS.
The compiler may contract multiplies and adds into FMAs differently in the
two kernels, so the results agree to rounding, not bit for bit: the relative
L2 difference stays within 50 eps of the element type (a few ulps per value;
one transform pass is about log2(N^3) roundings).  Checked for right-hand
sides at every size that has the kernel (FP32 up to N = 64, FP64 up to
N = 48), RK4 steps, a batch of uneven sizes, the implicit step (its stopping
flags reach the fused kernel too) and dealias "none"; each also against the
oracle with the single-field parity tolerances.
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import inputs
from hotrun import fp32_tol, rel_l2, round32, run, run_implicit

pytestmark = pytest.mark.gpu

NU = 1.0 / 1600.0
DT = 1e-3
FUSED = {"yz_fused": 0}
SEPARATE = {"yz_fused": -1}
SIZES_F32 = [8, 16, 18, 24, 32, 36, 48, 54, 64]
SIZES_F64 = [8, 16, 18, 24, 32, 36, 48]


def close(a, b, dtype, dealias="two_thirds"):
    """Agreement to rounding: relative L2 within 50 eps of the type, and
    exact zeros outside the retained set in both.  (Inside it a value that
    cancels to exactly 0 in one path may come out a few ulps from 0 in the
    other.)"""
    eps = float(np.finfo(np.float32 if dtype == "f32" else np.float64).eps)
    out = ~oracle.retained_mask(a.shape[1], dealias)
    return rel_l2(a, b) < 50 * eps and np.all(a[:, out] == 0) and np.all(b[:, out] == 0)


@pytest.mark.parametrize("dtype,N", [("f32", n) for n in SIZES_F32] + [("f64", n) for n in SIZES_F64])
def test_rhs_fused_equals_separate_and_matches_oracle(dtype, N):
    print(f"yz rhs N={N} {dtype}", flush=True)
    u = inputs.rough_random(N, 70 + N)
    (fused,) = run("rhs", [u], dtype, nu=NU, variants=FUSED)
    (sep,) = run("rhs", [u], dtype, nu=NU, variants=SEPARATE)
    assert close(fused, sep, dtype)
    ref = oracle.rhs(round32(u) if dtype == "f32" else u, NU)
    assert rel_l2(fused, ref) < (1e-12 if dtype == "f64" else fp32_tol(N))


@pytest.mark.parametrize("dtype,N", [("f32", 64), ("f32", 54), ("f64", 48)])
def test_rk4_fused_equals_separate(dtype, N):
    u = inputs.smooth_random(N, 5)
    (fused,) = run("rk4", [u], dtype, nu=NU, dt=DT, nsteps=2, variants=FUSED)
    (sep,) = run("rk4", [u], dtype, nu=NU, dt=DT, nsteps=2, variants=SEPARATE)
    assert close(fused, sep, dtype)
    ref = oracle.rk4(round32(u) if dtype == "f32" else u, NU, DT, 2)
    assert rel_l2(fused, ref) < (1e-12 if dtype == "f64" else fp32_tol(N))


def test_batch_fused_equals_separate():
    fields = [inputs.rough_random(n, 100 + i) for i, n in enumerate([16, 64, 24, 128, 64, 36, 18])]
    fused = run("rk4", fields, "f32", nu=NU, dt=DT, nsteps=1, variants=FUSED)
    sep = run("rk4", fields, "f32", nu=NU, dt=DT, nsteps=1, variants=SEPARATE)
    for a, b in zip(fused, sep):
        assert close(a, b, "f32")


def test_implicit_fused_equals_separate():
    fields = [inputs.smooth_random(n, 200 + n) for n in (32, 48, 64)]
    kw = dict(dtype="f32", nu=0.01, dt=1e-2, nsteps=2, tol=1e-5, max_iter=20)
    out_f, sw_f, nc_f, rc_f = run_implicit(fields, variants=FUSED, **kw)
    out_s, sw_s, nc_s, rc_s = run_implicit(fields, variants=SEPARATE, **kw)
    assert (sw_f, nc_f, rc_f) == (sw_s, nc_s, rc_s)
    for a, b in zip(out_f, out_s):
        assert close(a, b, "f32")


def test_dealias_none_fused_equals_separate():
    N = 32
    u = inputs.rough_random(N, 9, dealias="none")
    (fused,) = run("rhs", [u], "f32", dealias="none", nu=0.01, variants=FUSED)
    (sep,) = run("rhs", [u], "f32", dealias="none", nu=0.01, variants=SEPARATE)
    assert close(fused, sep, "f32", "none")
    assert rel_l2(fused, oracle.rhs(round32(u), 0.01, dealias="none")) < fp32_tol(N)
