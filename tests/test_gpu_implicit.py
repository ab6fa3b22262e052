"""GPU parity of the implicit-midpoint step (Picard sweeps) against the
oracle, through the C ABI.

Bars:
  * FP64: the state agrees with the oracle's to 1e-12 of the state plus
    10 tol of the increment (both stop once the sweep update is within tol of
    the increment, so their fixed-point iterates can differ by that much),
    and the number of sweeps per step is the same.
  * FP32 (tol 1e-5): the state to the FP32 bar of the RK4 tests, 10 eps32
    log2(N^3), against the oracle on the FP32-rounded input; the increment
    to 20 tol plus the FP32 rounding of the state seen relative to it.
  * Beltrami fields, whose nonlinear term vanishes: the exact
    Crank-Nicolson factor (1 - a)/(1 + a) and exactly two sweeps per step.
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import fp32_tol, rel_l2, round32, run_implicit

pytestmark = pytest.mark.gpu

NU = 1.0 / 1600.0


def _state_err(got, ref, u0):
    """||got - ref|| relative to the state and to the increment."""
    return np.linalg.norm(got - ref), np.linalg.norm(ref), np.linalg.norm(ref - u0)


@pytest.mark.parametrize("N,kind", [(16, "rough"), (32, "smooth"), (24, "rough")])
def test_one_step_fp64_matches_oracle(N, kind):
    print(f"implicit 1 step N={N} {kind}", flush=True)
    u0 = (inputs.rough_random(N, N) if kind == "rough" else inputs.smooth_random(N, N)) * 4.0
    dt, tol = 0.02, 1e-10
    (got,), sw, nc, rc = run_implicit([u0], "f64", NU, dt, 1, tol)
    ref, s_ref, ok, _ = oracle.implicit_midpoint_step(u0, NU, dt, tol)
    assert ok and rc == binding.HOT_OK and nc == [0]
    err, nu_, ninc = _state_err(got, ref, u0)
    assert err <= 1e-12 * nu_ + 10 * tol * ninc
    assert sw == [s_ref]
    M = oracle.retained_mask(N)
    assert np.all(got[:, ~M] == 0)


@pytest.mark.parametrize("nsteps", [4, 7])
def test_several_steps_fp64_use_the_extrapolation_predictor(nsteps):
    # 7 steps: every predictor depth (0 to 4 increments) and the rotation of
    # the five buffers past one full turn
    N, dt, tol = 24, 0.02, 1e-10
    u0 = inputs.smooth_random(N, 3) * 4.0
    (got,), sw, nc, rc = run_implicit([u0], "f64", NU, dt, nsteps, tol)
    ref, s_ref, incs, _ = oracle.implicit_midpoint(u0, NU, dt, nsteps, tol)
    err, nu_, _ = _state_err(got, ref, u0)
    assert err <= 1e-12 * nu_ + 10 * tol * sum(np.linalg.norm(d) for d in incs)
    assert sw == [sum(s_ref)] and nc == [0] and rc == binding.HOT_OK


@pytest.mark.parametrize("N", [16, 32, 64])
def test_fp32_matches_oracle(N):
    print(f"implicit fp32 N={N}", flush=True)
    u0 = inputs.rough_random(N, 2 * N)
    dt, tol = 0.01, 1e-5
    (got,), sw, nc, rc = run_implicit([u0], "f32", NU, dt, 2, tol)
    x = round32(u0)
    ref, _, incs, _ = oracle.implicit_midpoint(x, NU, dt, 2, 1e-12)
    assert rc == binding.HOT_OK and nc == [0]
    assert rel_l2(got, ref) < fp32_tol(N)
    inc_got, inc_ref = got - x, ref - x
    eps32 = float(np.finfo(np.float32).eps)
    bar = 20 * tol + 10 * eps32 * np.linalg.norm(ref) / np.linalg.norm(inc_ref)
    assert np.linalg.norm(inc_got - inc_ref) <= bar * np.linalg.norm(inc_ref)


@pytest.mark.parametrize("dtype,N", [("f64", 32), ("f32", 64)])
def test_beltrami_crank_nicolson_factor(dtype, N):
    K2, nu, dt, n = 9, 0.05, 0.1, 3
    u0 = inputs.beltrami(N, K2, seed=5)
    (got,), sw, nc, rc = run_implicit([u0], dtype, nu, dt, n, 1e-5 if dtype == "f32" else 1e-12)
    a = 0.5 * dt * nu * K2
    x = round32(u0) if dtype == "f32" else u0
    bar = fp32_tol(N) if dtype == "f32" else 1e-13
    assert rel_l2(got, ((1 - a) / (1 + a)) ** n * x) < bar
    assert sw == [2 * n] and nc == [0] and rc == binding.HOT_OK


def test_uneven_batch_matches_single_instances():
    dt, tol = 0.02, 1e-10
    fields = [inputs.rough_random(16, 1) * 4, inputs.smooth_random(24, 2) * 4, inputs.rough_random(32, 3),
              inputs.smooth_random(16, 4) * 0.5]
    outs, sw, nc, rc = run_implicit(fields, "f64", NU, dt, 3, tol)
    assert rc == binding.HOT_OK and nc == [0] * 4
    for f, g, s in zip(fields, outs, sw):
        ref, s_ref, incs, _ = oracle.implicit_midpoint(f, NU, dt, 3, tol)
        err, nu_, _ = _state_err(g, ref, f)
        assert err <= 1e-12 * nu_ + 10 * tol * sum(np.linalg.norm(d) for d in incs)
        assert s == sum(s_ref)
    # instances stop on their own: the weak field takes fewer sweeps
    assert len(set(sw)) > 1


@pytest.mark.parametrize("check", [0, 1, 2, 5])
def test_flag_checks_change_nothing_but_the_launches(check):
    # sweeps go out in rounds of `check` between the host's looks at the
    # stopping flags (0: never look): results and sweep counts are the same
    # bit for bit, with uneven sizes on their own graph branches or streams,
    # and with a cap (max_iter 4) that some steps reach
    dt = 0.02
    fields = [inputs.rough_random(16, 11) * 4, inputs.smooth_random(24, 12) * 4, inputs.rough_random(32, 13),
              inputs.smooth_random(16, 14) * 0.5, inputs.rough_random(24, 15) * 8]
    for tol, max_iter in ((1e-10, 50), (1e-13, 4)):
        ref, sw_ref, nc_ref, rc_ref = run_implicit(fields, "f64", NU, dt, 3, tol, max_iter,
                                                   variants={"imp_decide": 3})
        got, sw, nc, rc = run_implicit(fields, "f64", NU, dt, 3, tol, max_iter, variants={"imp_decide": check})
        assert (sw, nc, rc) == (sw_ref, nc_ref, rc_ref)
        for a, b in zip(got, ref):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    assert any(nc_ref)  # the capped run did stop some steps at max_iter


def test_max_iter_stop_reports_and_keeps_the_last_iterate():
    N, dt = 16, 0.05
    u0 = inputs.rough_random(N, 6) * 4.0
    (got,), sw, nc, rc = run_implicit([u0], "f64", NU, dt, 2, 1e-14, 1)
    assert rc == binding.HOT_E_NOCONVERGE and nc == [2] and sw == [2]
    # the oracle with the same cap: one sweep per step from the same predictors
    u, hist = u0 * oracle.retained_mask(N), []
    for _ in range(2):
        pred = oracle.extrapolation_predictor(u, hist[-2:])
        u1, s, ok, _ = oracle.implicit_midpoint_step(u, NU, dt, 1e-14, 1, pred)
        assert s == 1 and not ok
        hist.append(u1 - u)
        u = u1
    assert rel_l2(got, u) < 1e-12


def test_in_place_and_zero_steps():
    N = 16
    u0 = inputs.rough_random(N, 8, dealias="none")
    (same,), sw, _, _ = run_implicit([u0], "f64", NU, 0.01, 0)
    np.testing.assert_array_equal(same, u0 * oracle.retained_mask(N))
    assert sw == [0]
    (got,), _, _, _ = run_implicit([u0], "f64", NU, 0.01, 2, 1e-10, inplace=True)
    ref, _, _, _ = oracle.implicit_midpoint(u0, NU, 0.01, 2, 1e-10)
    assert rel_l2(got, ref) < 1e-9
