"""How fast the Picard sweeps of the implicit-midpoint oracle converge, what
a warm start must achieve to save one sweep, and that the three-increment
(quadratic) extrapolation achieves it (CPU, oracle only).

Setting of the implicit batch: R1 fields, Re = 1600 (nu = 1/1600, Sec. 4),
dt = 1e-2, two steps of history, then the step under study.  The reference
increment comes from the oracle's step converged to 1e-14; e_k is the error
of the k-th iterate relative to the increment (e_0: the extrapolation
2 D1 - D2), in the norm of the stopping test.  The sweep map contracts by
rho_k = e_{k+1} / e_k, a few hundredths here, so the stopping test
||d_k - d_{k-1}|| <= tau ||d_k|| passes at the first sweep k with
e_{k-1} <~ tau: with e_0 ~ 1e-3 and tau = 1e-5 that is the third sweep.
Stopping at the second sweep instead needs e_1 = rho_0 e_0 <= tau, i.e. a
predictor whose error is at most tau / (rho_0 e_0) of the extrapolation's.
"""
import numpy as np
import pytest

import oracle
from oracle.implicit_midpoint import extrapolation_predictor, half_norm, midpoint_sweep
from paper_1607_00850_amd import inputs

NU, DT, TAU = 1.0 / 1600.0, 1e-2, 1e-5


def _errors(N, seed, sweeps=5):
    u0 = inputs.smooth_random(N, seed)
    u, _, incs, _ = oracle.implicit_midpoint(u0, NU, DT, 2, 1e-13)
    pred = extrapolation_predictor(u, incs)
    ref, _, ok, _ = oracle.implicit_midpoint_step(u, NU, DT, 1e-14, 80, pred)
    assert ok
    inc = half_norm(ref - u)
    w = pred * oracle.retained_mask(N)
    errs = [half_norm(w - ref) / inc]
    for _ in range(sweeps):
        w, _ = midpoint_sweep(u, w, NU, DT)
        errs.append(half_norm(w - ref) / inc)
    return np.array(errs)


@pytest.mark.parametrize("N,seed", [(32, 20002), (64, 20000)])
def test_sweeps_contract_and_the_gain_one_sweep_needs(N, seed):
    e = _errors(N, seed)
    rho = e[1:] / e[:-1]
    # the extrapolation is good to about 1e-3 of the increment
    assert 3e-4 < e[0] < 3e-3
    # the sweeps contract by a few hundredths each (well below 1: the
    # nonlinear term over dt is small against the increment)
    assert np.all(rho < 0.1)
    # three sweeps at tau = 1e-5: the change of sweep k is about e_{k-1}
    stop = 1 + int(np.argmax(e <= TAU))
    assert stop == 3
    # what a warm start must reach to stop after two sweeps
    need = TAU / (rho[0] * e[0])
    print(f"N={N}: e_0 = {e[0]:.2e}, rho = {np.round(rho, 3)}, "
          f"a warm start saves a sweep only with error <= {need:.2f} of the extrapolation's", flush=True)
    assert 0.2 < need < 0.6


@pytest.mark.parametrize("N,seed", [(32, 20002), (64, 20000)])
def test_three_increment_predictor_saves_a_sweep(N, seed):
    """With three steps of history the plain predictor is the quadratic
    extrapolation 3 D1 - 3 D2 + D3: its error is about a fifteenth of the
    linear one's, well inside the bound above, and the sweeps stop at the
    second instead of the third."""
    u0 = inputs.smooth_random(N, seed)
    u, _, incs, _ = oracle.implicit_midpoint(u0, NU, DT, 3, 1e-13)
    lin = u + 2.0 * incs[-1] - incs[-2]
    ref, _, ok, _ = oracle.implicit_midpoint_step(u, NU, DT, 1e-14, 80, lin)
    assert ok
    inc = half_norm(ref - u)
    m = oracle.retained_mask(N)
    errs = {}
    for name, pred in (("linear", lin), ("quadratic", extrapolation_predictor(u, incs))):
        w = pred * m
        e = [half_norm(w - ref) / inc]
        for _ in range(3):
            w, _ = midpoint_sweep(u, w, NU, DT)
            e.append(half_norm(w - ref) / inc)
        errs[name] = np.array(e)
    ratio = errs["quadratic"][0] / errs["linear"][0]
    print(f"N={N}: e_0 linear {errs['linear'][0]:.2e}, quadratic {errs['quadratic'][0]:.2e} (ratio {ratio:.3f})",
          flush=True)
    assert ratio < 0.2
    assert 1 + int(np.argmax(errs["linear"] <= TAU)) == 3
    assert 1 + int(np.argmax(errs["quadratic"] <= TAU)) == 2
    # the oracle's own step from that predictor stops there too
    _, sweeps, ok, _ = oracle.implicit_midpoint_step(u, NU, DT, TAU, 20, extrapolation_predictor(u, incs))
    assert ok and sweeps == 2


@pytest.mark.parametrize("N,seed", [(32, 20002), (64, 20000)])
def test_four_increment_predictor_meets_tau_at_once(N, seed):
    """With four steps of history the plain predictor is the cubic
    extrapolation 4 D1 - 6 D2 + 4 D3 - D4: its error is below tau itself, so
    the change of the first sweep already passes the stopping test, and the
    iterate it returns is within a few hundredths of tau of the fixed point."""
    u0 = inputs.smooth_random(N, seed)
    u, _, incs, _ = oracle.implicit_midpoint(u0, NU, DT, 4, 1e-13)
    pred = extrapolation_predictor(u, incs)
    ref, _, ok, _ = oracle.implicit_midpoint_step(u, NU, DT, 1e-14, 80, pred)
    assert ok
    inc = half_norm(ref - u)
    m = oracle.retained_mask(N)
    e0 = half_norm(pred * m - ref) / inc
    w1, _ = midpoint_sweep(u, pred * m, NU, DT)
    e1 = half_norm(w1 - ref) / inc
    print(f"N={N}: cubic extrapolation e_0 = {e0:.2e}, after one sweep {e1:.2e}", flush=True)
    assert e0 < TAU and e1 < 0.1 * TAU
    _, sweeps, ok, _ = oracle.implicit_midpoint_step(u, NU, DT, TAU, 20, pred)
    assert ok and sweeps == 1
