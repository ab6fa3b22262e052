"""Plain FP64 CPU oracle of one implicit-midpoint time step of Eq. NSfinal,
solved by Picard sweeps (fixed-point iteration).

TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg use this module; the GPU library shares no code
with it and never calls it.

Sec. 2 leaves the time integrator open.  The paper runs a fourth-order
Runge-Kutta method, which is explicit and has no inner iteration.  This module
is the implicit alternative: the implicit midpoint rule, which is
Crank-Nicolson on the viscous (linear) term.  With m = (u^n + u^{n+1})/2,

    u^{n+1} - u^n = dt * F(m),     F(v) = F_NL(v) - nu |k|^2 v,

where F is the right-hand side of Eq. NSfinal and F_NL its projected,
dealiased nonlinear part (F with nu = 0).  Solving the linear part per mode
(a = dt nu |k|^2 / 2) gives the sweep

    G(w) = [(1 - a) u^n + dt F_NL((u^n + w) / 2)] / (1 + a),

and u^{n+1} is the fixed point of G.  The Picard iteration starts from a
predictor w_0 and applies w_{j+1} = G(w_j).  It stops after the first sweep
with ||w_{j+1} - w_j|| <= tau ||w_{j+1} - u^n||, or after max_iter sweeps.

Readings (the paper is silent on all of them):
  * norm: the L2 norm of the real field, written over the half-spectrum with
    weight 1 on the kz = 0 and kz = N/2 planes and 2 elsewhere (Parseval);
  * predictor ("plain"): u^n plus the polynomial through the last m =
    min(4, steps so far) increments D1 (newest) ... Dm, evaluated one step
    ahead: sum_j (-1)^(j+1) binom(m, j) D_j, i.e. u^n, u^n + D1,
    u^n + 2 D1 - D2, u^n + 3 D1 - 3 D2 + D3, u^n + 4 D1 - 6 D2 + 4 D3 - D4
    (exact when the state is a polynomial in time of degree m);
  * the state is projected onto the retained set first, as in the RK4 oracle.

Pins (tests marked "not gpu"):
  * the exact Crank-Nicolson factor (1 - a)/(1 + a) for Beltrami fields, whose
    nonlinear term vanishes;
  * the defining equation u^{n+1} - u^n = dt F(m), checked with the pinned
    right-hand side of Eq. NSfinal;
  * time symmetry: a step of -dt undoes a step of dt;
  * the discrete energy budget E^{n+1} - E^n = -dt nu sum w |k|^2 |m|^2 / N^6,
    which conserves E when nu = 0;
  * second-order convergence against a fine RK4 reference.
"""
from __future__ import annotations

from math import comb

import numpy as np

from .spectral_ns import retained_mask, rhs, wavenumbers

__all__ = [
    "nonlinear",
    "half_norm",
    "midpoint_sweep",
    "extrapolation_predictor",
    "implicit_midpoint_step",
    "implicit_midpoint",
]


def nonlinear(uh: np.ndarray, dealias: str = "two_thirds") -> np.ndarray:
    """F_NL: the projected, dealiased nonlinear term of Eq. NSfinal, i.e. the
    right-hand side with the viscous term left out (nu = 0)."""
    return rhs(uh, 0.0, dealias)


def half_norm(x: np.ndarray) -> float:
    """L2 norm of the real field a half-spectrum vector field represents, up
    to the constant N^3 of Parseval: sqrt(sum_k w_k |x_k|^2), weight 1 on the
    kz = 0 and kz = N/2 planes and 2 elsewhere."""
    N = x.shape[1]
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    return float(np.sqrt(np.sum(w * np.sum(np.abs(x) ** 2, axis=(0, 1, 2)))))


def _half_coefficient(N: int, nu: float, dt: float) -> np.ndarray:
    """a = dt nu |k|^2 / 2 on the half-spectrum grid."""
    kx, ky, kz = wavenumbers(N)
    return 0.5 * dt * nu * (kx * kx + ky * ky + kz * kz)


def midpoint_sweep(u0: np.ndarray, w: np.ndarray, nu: float, dt: float, dealias: str = "two_thirds"):
    """One Picard sweep G(w) = [(1 - a) u0 + dt F_NL((u0 + w)/2)] / (1 + a).
    Returns (G(w), F_NL at the midpoint)."""
    N = u0.shape[1]
    a = _half_coefficient(N, nu, dt)
    fnl = nonlinear(0.5 * (u0 + w), dealias)
    return ((1.0 - a) * u0 + dt * fnl) / (1.0 + a), fnl


PREDICTOR_DEPTH = 4  # increments the plain predictor extrapolates at most


def extrapolation_predictor(u0: np.ndarray, history) -> np.ndarray:
    """Plain predictor from the increments of the previous steps (oldest
    first): u0 plus the polynomial through the last m = min(4, len(history))
    increments one step ahead, sum_j (-1)^(j+1) binom(m, j) D_j with D1 the
    newest."""
    m = min(PREDICTOR_DEPTH, len(history))
    pred = u0.copy()
    for j in range(1, m + 1):
        pred = pred + (-1) ** (j + 1) * comb(m, j) * history[-j]
    return pred


def implicit_midpoint_step(u0: np.ndarray, nu: float, dt: float, tau: float = 1e-10, max_iter: int = 50,
                           predictor: np.ndarray | None = None, dealias: str = "two_thirds"):
    """One implicit-midpoint step from u0 by Picard sweeps.

    Returns (u1, sweeps, converged, fnl): the last iterate, the number of
    sweeps done, whether the stopping test passed, and F_NL at the last
    sweep's midpoint."""
    N = u0.shape[1]
    M = retained_mask(N, dealias)
    u0 = u0 * M
    w = u0.copy() if predictor is None else predictor * M
    fnl = None
    for sweep in range(1, max_iter + 1):
        w_next, fnl = midpoint_sweep(u0, w, nu, dt, dealias)
        update = half_norm(w_next - w)
        increment = half_norm(w_next - u0)
        w = w_next
        if update <= tau * increment:
            return w, sweep, True, fnl
    return w, max_iter, False, fnl


def implicit_midpoint(u0: np.ndarray, nu: float, dt: float, nsteps: int, tau: float = 1e-10, max_iter: int = 50,
                      dealias: str = "two_thirds"):
    """nsteps implicit-midpoint steps, each started from the plain
    extrapolation predictor of the increments of the steps before it.

    Returns (u, sweeps, increments, fnls): the final state, the sweeps of each
    step, the increment u^{n+1} - u^n of each step, and F_NL at each step's
    last midpoint."""
    N = u0.shape[1]
    u = u0 * retained_mask(N, dealias)
    sweeps, incs, fnls = [], [], []
    for _ in range(nsteps):
        pred = extrapolation_predictor(u, incs[-PREDICTOR_DEPTH:])
        u1, s, ok, fnl = implicit_midpoint_step(u, nu, dt, tau, max_iter, pred, dealias)
        if not ok:
            raise RuntimeError(f"Picard iteration did not reach tau={tau} in {max_iter} sweeps")
        incs.append(u1 - u)
        fnls.append(fnl)
        sweeps.append(s)
        u = u1
    return u, sweeps, incs, fnls
