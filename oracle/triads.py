"""The right-hand side of Eq. NSfinal for a field with few modes, with the
dealiased product taken from its definition as a Galerkin triad sum rather
than through transforms (test infrastructure, like the rest of this package:
only the tests, the package smoke check and the benchmark's CPU-baseline leg
use it).

Its cost grows with the square of the number of modes and not with N, so it
gives the exact right-hand side of a sparse field at any mesh size, 1024^3
included, where the transform-based oracle cannot run.

Pins (tests marked "not gpu"): equal to the transform-based ``rhs`` at small N
for sparse random fields, both dealiasing modes; the energy identity of the
Galerkin nonlinear term at N = 1024; the closed-form Taylor-Green right-hand
side.
"""
from __future__ import annotations

import numpy as np

__all__ = ["rhs_triads"]


def _kept(k: np.ndarray, N: int, dealias: str) -> np.ndarray:
    """The retained set (the same rule as retained_mask): 3|k_i| < N on every
    axis for the 2/3 rule, |k_i| < N/2 (no Nyquist plane) for ``none``."""
    a = np.abs(k)
    if dealias == "two_thirds":
        return np.all(3 * a < N, axis=-1)
    if dealias == "none":
        return np.all(a < N // 2, axis=-1)
    raise ValueError(f"unknown dealias mode {dealias!r}")


def _cross(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a x b by components (the formula of Sec. 3.4), vectors on axis 0."""
    return np.stack([
        a[1] * b[2] - a[2] * b[1],
        a[2] * b[0] - a[0] * b[2],
        a[0] * b[1] - a[1] * b[0],
    ])


def rhs_triads(k: np.ndarray, uk: np.ndarray, N: int, nu: float, dealias: str = "two_thirds"):
    """du_k/dt of Eq. NSfinal for the field sum_m uk[:, m] exp(i k_m . x) / N^3
    (plus the complex conjugates that make it real).

    k: (n, 3) signed integer wavenumbers of the stored half-spectrum entries,
    k_z >= 0; on the k_z = 0 plane both k and -k are stored, with conjugate
    values.  uk: (3, n) complex coefficients, scaled as in Eq. ffteq on the
    N-point mesh.

    Steps:
      0. drop the entries outside the retained set (the state lives in the
         Galerkin set);
      1. complete the spectrum of the real field: u(-k) = conj u(k) for the
         k_z > 0 entries;
      2. omega_hat_q = i q x u_hat_q                              (Sec. 2)
      3. (u x omega)^_s = N^-3 sum over all pairs (p, q) of completed modes
         with p + q = s (mod N) of u_hat_p x omega_hat_q: the forward
         transform (Eq. ffteq) of the product sampled on the mesh, where two
         wavenumbers that differ by N are one mesh mode;
      4. keep the retained s with s_z >= 0 (the dealiasing mask on the half
         spectrum);
      5. N_hat - nu |k|^2 u_hat - k (k . N_hat) / |k|^2, the last term zero
         at k = 0 (Eq. NSfinal with the pressure eliminated).

    Returns (kout, vals): the (m, 3) signed wavenumbers of every retained
    half-spectrum mode that the product or the state reaches, and the (3, m)
    right-hand side there.  Every other mode of the result is zero.
    """
    k = np.asarray(k, dtype=np.int64).reshape(-1, 3)
    uk = np.asarray(uk, dtype=np.complex128).reshape(3, -1)
    if np.any(k[:, 2] < 0):
        raise ValueError("stored wavenumbers must have k_z >= 0")
    keep = _kept(k, N, dealias)
    k, uk = k[keep], uk[:, keep]
    up = k[:, 2] > 0
    fk = np.concatenate([k, -k[up]])
    fu = np.concatenate([uk, np.conj(uk[:, up])], axis=1)
    fw = 1j * _cross(fk.T, fu)
    n = len(fk)
    P = np.repeat(np.arange(n), n)
    Q = np.tile(np.arange(n), n)
    s = fk[P] + fk[Q]
    s = (s + N // 2) % N - N // 2  # the mesh mode of p + q, signed
    sel = _kept(s, N, dealias) & (s[:, 2] >= 0)
    s, P, Q = s[sel], P[sel], Q[sel]
    terms = _cross(fu[:, P], fw[:, Q]) / float(N) ** 3
    kout, inv = np.unique(np.concatenate([s, k]), axis=0, return_inverse=True)
    inv = inv.ravel()
    m = len(kout)
    Nh = np.zeros((3, m), dtype=np.complex128)
    for c in range(3):
        Nh[c] = (np.bincount(inv[: len(s)], weights=terms[c].real, minlength=m)
                 + 1j * np.bincount(inv[: len(s)], weights=terms[c].imag, minlength=m))
    uh = np.zeros((3, m), dtype=np.complex128)
    uh[:, inv[len(s):]] = uk
    kf = kout.T.astype(np.float64)
    k2 = np.sum(kf * kf, axis=0)
    kdotN = kf[0] * Nh[0] + kf[1] * Nh[1] + kf[2] * Nh[2]
    p = np.where(k2 == 0, 0.0, kdotN / np.where(k2 == 0, 1.0, k2))
    return kout, Nh - nu * k2 * uh - kf * p
