"""Plain, slow, FP64 CPU oracle of one RK4 step of the Fourier-Galerkin
Navier-Stokes right-hand side (Mortensen, "Massively parallel implementation in
Python of a pseudo-spectral DNS code for turbulent flows", arXiv 1607.00850).

TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg use this module; the GPU library shares no code
with it and never calls it.

Every function follows the paper's definitions in the paper's order and
notation, with numpy.fft (pocketfft) as the serial FFT (Sec. 3.3 allows any
serial FFT provider).  Nothing is fused, blocked or reordered.

Layout: a spectral vector field is ``uhat[3][kx][ky][kz]`` with kx, ky in FFT
order (N entries) and kz in 0..N/2 -- the single-rank spectral array of
Sec. 3.3 -- i.e. exactly numpy's ``rfftn`` over axes (1, 2, 3).  A physical
field is ``u[3][x][y][z]`` on the mesh of Eq. realmesh.

Readings where the paper is silent or ambiguous (each also listed in the
design notes):
  * dealiasing is "the same technique" as Tarang (Sec. 4) -- read as the 2/3
    rule with a box cut: mode k is kept iff 3|k_i| < N on every axis.  A
    second mode ("none") keeps every mode except the Nyquist planes.
  * the state lives in the retained (Galerkin) set: the input is projected
    onto it first, so modes outside it are dropped, and the output is zero
    there.
  * the Nyquist index N/2 carries +N/2 (Eq. wavemesh); it is never retained.
  * at k = 0 the pressure term k (k.N)/|k|^2 is taken as zero.
  * "fourth order Runge-Kutta" (Sec. 2) is the classical scheme.

Pins (tests marked "not gpu"): brute-force DFT sums of Eq. ffteq; the
closed-form Taylor-Green right-hand side at t = 0; exact Beltrami decay under
RK4; the brute-force Galerkin triad sum for the dealiased product; the energy
budget, divergence and mean-mode identities; RK4 convergence order; numpy.cross
for the component formula; the slab-decomposed transform with P virtual ranks
against the serial one.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "wavenumbers",
    "retained_mask",
    "forward",
    "inverse",
    "forward_slab",
    "inverse_slab",
    "curl",
    "cross",
    "rhs",
    "rk4_step",
    "rk4",
    "energy",
    "dissipation_rate",
]

DEALIAS_MODES = ("two_thirds", "none")


def wavenumbers(N: int):
    """Integer wavenumber grids of Eq. wavemesh, broadcastable to the
    half-spectrum shape (N, N, N/2+1).  Index j on the x and y axes carries
    k = j for j <= N/2 and k = j - N above; the z axis stores k = 0..N/2."""
    j = np.arange(N)
    k = np.where(j <= N // 2, j, j - N).astype(np.int64)
    kz = np.arange(N // 2 + 1, dtype=np.int64)
    return k[:, None, None], k[None, :, None], kz[None, None, :]


def retained_mask(N: int, dealias: str = "two_thirds") -> np.ndarray:
    """Boolean mask of the kept modes on the half-spectrum.

    ``two_thirds``: keep k iff 3|k_x| < N and 3|k_y| < N and 3|k_z| < N
    (strict, in integers).  ``none``: keep every mode whose |k_i| < N/2 on all
    axes (the Nyquist planes are dropped).  Dealiasing technique: Sec. 4."""
    kx, ky, kz = wavenumbers(N)
    if dealias == "two_thirds":
        m = (3 * np.abs(kx) < N) & (3 * np.abs(ky) < N) & (3 * np.abs(kz) < N)
    elif dealias == "none":
        h = N // 2
        m = (np.abs(kx) < h) & (np.abs(ky) < h) & (np.abs(kz) < h)
    else:
        raise ValueError(f"unknown dealias mode {dealias!r}")
    return np.broadcast_to(m, (N, N, N // 2 + 1)).copy()


def forward(u: np.ndarray) -> np.ndarray:
    """uhat_k = sum_x u(x) exp(-i k.x) (Eq. ffteq, second line), on the last
    three axes; unnormalised.  The serial provider is numpy.fft (Sec. 3.3)."""
    return np.fft.rfftn(u, axes=(-3, -2, -1))


def inverse(uh: np.ndarray, N: int) -> np.ndarray:
    """u(x) = (1/N^3) sum_k uhat_k exp(i k.x) (Eq. ffteq, first line) from the
    half-spectrum; the 1/N^3 is numpy's ``irfftn`` normalisation."""
    return np.fft.irfftn(uh, s=(N, N, N), axes=(-3, -2, -1))


def forward_slab(u: np.ndarray, P: int) -> np.ndarray:
    """The forward transform as the slab-decomposed 3D FFT of Sec. 3 ("Three
    dimensional Fourier transforms with MPI") run by P virtual ranks, then
    reassembled.  Rank r owns the physical x-planes [r Np, (r+1) Np),
    Np = N/P.  Each rank transforms its planes along z (real to complex) and
    y; an all-to-all then hands rank q the ky columns [q Np, (q+1) Np) of
    every rank's planes, stacked in x order, and rank q finishes with the
    transform along x.  Unnormalised, as forward()."""
    N = u.shape[-1]
    if N % P:
        raise ValueError("P must divide N")
    Np = N // P
    planes = [np.fft.fft(np.fft.rfft(u[..., r * Np:(r + 1) * Np, :, :], axis=-1), axis=-2) for r in range(P)]
    slabs = []
    for q in range(P):
        received = [planes[r][..., :, q * Np:(q + 1) * Np, :] for r in range(P)]
        slabs.append(np.fft.fft(np.concatenate(received, axis=-3), axis=-3))
    return np.concatenate(slabs, axis=-2)


def inverse_slab(uh: np.ndarray, N: int, P: int) -> np.ndarray:
    """The inverse of forward_slab in the reverse order (Sec. 2: the inverse
    transforms run in the opposite order): rank q transforms its ky columns
    back along x, an all-to-all returns the x-planes [r Np, (r+1) Np) to
    rank r, which transforms along y and then z (complex to real).  With the
    1/N^3 of Eq. ffteq, as inverse()."""
    if N % P:
        raise ValueError("P must divide N")
    Np = N // P
    cols = [np.fft.ifft(uh[..., :, q * Np:(q + 1) * Np, :], axis=-3) for q in range(P)]
    planes = []
    for r in range(P):
        received = [cols[q][..., r * Np:(r + 1) * Np, :, :] for q in range(P)]
        planes.append(np.fft.irfft(np.fft.ifft(np.concatenate(received, axis=-2), axis=-2), n=N, axis=-1))
    return np.concatenate(planes, axis=-3)


def curl(uh: np.ndarray) -> np.ndarray:
    """Spectral curl, omega_hat = i k x uhat (omega = curl u, Sec. 2; the
    derivative becomes multiplication by i k under Eq. ffteq)."""
    N = uh.shape[1]
    kx, ky, kz = wavenumbers(N)
    return 1j * np.stack([
        ky * uh[2] - kz * uh[1],
        kz * uh[0] - kx * uh[2],
        kx * uh[1] - ky * uh[0],
    ])


def cross(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """c = a x b by components, the formula of the cross-product routine in
    Sec. 3.4: c0 = a1 b2 - a2 b1, c1 = a2 b0 - a0 b2, c2 = a0 b1 - a1 b0."""
    return np.stack([
        a[1] * b[2] - a[2] * b[1],
        a[2] * b[0] - a[0] * b[2],
        a[0] * b[1] - a[1] * b[0],
    ])


def rhs(uh: np.ndarray, nu: float, dealias: str = "two_thirds") -> np.ndarray:
    """Right-hand side of Eq. NSfinal for a half-spectrum velocity:

        du_k/dt = (u x w)^_k - nu |k|^2 u_k - k (k . (u x w)^_k) / |k|^2

    with the pressure already eliminated (Eq. pressure).  Steps, in the
    paper's order:
      0. project the state onto the retained set (dealiasing reading);
      1. omega_hat = i k x uhat                          (Sec. 2)
      2. u = F^-1(uhat), omega = F^-1(omega_hat)         (Eq. ffteq)
      3. c = u x omega                                   (Sec. 3.4 formula)
      4. N_hat = mask * F(c)                             (Eq. ffteq; dealias)
      5. N_hat - nu|k|^2 uhat - k (k.N_hat)/|k|^2, last term 0 at k = 0
    """
    N = uh.shape[1]
    M = retained_mask(N, dealias)
    uh = uh * M
    wh = curl(uh)
    u = inverse(uh, N)
    w = inverse(wh, N)
    c = cross(u, w)
    Nh = forward(c) * M
    kx, ky, kz = wavenumbers(N)
    k2 = kx * kx + ky * ky + kz * kz
    k2_safe = np.where(k2 == 0, 1, k2)
    kdotN = kx * Nh[0] + ky * Nh[1] + kz * Nh[2]
    p = np.where(k2 == 0, 0.0, kdotN / k2_safe)
    return np.stack([
        Nh[0] - nu * k2 * uh[0] - kx * p,
        Nh[1] - nu * k2 * uh[1] - ky * p,
        Nh[2] - nu * k2 * uh[2] - kz * p,
    ])


def rk4_step(uh: np.ndarray, nu: float, dt: float, dealias: str = "two_thirds") -> np.ndarray:
    """One classical fourth-order Runge-Kutta step of Eq. NSfinal (Sec. 2):
    k1 = F(u), k2 = F(u + dt/2 k1), k3 = F(u + dt/2 k2), k4 = F(u + dt k3),
    u_next = u + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    N = uh.shape[1]
    uh = uh * retained_mask(N, dealias)
    k1 = rhs(uh, nu, dealias)
    k2 = rhs(uh + 0.5 * dt * k1, nu, dealias)
    k3 = rhs(uh + 0.5 * dt * k2, nu, dealias)
    k4 = rhs(uh + dt * k3, nu, dealias)
    return uh + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk4(uh: np.ndarray, nu: float, dt: float, nsteps: int, dealias: str = "two_thirds") -> np.ndarray:
    """nsteps RK4 steps from uhat (projected onto the retained set first)."""
    N = uh.shape[1]
    out = uh * retained_mask(N, dealias)
    for _ in range(nsteps):
        out = rk4_step(out, nu, dt, dealias)
    return out


def _half_weights(N: int) -> np.ndarray:
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    return w


def energy(uh: np.ndarray) -> float:
    """Kinetic energy E = (1/2) mean |u|^2 = sum_k |uhat_k|^2 / (2 N^6)
    (Parseval under Eq. ffteq), the full-spectrum sum written over the
    half-spectrum with weight 1 on the kz = 0, N/2 planes and 2 elsewhere."""
    N = uh.shape[1]
    s = np.sum(_half_weights(N) * np.sum(np.abs(uh) ** 2, axis=(0, 1, 2)))
    return float(s / (2.0 * float(N) ** 6))


def dissipation_rate(uh: np.ndarray, nu: float) -> float:
    """nu <|omega|^2> = nu sum_k |k|^2 |uhat_k|^2 / N^6 for a solenoidal field
    (the rate at which the viscous term of Eq. NSfinal removes energy)."""
    N = uh.shape[1]
    kx, ky, kz = wavenumbers(N)
    k2 = kx * kx + ky * ky + kz * kz
    s = np.sum(_half_weights(N) * np.sum(k2 * np.sum(np.abs(uh) ** 2, axis=0), axis=(0, 1)))
    return float(nu * s / float(N) ** 6)
