"""Seeded synthetic velocity fields in the canonical spectral layout.

This module is the only code shared by the CPU oracle's tests and the GPU path.
It draws inputs and nothing else: no transform, curl, cross product, projection
or time stepping lives here.  Every array it returns is a half-spectrum
``uhat[3][kx][ky][kz]`` (complex128, kz in 0..N/2, kx and ky in FFT order), the
layout of the spectral field of Sec. 3.3 on a single rank.

Families (value ranges follow the Taylor-Green case of Sec. 4: velocities of
order one, kinetic energy 1/8):

* ``taylor_green``  -- the initial condition of Sec. 4, written out exactly as
  its eight Fourier modes (no transform needed).
* ``smooth_random`` -- "R1": a random solenoidal field with energy spectrum
  shaped as |k|^4 exp(-2|k|^2/9) (peak near |k| = 3), band-limited to
  |k_i| <= 16 so that the same seed gives the same physical field at every
  N >= 49, scaled to E = 1/8.
* ``rough_random``  -- "R2": random solenoidal field that fills every retained
  mode with equal expected energy, scaled to E = 1/8 (stress case).
* ``beltrami``      -- random helical field on one shell |k|^2 = K2.  Its
  vorticity is parallel to it, so the nonlinear term vanishes (used for exact
  decay checks).
* ``wide_sparse_modes`` -- a random solenoidal field on a few modes that reach
  the faces and corners of the retained box (full-size checks against the
  triad-sum oracle); ``plane_sparse_modes`` -- the same for a field that does
  not depend on x, with kz held below a bound (one slab share at full size).

Randomness: numpy.random.default_rng(seed) (PCG64), drawn in an order that
does not depend on N where stated.
"""
from __future__ import annotations

import functools

import numpy as np

__all__ = [
    "signed_index",
    "taylor_green",
    "taylor_green_physical",
    "smooth_random",
    "smooth_random_modes",
    "rough_random",
    "beltrami",
    "beltrami_modes",
    "wide_sparse_modes",
    "plane_sparse_modes",
    "kinetic_energy",
]


def signed_index(N: int) -> np.ndarray:
    """Wavenumber of FFT index j on an axis of length N (Eq. wavemesh): j for
    j <= N/2, j - N above (so index N/2 carries +N/2)."""
    j = np.arange(N)
    return np.where(j <= N // 2, j, j - N)


def _half_shape(N):
    return (3, N, N, N // 2 + 1)


def taylor_green(N: int) -> np.ndarray:
    """Exact half-spectrum of u = sin x cos y cos z, v = -cos x sin y cos z,
    w = 0 (Sec. 4) under the unnormalised forward transform of Eq. ffteq.

    Expanding the trigonometric products gives 8 modes (+-1, +-1, +-1); the
    u-coefficient of mode (sx, sy, sz) is N^3 * sx / (8i), the v-coefficient
    N^3 * (-sy) / (8i).  Only sz = +1 is stored in the half-spectrum.
    """
    if N < 4 or N % 2:
        raise ValueError("N must be even and >= 4")
    uh = np.zeros(_half_shape(N), dtype=np.complex128)
    n3 = float(N) ** 3
    for sx in (-1, 1):
        for sy in (-1, 1):
            ix, iy = sx % N, sy % N
            uh[0, ix, iy, 1] = n3 * sx / 8j
            uh[1, ix, iy, 1] = n3 * (-sy) / 8j
    return uh


def taylor_green_physical(N: int) -> np.ndarray:
    """The same field sampled on the mesh of Eq. realmesh, shape (3, N, N, N)."""
    x = 2 * np.pi * np.arange(N) / N
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([
        np.sin(X) * np.cos(Y) * np.cos(Z),
        -np.cos(X) * np.sin(Y) * np.cos(Z),
        np.zeros_like(X),
    ])


def kinetic_energy(uh: np.ndarray) -> float:
    """E = <|u|^2>/2 from a half-spectrum (Parseval with the 1/N^3 of Eq.
    ffteq): E = sum_half w |uhat|^2 / (2 N^6), w = 1 on the kz = 0 and kz = N/2
    planes and 2 elsewhere.  Used only to scale generated fields."""
    N = uh.shape[1]
    w = np.full(uh.shape[-1], 2.0)
    w[0] = 1.0
    if N % 2 == 0:
        w[-1] = 1.0
    return float(np.sum(w * np.sum(np.abs(uh) ** 2, axis=(0, 1, 2))) / (2.0 * float(N) ** 6))


def _plane_basis(k: np.ndarray):
    """Two orthonormal vectors spanning the plane perpendicular to each row of
    k (shape (..., 3), k != 0).  Geometry for sampling only."""
    kf = k.astype(np.float64)
    kn = np.linalg.norm(kf, axis=-1, keepdims=True)
    khat = kf / kn
    # reference direction: the coordinate axis least aligned with k
    ref = np.zeros_like(kf)
    ax = np.argmin(np.abs(khat), axis=-1)
    np.put_along_axis(ref, ax[..., None], 1.0, axis=-1)
    e1 = np.cross(ref, khat)
    e1 /= np.linalg.norm(e1, axis=-1, keepdims=True)
    e2 = np.cross(khat, e1)
    return e1, e2


def _place_band(N, kvec, amp, keep):
    """Scatter band-limited complex vectors amp[m] (m over kvec rows) into a
    half-spectrum of size N, making it Hermitian on kz = 0.  Rows whose
    wavenumber is not representable/retained (``keep`` false) are dropped."""
    uh = np.zeros(_half_shape(N), dtype=np.complex128)
    kx, ky, kz = kvec[:, 0], kvec[:, 1], kvec[:, 2]
    sel = keep & (kz >= 0)
    # upper half (kz > 0): store directly
    up = sel & (kz > 0)
    uh[:, kx[up] % N, ky[up] % N, kz[up]] = amp[up].T
    # kz = 0 plane: make u(-k) = conj(u(k)) by averaging the two draws
    z0 = sel & (kz == 0)
    plane = np.zeros((3, N, N), dtype=np.complex128)
    plane[:, kx[z0] % N, ky[z0] % N] = amp[z0].T
    neg = np.conj(plane[:, (-np.arange(N)) % N][:, :, (-np.arange(N)) % N])
    uh[:, :, :, 0] = 0.5 * (plane + neg)
    return uh


def _band_vectors(kmax: int):
    r = np.arange(-kmax, kmax + 1)
    KX, KY, KZ = np.meshgrid(r, r, r, indexing="ij")
    k = np.stack([KX.ravel(), KY.ravel(), KZ.ravel()], axis=-1)
    return k


def _retained(N, k, dealias):
    """Which integer wavenumbers are stored and kept at size N: the 2/3 rule
    (3|k_i| < N on every axis) or all but the Nyquist planes."""
    a = np.abs(k)
    if dealias == "two_thirds":
        return np.all(3 * a < N, axis=-1)
    if dealias == "none":
        return np.all(a < N // 2, axis=-1)
    raise ValueError(dealias)


@functools.lru_cache(maxsize=4)
def _band_basis(band: int):
    """The band cube's wavenumbers, their R1 spectral shape and plane bases
    (independent of the seed, so computed once per band)."""
    k = _band_vectors(band)
    nz = np.any(k != 0, axis=-1)
    k2 = np.sum(k * k, axis=-1).astype(np.float64)
    shape = np.where(nz, k2 * np.exp(-k2 / 9.0), 0.0)
    e1, e2 = _plane_basis(k[nz])
    return k, nz, shape, e1, e2


def smooth_random_modes(N: int, seed: int, dealias: str = "two_thirds", band: int = 16):
    """R1 in sparse form: FFT indices (ix, iy, iz) and values (3, n) of the
    nonzero half-spectrum entries.  Spectrum |k|^4 exp(-2|k|^2/9), random
    solenoidal directions, band-limited to |k_i| <= band, E = 1/8.  The draws
    cover the whole band cube in a fixed order, so the field does not depend
    on N (beyond truncation by the retained set)."""
    rng = np.random.default_rng(seed)
    k, nz, shape, e1, e2 = _band_basis(band)
    n = len(k)
    a1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a2 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    amp = np.zeros((n, 3), dtype=np.complex128)
    amp[nz] = (a1[nz, None] * e1 + a2[nz, None] * e2) * shape[nz, None]
    # the cube is ordered lexicographically and symmetric, so -k sits at n-1-m;
    # on kz = 0 take u(k) = (a(k) + conj a(-k))/2 so that u(-k) = conj u(k)
    z0 = k[:, 2] == 0
    amp[z0] = 0.5 * (amp[z0] + np.conj(amp[::-1][z0]))
    keep = _retained(N, k, dealias) & nz & (k[:, 2] >= 0)
    kk, vals = k[keep], amp[keep].T.copy()
    w = np.where(kk[:, 2] == 0, 1.0, 2.0)
    E = float(np.sum(w * np.sum(np.abs(vals) ** 2, axis=0)) / (2.0 * float(N) ** 6))
    if E > 0:
        vals *= np.sqrt(0.125 / E)
    return kk[:, 0] % N, kk[:, 1] % N, kk[:, 2], vals


def smooth_random(N: int, seed: int, dealias: str = "two_thirds", band: int = 16) -> np.ndarray:
    """R1 as a dense half-spectrum (see smooth_random_modes)."""
    ix, iy, iz, vals = smooth_random_modes(N, seed, dealias, band)
    uh = np.zeros(_half_shape(N), dtype=np.complex128)
    uh[:, ix, iy, iz] = vals
    return uh


def rough_random(N: int, seed: int, dealias: str = "two_thirds") -> np.ndarray:
    """R2: random solenoidal field on every retained mode (flat spectrum in
    expectation), E = 1/8.  Drawn over the retained cube of this N."""
    if dealias == "two_thirds":
        kmax = (N - 1) // 3
    else:
        kmax = N // 2 - 1
    rng = np.random.default_rng(seed)
    r = np.arange(-kmax, kmax + 1)
    rz = np.arange(0, kmax + 1)
    KX, KY, KZ = np.meshgrid(r, r, rz, indexing="ij")
    k = np.stack([KX.ravel(), KY.ravel(), KZ.ravel()], axis=-1)
    n = len(k)
    a1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a2 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    nz = np.any(k != 0, axis=-1)
    amp = np.zeros((n, 3), dtype=np.complex128)
    e1, e2 = _plane_basis(k[nz])
    amp[nz] = a1[nz, None] * e1 + a2[nz, None] * e2
    uh = _place_band(N, k, amp, nz)
    E = kinetic_energy(uh)
    return uh * np.sqrt(0.125 / E)


def _shell_vectors(K2: int) -> np.ndarray:
    """Integer vectors with |k|^2 = K2, in lexicographic (kx, ky, kz) order:
    the rows of _band_vectors(floor(sqrt(K2))) that lie on the shell, found
    per (kx, ky) column instead of by scanning the whole cube."""
    kmax = int(np.floor(np.sqrt(K2)))
    r = np.arange(-kmax, kmax + 1)
    KX, KY = np.meshgrid(r, r, indexing="ij")
    kx, ky = KX.ravel(), KY.ravel()
    rem = K2 - kx * kx - ky * ky
    ok = rem >= 0
    kx, ky, rem = kx[ok], ky[ok], rem[ok]
    s = np.floor(np.sqrt(rem.astype(np.float64))).astype(np.int64)
    s += (s + 1) * (s + 1) <= rem  # exact integer square root
    s -= s * s > rem
    on = s * s == rem
    kx, ky, s = kx[on], ky[on], s[on]
    col = np.arange(len(kx))
    two = s > 0  # kz = -s then +s; one row where s = 0
    rows = np.concatenate([np.stack([kx[two], ky[two], -s[two]], -1), np.stack([kx, ky, s], -1)])
    key = np.concatenate([2 * col[two], 2 * col + 1])
    return rows[np.argsort(key, kind="stable")]


def beltrami_modes(N: int, K2: int, seed: int, sign: int = 1):
    """Random field on the shell |k|^2 = K2 in sparse form: FFT indices
    (ix, iy, iz) and values (3, n) of the nonzero half-spectrum entries.
    Built from helical vectors h = (e1 + i*sign*e2)/sqrt(2), for which
    i k x h = sign*|k| h, so the vorticity is sign*sqrt(K2) times the velocity
    and u x omega = 0.  Scaled to E = 1/8 on the N grid.  Requires the shell
    to survive the 2/3 rule."""
    k = _shell_vectors(K2)
    if len(k) == 0:
        raise ValueError("empty shell")
    if not np.all(_retained(N, k, "two_thirds")):
        raise ValueError("shell not retained at this N")
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(len(k)) + 1j * rng.standard_normal(len(k))
    e1, e2 = _plane_basis(k)
    # right-handed pair: e1 x e2 = k/|k|  (true by construction of _plane_basis)
    h = (e1 + 1j * sign * e2) / np.sqrt(2.0)
    amp = a[:, None] * h
    # Hermitian pairing u(-k) = conj(u(k)) keeps the helicity sign; the shell
    # is symmetric and lexicographically ordered, so -k sits at n-1-m
    amp = 0.5 * (amp + np.conj(amp[::-1]))
    up = k[:, 2] >= 0
    kk, vals = k[up], amp[up].T.copy()
    w = np.where(kk[:, 2] == 0, 1.0, 2.0)
    E = float(np.sum(w * np.sum(np.abs(vals) ** 2, axis=0)) / (2.0 * float(N) ** 6))
    vals *= np.sqrt(0.125 / E)
    return kk[:, 0] % N, kk[:, 1] % N, kk[:, 2], vals


def beltrami(N: int, K2: int, seed: int, sign: int = 1) -> np.ndarray:
    """Dense half-spectrum of beltrami_modes(N, K2, seed, sign)."""
    ix, iy, iz, vals = beltrami_modes(N, K2, seed, sign)
    uh = np.zeros(_half_shape(N), dtype=np.complex128)
    uh[:, ix, iy, iz] = vals
    return uh


def wide_sparse_modes(N: int, count: int, seed: int, dealias: str = "two_thirds"):
    """A random solenoidal field on a few modes spread over the whole retained
    set, in the sparse form of smooth_random_modes: FFT indices (ix, iy, iz)
    and values (3, n).  The modes are the corners, edge midpoints and face
    centres of the retained box (components 0 and +-kmax, +-(kmax - 1)) and
    `count` wavenumbers drawn uniformly from the retained half box.  On the
    kz = 0 plane both k and -k are stored, with conjugate values.  E = 1/8 on
    the N grid."""
    kmax = (N - 1) // 3 if dealias == "two_thirds" else N // 2 - 1
    rng = np.random.default_rng(seed)
    drawn = np.stack([rng.integers(-kmax, kmax + 1, count), rng.integers(-kmax, kmax + 1, count),
                      rng.integers(0, kmax + 1, count)], axis=-1)
    c = np.array([-kmax, 0, kmax])
    d = np.array([-(kmax - 1), kmax - 1])
    box = np.stack(np.meshgrid(c, c, np.array([0, kmax]), indexing="ij"), -1).reshape(-1, 3)
    near = np.stack(np.meshgrid(d, d, np.array([kmax - 1]), indexing="ij"), -1).reshape(-1, 3)
    k = np.concatenate([box, near, drawn])
    z0 = k[k[:, 2] == 0]
    k = np.unique(np.concatenate([k, -z0]), axis=0)  # lexicographic, -k paired on kz = 0
    k = k[np.any(k != 0, axis=-1)]
    n = len(k)
    a1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a2 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    e1, e2 = _plane_basis(k)
    vals = (a1[:, None] * e1 + a2[:, None] * e2).T.copy()
    # kz = 0: the row of -k takes the conjugate of the row of k (k > -k in
    # lexicographic order keeps its own draw)
    z = np.nonzero(k[:, 2] == 0)[0]
    row = {tuple(k[m]): m for m in z}
    for m in z:
        q = row[tuple(-k[m])]
        if tuple(k[m]) < tuple(k[q]):
            vals[:, m] = np.conj(vals[:, q])
    w = np.where(k[:, 2] == 0, 1.0, 2.0)
    E = float(np.sum(w * np.sum(np.abs(vals) ** 2, axis=0)) / (2.0 * float(N) ** 6))
    vals *= np.sqrt(0.125 / E)
    return k[:, 0] % N, k[:, 1] % N, k[:, 2], vals


def plane_sparse_modes(N: int, count: int, seed: int, kz_max: int):
    """A random solenoidal field that does not depend on x (every mode has
    kx = 0) on a few modes, in the sparse form of smooth_random_modes: ky
    over the whole retained range (+-kmax included), kz in 0..kz_max (both
    ends included).  On the kz = 0 plane both k and -k are stored, with
    conjugate values.  E = 1/8 on the N grid."""
    kmax = (N - 1) // 3
    if not 0 < kz_max <= kmax:
        raise ValueError("kz_max outside the retained range")
    rng = np.random.default_rng(seed)
    drawn = np.stack([np.zeros(count, dtype=np.int64), rng.integers(-kmax, kmax + 1, count),
                      rng.integers(0, kz_max + 1, count)], axis=-1)
    ends = np.array([[0, ky, kz] for ky in (-kmax, -1, 1, kmax) for kz in (0, kz_max)] + [[0, 0, kz_max]])
    k = np.concatenate([ends, drawn])
    z0 = k[k[:, 2] == 0]
    k = np.unique(np.concatenate([k, -z0]), axis=0)
    k = k[np.any(k != 0, axis=-1)]
    n = len(k)
    a1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a2 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    e1, e2 = _plane_basis(k)
    vals = (a1[:, None] * e1 + a2[:, None] * e2).T.copy()
    z = np.nonzero(k[:, 2] == 0)[0]
    row = {tuple(k[m]): m for m in z}
    for m in z:
        q = row[tuple(-k[m])]
        if tuple(k[m]) < tuple(k[q]):
            vals[:, m] = np.conj(vals[:, q])
    w = np.where(k[:, 2] == 0, 1.0, 2.0)
    E = float(np.sum(w * np.sum(np.abs(vals) ** 2, axis=0)) / (2.0 * float(N) ** 6))
    vals *= np.sqrt(0.125 / E)
    return k[:, 0] % N, k[:, 1] % N, k[:, 2], vals


BATCH_SIZES = (16, 18, 24, 32, 36, 48, 54, 64)


def batch_sizes(count: int, seed: int, sizes=BATCH_SIZES) -> np.ndarray:
    """Sizes of a batch of uneven instances: N log-uniform over [min, max] of
    `sizes` (so N^3 spans a factor 64 for 16..64), each rounded in log space
    to the nearest allowed size (2^a 3^b)."""
    allowed = np.asarray(sizes)
    rng = np.random.default_rng(seed)
    logn = rng.uniform(np.log(allowed.min()), np.log(allowed.max()), count)
    pick = np.argmin(np.abs(np.log(allowed)[None, :] - logn[:, None]), axis=1)
    return allowed[pick]
