// Pass kernels of one evaluation of the right-hand side of Eq. NSfinal and of
// one classical RK4 stage, for one N^3 instance.
//
// Spectral data inside the library is "compact": only the retained modes are
// stored.  On the x and y axes the retained FFT positions are [0, lo) and
// [N-hi, N) (M = lo + hi rows; row i holds position i for i < lo and
// i + N - M above); on the half (z) axis they are kz in [0, Mz).  With the 2/3
// rule lo = K+1, hi = K, Mz = K+1 where K = floor((N-1)/3); with every mode
// kept (plain transforms) lo = N/2+1, hi = N/2-1, Mz = N/2+1, which is the
// canonical half-spectrum layout itself.
//
// Per right-hand side (Eq. ffteq order: inverse x, y, z; forward z, y, x):
//   P1  x inverse, curl fused on load        U[3][M][M*Mz]  -> A1[6][N][M*Mz]
//   P2  y inverse                            A1[6][N][M][Mz] -> A2[6][N][N][Mz]
//   P3  z C2R, u x omega, z R2C              A2[6][N*N][Mz] -> A2[0..3) (in place)
//   P4  y forward                            A2[3][N][N][Mz] -> A1[3][N][M][Mz]
//   P5  x forward                            A1[3][N][M*Mz] -> Nh[3][M][M*Mz]
//   E   mask/projection/viscous/RK4 stage    Nh, U0, U1, Acc (compact, elementwise)
#pragma once

#include "fft_core.hpp"

namespace hot {

struct Geo {
  int N;
  int lo, hi, M;  // x and y axes
  int Mz;         // z (half) axis
};

__device__ __forceinline__ bool kept(int p, const Geo& g) { return p < g.lo || p >= g.N - g.hi; }
// compact row of a retained position
__device__ __forceinline__ int crow(int p, const Geo& g) { return p < g.lo ? p : p - (g.N - g.M); }
// FFT position of compact row i
__device__ __forceinline__ int cpos(int i, const Geo& g) { return i < g.lo ? i : i + (g.N - g.M); }
// signed wavenumber (Eq. wavemesh) of FFT position p
__device__ __forceinline__ int kwave(int p, int N) { return 2 * p <= N ? p : p - N; }

extern __device__ const TwTable<float, 1024> g_tw1024_f;
extern __device__ const TwTable<double, 1024> g_tw1024_d;
extern __device__ const TwTable<float, 1728> g_tw1728_f;
extern __device__ const TwTable<double, 1728> g_tw1728_d;

template <typename T, int N>
__device__ __forceinline__ const cx<T>* twiddles() {
  if constexpr (std::is_same<T, float>::value) {
    if constexpr (tw_size<N>() == 1024) return g_tw1024_f.w;
    else return g_tw1728_f.w;
  } else {
    if constexpr (tw_size<N>() == 1024) return g_tw1024_d.w;
    else return g_tw1728_d.w;
  }
}

// LDS view for a tile of W interleaved columns (strided passes).
template <typename T, int W>
struct LdsCols {
  cx<T>* base;
  int c;
  __device__ __forceinline__ void put(int pos, cx<T> v) { base[pos * W + c] = v; }
  __device__ __forceinline__ cx<T> get(int pos) const { return base[pos * W + c]; }
  __device__ __forceinline__ void sync() { __syncthreads(); }
};

// LDS view for one contiguous line owned by part of one wave.
template <typename T>
struct LdsLine {
  cx<T>* base;
  __device__ __forceinline__ void put(int pos, cx<T> v) { base[pos] = v; }
  __device__ __forceinline__ cx<T> get(int pos) const { return base[pos]; }
  __device__ __forceinline__ void sync() { wave_sync(); }
};

// ---------------------------------------------------------------------------
// Strided axis pass: columns are contiguous, lines run along rows.
// The array is a batch of [rows][Q] blocks; global column g = b*Q + q.
// IN_C / OUT_C: rows are compact (retained positions only) or all N.
// ---------------------------------------------------------------------------
template <typename T, class Plan, int DIR, int W, bool IN_C, bool OUT_C>
__global__ __launch_bounds__(W* Plan::Tl) void k_strided(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int Q, long ncols, long ld_in, long ld_out,
    long bs_in, long bs_out, long cs_in, long cs_out, Geo g) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  __shared__ cx<T> sm[N * W];
  const int tid = threadIdx.x;
  const int c = tid % W, j = tid / W;
  const long gc = (long)blockIdx.x * W + c;
  const bool valid = gc < ncols;
  const long b = valid ? gc / Q : 0;
  const long q = valid ? gc - b * Q : 0;
  const cx<T>* src = in + blockIdx.y * cs_in + b * bs_in + q;
  cx<T>* dst = out + blockIdx.y * cs_out + b * bs_out + q;
  cx<T> v[R];
  static_for<0, R>([&](auto s) {
    const int p = j + s * Tl;
    cx<T> x = {T(0), T(0)};
    if (IN_C) {
      if (valid && kept(p, g)) x = src[(long)crow(p, g) * ld_in];
    } else {
      if (valid) x = src[(long)p * ld_in];
    }
    v[s] = x;
  });
  LdsCols<T, W> lds{sm, c};
  Plan::template fft<T, DIR>(v, j, lds, twiddles<T, N>());
  static_for<0, R>([&](auto s) {
    const int p = j + s * Tl;
    if (OUT_C) {
      if (valid && kept(p, g)) dst[(long)crow(p, g) * ld_out] = v[s];
    } else {
      if (valid) dst[(long)p * ld_out] = v[s];
    }
  });
}

// ---------------------------------------------------------------------------
// P1: inverse transform along x of the velocity and of the vorticity
// omega_hat = i k x u_hat (curl fused into the load).  Input compact state
// U[3][M rows (kx)][Q = M*Mz cols (ky,kz)], output A[6][N rows (x)][Q].
// Block b: the 6 output components of one tile go to blocks with equal
// b mod 8 so that their shared input rows meet in the same L2.
// ---------------------------------------------------------------------------
template <typename T, class Plan, int W>
__global__ __launch_bounds__(W* Plan::Tl) void k_x_inv_curl(const cx<T>* __restrict__ U, long csU,
                                                            cx<T>* __restrict__ A, long csA, int ntiles,
                                                            Geo g) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  __shared__ cx<T> sm[N * W];
  const int blk = blockIdx.x;
  const int xcd = blk & 7, slot = blk >> 3;
  const int o = slot % 6;
  const int tile = (slot / 6) * 8 + xcd;
  if (tile >= ntiles) return;  // whole block leaves together
  const int tid = threadIdx.x;
  const int c = tid % W, j = tid / W;
  const long Q = (long)g.M * g.Mz;
  const long q = (long)tile * W + c;
  const bool valid = q < Q;
  const int iy = valid ? (int)(q / g.Mz) : 0;
  const int kz = valid ? (int)(q - (long)iy * g.Mz) : 0;
  const T ky = T(kwave(cpos(iy, g), N));
  const T kzf = T(kz);
  const cx<T>* u0 = U + q;
  const cx<T>* u1 = U + csU + q;
  const cx<T>* u2 = U + 2 * csU + q;
  cx<T> v[R];
  static_for<0, R>([&](auto s) {
    const int p = j + s * Tl;
    cx<T> x = {T(0), T(0)};
    if (valid && kept(p, g)) {
      const long off = (long)crow(p, g) * Q;
      const T kx = T(kwave(p, N));
      switch (o) {
        case 0: x = u0[off]; break;
        case 1: x = u1[off]; break;
        case 2: x = u2[off]; break;
        case 3: x = mul_i(u2[off] * ky - u1[off] * kzf); break;
        case 4: x = mul_i(u0[off] * kzf - u2[off] * kx); break;
        default: x = mul_i(u1[off] * kx - u0[off] * ky); break;
      }
    }
    v[s] = x;
  });
  LdsCols<T, W> lds{sm, c};
  Plan::template fft<T, +1>(v, j, lds, twiddles<T, N>());
  if (valid) {
    cx<T>* dst = A + o * csA + q;
    static_for<0, R>([&](auto s) { dst[(long)(j + s * Tl) * Q] = v[s]; });
  }
}

// ---------------------------------------------------------------------------
// z-axis line helpers.  A thread group of Tl = N/R lanes (inside one wave)
// owns one line; the line's LDS region holds N complex values.
// ---------------------------------------------------------------------------

// Hermitian completion of a half-spectrum line pair (a, b) into
// Z_p = a_p + i b_p on the full circle, as the complex input of one inverse
// FFT that returns a in its real part and b in its imaginary part.  As in a
// real inverse transform, the imaginary parts of the kz = 0 and kz = N/2
// coefficients are dropped.
template <typename T, int N>
__device__ __forceinline__ cx<T> completed_pair(const cx<T>* a, const cx<T>* b, int p, int Mz) {
  if (p < Mz && 2 * p <= N) {
    cx<T> x = a[p], y = b[p];
    if (p == 0 || 2 * p == N) {
      x.y = T(0);
      y.y = T(0);
    }
    return {x.x - y.y, x.y + y.x};
  }
  const int m = N - p;
  if (2 * p > N && m < Mz) {
    const cx<T> x = a[m], y = b[m];
    return {x.x + y.y, y.x - x.y};  // conj(x) + i conj(y)
  }
  return {T(0), T(0)};
}

template <typename T, int N>
__device__ __forceinline__ cx<T> completed_one(const cx<T>* a, int p, int Mz) {
  if (p < Mz && 2 * p <= N) {
    cx<T> x = a[p];
    if (p == 0 || 2 * p == N) x.y = T(0);
    return x;
  }
  const int m = N - p;
  if (2 * p > N && m < Mz) return conj(a[m]);
  return {T(0), T(0)};
}

// ---------------------------------------------------------------------------
// P3: per z-line, inverse real transforms of u and omega (three complex FFTs,
// two real lines each), the cross product c = u x omega (component formula
// of Sec. 3.4) scaled by 1/N^6 (the 1/N^3 of Eq. ffteq for each factor), and
// the forward real transform of c (c0 + i c1 in one FFT, c2 in another).
// In place: reads components 0..5 of the line, writes 0..2.
// ---------------------------------------------------------------------------
template <typename T, class Plan>
__global__ __launch_bounds__(256) void k_z_cross(cx<T>* __restrict__ A, long csA, long nlines, Geo g,
                                                 T scale) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  static_assert(64 % Tl == 0, "a z line must sit inside one wave");
  constexpr int LPB = 256 / Tl;  // lines per block
  __shared__ cx<T> sm[LPB * N];
  const int tid = threadIdx.x;
  const int li = tid / Tl, j = tid % Tl;
  const long line = (long)blockIdx.x * LPB + li;
  const bool valid = line < nlines;
  const int Mz = g.Mz;
  LdsLine<T> lds{sm + li * N};
  const cx<T>* tw = twiddles<T, N>();
  const long base = valid ? line * Mz : 0;

  cx<T> ph[3][R];
  static_for<0, 3>([&](auto pr) {
    const cx<T>* a = A + (2 * pr) * csA + base;
    const cx<T>* b = A + (2 * pr + 1) * csA + base;
    static_for<0, R>([&](auto s) {
      const int p = j + s * Tl;
      ph[pr][s] = valid ? completed_pair<T, N>(a, b, p, Mz) : cx<T>{T(0), T(0)};
    });
    Plan::template fft<T, +1>(ph[pr], j, lds, tw);
  });
  // u = (ph0.x, ph0.y, ph1.x), omega = (ph1.y, ph2.x, ph2.y)
  cx<T> z01[R], z2[R];
  static_for<0, R>([&](auto s) {
    const T u0 = ph[0][s].x, u1 = ph[0][s].y, u2 = ph[1][s].x;
    const T w0 = ph[1][s].y, w1 = ph[2][s].x, w2 = ph[2][s].y;
    z01[s] = {(u1 * w2 - u2 * w1) * scale, (u2 * w0 - u0 * w2) * scale};
    z2[s] = {(u0 * w1 - u1 * w0) * scale, T(0)};
  });
  Plan::template fft<T, -1>(z2, j, lds, tw);
  Plan::template fft<T, -1>(z01, j, lds, tw);
  // separate the two real transforms packed in z01:
  // C0_k = (Z_k + conj Z_{N-k})/2, C1_k = (Z_k - conj Z_{N-k})/(2i)
  static_for<0, R>([&](auto s) { lds.put(j + s * Tl, z01[s]); });
  lds.sync();
  if (valid) {
    cx<T>* o0 = A + base;
    cx<T>* o1 = A + csA + base;
    cx<T>* o2 = A + 2 * csA + base;
    static_for<0, R>([&](auto s) {
      const int k = j + s * Tl;
      if (k < Mz) {
        const cx<T> zk = lds.get(k);
        const cx<T> zm = lds.get((N - k) % N);
        o0[k] = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
        o1[k] = {T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
        o2[k] = z2[s];
      }
    });
  }
}

// ---------------------------------------------------------------------------
// Plain z transforms (the R2C / C2R operations).  The C2R pass applies the
// 1/N^3 of the inverse transform of Eq. ffteq (scale).
// ---------------------------------------------------------------------------
template <typename T, class Plan>
__global__ __launch_bounds__(256) void k_z_c2r(const cx<T>* __restrict__ in, T* __restrict__ out,
                                               long nlines, Geo g, T scale) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  static_assert(64 % Tl == 0, "a z line must sit inside one wave");
  constexpr int LPB = 256 / Tl;
  __shared__ cx<T> sm[LPB * N];
  const int tid = threadIdx.x;
  const int li = tid / Tl, j = tid % Tl;
  const long line = (long)blockIdx.x * LPB + li;
  const bool valid = line < nlines;
  LdsLine<T> lds{sm + li * N};
  const cx<T>* a = in + (valid ? line * g.Mz : 0);
  cx<T> v[R];
  static_for<0, R>([&](auto s) {
    v[s] = valid ? completed_one<T, N>(a, j + s * Tl, g.Mz) : cx<T>{T(0), T(0)};
  });
  Plan::template fft<T, +1>(v, j, lds, twiddles<T, N>());
  if (valid) {
    T* o = out + line * N;
    static_for<0, R>([&](auto s) { o[j + s * Tl] = v[s].x * scale; });
  }
}

template <typename T, class Plan>
__global__ __launch_bounds__(256) void k_z_r2c(const T* __restrict__ in, cx<T>* __restrict__ out, long nlines,
                                               Geo g) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  static_assert(64 % Tl == 0, "a z line must sit inside one wave");
  constexpr int LPB = 256 / Tl;
  __shared__ cx<T> sm[LPB * N];
  const int tid = threadIdx.x;
  const int li = tid / Tl, j = tid % Tl;
  const long line = (long)blockIdx.x * LPB + li;
  const bool valid = line < nlines;
  LdsLine<T> lds{sm + li * N};
  const T* a = in + (valid ? line * N : 0);
  cx<T> v[R];
  static_for<0, R>([&](auto s) { v[s] = {valid ? a[j + s * Tl] : T(0), T(0)}; });
  Plan::template fft<T, -1>(v, j, lds, twiddles<T, N>());
  if (valid) {
    cx<T>* o = out + line * g.Mz;
    static_for<0, R>([&](auto s) {
      const int k = j + s * Tl;
      if (k < g.Mz) o[k] = v[s];
    });
  }
}

// ---------------------------------------------------------------------------
// Elementwise: projection, viscous term and the classical RK4 stage update.
//   du = Nh - k (k.Nh)/|k|^2 - nu |k|^2 Us      (Eq. NSfinal; k = 0: no pressure)
// Nh is already dealiased (compact storage holds retained modes only).
// mode 0..3: RK4 stage s with U0 = step start, U1 = stage input, Acc = sum:
//   s=0: Acc = U0 + dt/6 du,  U1 = U0 + dt/2 du   (stage input is U0)
//   s=1: Acc += dt/3 du,      U1 = U0 + dt/2 du
//   s=2: Acc += dt/3 du,      U1 = U0 + dt du
//   s=3: U0 = Acc + dt/6 du
// mode 4: plain right-hand side, Acc = du (stage input U0).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_rk_stage(const cx<T>* __restrict__ Nh, cx<T>* __restrict__ U0,
                                                  cx<T>* __restrict__ U1, cx<T>* __restrict__ Acc, long C,
                                                  Geo g, int mode, T nu, T dt) {
  const long stride = (long)gridDim.x * blockDim.x;
  const long MMz = (long)g.M * g.Mz;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < C; e += stride) {
    const int ix = (int)(e / MMz);
    const long r = e - ix * MMz;
    const int iy = (int)(r / g.Mz);
    const int kz = (int)(r - (long)iy * g.Mz);
    const int kxi = kwave(cpos(ix, g), g.N), kyi = kwave(cpos(iy, g), g.N);
    const int k2i = kxi * kxi + kyi * kyi + kz * kz;
    const T kx = T(kxi), ky = T(kyi), kzf = T(kz), k2 = T(k2i);
    const cx<T> n0 = Nh[e], n1 = Nh[C + e], n2 = Nh[2 * C + e];
    const cx<T>* us = (mode == 0 || mode == 4) ? U0 : U1;
    const cx<T> s0 = us[e], s1 = us[C + e], s2 = us[2 * C + e];
    cx<T> kn = {T(0), T(0)};
    if (k2i != 0) {
      const T inv = T(1) / k2;
      kn = (n0 * kx + n1 * ky + n2 * kzf) * inv;
    }
    const T vk = nu * k2;
    const cx<T> d0 = n0 - kn * kx - s0 * vk;
    const cx<T> d1 = n1 - kn * ky - s1 * vk;
    const cx<T> d2 = n2 - kn * kzf - s2 * vk;
    if (mode == 4) {
      Acc[e] = d0;
      Acc[C + e] = d1;
      Acc[2 * C + e] = d2;
      continue;
    }
    if (mode == 3) {
      const T h = dt / T(6);
      U0[e] = Acc[e] + d0 * h;
      U0[C + e] = Acc[C + e] + d1 * h;
      U0[2 * C + e] = Acc[2 * C + e] + d2 * h;
      continue;
    }
    const cx<T> a0 = U0[e], a1 = U0[C + e], a2 = U0[2 * C + e];
    const T ha = (mode == 0) ? dt / T(6) : dt / T(3);
    const T hu = (mode == 2) ? dt : dt / T(2);
    if (mode == 0) {
      Acc[e] = a0 + d0 * ha;
      Acc[C + e] = a1 + d1 * ha;
      Acc[2 * C + e] = a2 + d2 * ha;
    } else {
      Acc[e] = Acc[e] + d0 * ha;
      Acc[C + e] = Acc[C + e] + d1 * ha;
      Acc[2 * C + e] = Acc[2 * C + e] + d2 * ha;
    }
    U1[e] = a0 + d0 * hu;
    U1[C + e] = a1 + d1 * hu;
    U1[2 * C + e] = a2 + d2 * hu;
  }
}

// ---------------------------------------------------------------------------
// Canonical <-> compact.  Canonical: [3][N][N][N/2+1].  Compact: [3][M][M][Mz].
// Gather drops the modes outside the retained set (projection onto the
// Galerkin space); scatter writes zeros there.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gather(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, long C,
                                                Geo g) {
  const long stride = (long)gridDim.x * blockDim.x;
  const long Nh = g.N / 2 + 1;
  const long MMz = (long)g.M * g.Mz;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < 3 * C; e += stride) {
    const int c = (int)(e / C);
    const long r0 = e - c * C;
    const int ix = (int)(r0 / MMz);
    const long r = r0 - ix * MMz;
    const int iy = (int)(r / g.Mz);
    const int kz = (int)(r - (long)iy * g.Mz);
    const long src = (((long)c * g.N + cpos(ix, g)) * g.N + cpos(iy, g)) * Nh + kz;
    out[e] = in[src];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, long C,
                                                 Geo g) {
  const long stride = (long)gridDim.x * blockDim.x;
  const long Nh = g.N / 2 + 1;
  const long plane = (long)g.N * Nh;
  const long total = 3L * g.N * plane;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int c = (int)(e / ((long)g.N * plane));
    const long r0 = e - (long)c * g.N * plane;
    const int px = (int)(r0 / plane);
    const long r = r0 - px * plane;
    const int py = (int)(r / Nh);
    const int kz = (int)(r - (long)py * Nh);
    cx<T> v = {T(0), T(0)};
    if (kz < g.Mz && kept(px, g) && kept(py, g))
      v = in[(long)c * C + ((long)crow(px, g) * g.M + crow(py, g)) * g.Mz + kz];
    out[e] = v;
  }
}

}  // namespace hot
