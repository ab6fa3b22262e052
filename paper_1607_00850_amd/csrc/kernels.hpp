// Pass kernels of one evaluation of the right-hand side of Eq. NSfinal and of
// one classical RK4 stage, for one N^3 instance.
//
// Spectral data inside the library is "compact": only the retained modes are
// stored.  On the x and y axes the retained FFT positions are [0, lo) and
// [N-hi, N) (M = lo + hi rows; row i holds position i for i < lo and
// i + N - M above); on the half (z) axis they are kz in [0, Mz), stored with a
// row pitch Mzp >= Mz that keeps rows 128-byte aligned (the padding slots are
// never read or written).  With the 2/3 rule lo = K+1, hi = K, Mz = K+1 where
// K = floor((N-1)/3); with every mode kept (plain transforms) lo = N/2+1,
// hi = N/2-1, Mz = Mzp = N/2+1: the canonical half-spectrum layout itself.
//
// Per right-hand side (Eq. ffteq order: inverse x, y, z; forward z, y, x):
//   P1  x inverse, curl fused on load        U[3][M][M*Mzp]  -> A1[6][N][M*Mzp]
//   P2  y inverse                            A1[6][N][M][Mzp] -> A2[6][N][N][Mzp]
//   P3  z C2R, u x omega, z R2C              A2[6][N*N][Mzp] -> A2[0..3) (in place)
//   P4  y forward                            A2[3][N][N][Mzp] -> A1[3][N][M][Mzp]
//   P5  x forward                            A1[3][N][M*Mzp] -> Nh[3][M][M*Mzp]
//   E   projection/viscous/RK4 stage         Nh, U0, U1, Acc (compact, elementwise)
#pragma once

#include "fft_core.hpp"

namespace hot {

struct Geo {
  int N;
  int lo, hi, M;  // x and y axes
  int Mz;         // retained z (half-axis) modes
  int Mzp;        // z pitch of compact arrays (>= Mz)
  int kz0;        // kz of local column 0: 0, or the first kz of a z-slab share
  int czp;        // z extent of the canonical in/out arrays: N/2+1, or a slab share's
  int tw;         // column tile of compact state arrays (cbase)
};

__device__ __forceinline__ bool kept(int p, const Geo& g) { return p < g.lo || p >= g.N - g.hi; }
// compact row of a retained position
__device__ __forceinline__ int crow(int p, const Geo& g) { return p < g.lo ? p : p - (g.N - g.M); }
// FFT position of compact row i
__device__ __forceinline__ int cpos(int i, const Geo& g) { return i < g.lo ? i : i + (g.N - g.M); }
// signed wavenumber (Eq. wavemesh) of FFT position p
__device__ __forceinline__ int kwave(int p, int N) { return 2 * p <= N ? p : p - N; }

// The 2/3-rule geometry of an N-point plan (|k| <= K = (N-1)/3, no row
// padding, row-major compact state), as compile-time values: a kernel that
// the launcher has checked runs on it (G23) gets every index as arithmetic on
// constants.
template <int N>
__device__ __forceinline__ Geo geo_two_thirds(Geo g) {
  constexpr int K = (N - 1) / 3;
  g.N = N;
  g.lo = K + 1;
  g.hi = K;
  g.M = 2 * K + 1;
  g.Mz = K + 1;
  g.Mzp = K + 1;
  g.kz0 = 0;
  g.tw = (2 * K + 1) * (K + 1);
  return g;
}

// Compact state arrays (per instance [3][C]: the state, the stage arrays, the
// nonlinear term and the implicit step's buffers) hold a component as column
// tiles: column q = (compact ky row) * Mzp + kz of compact kx row ix sits at
// cbase(q) + ix * tw, where cbase(q) = (q / tw) * M * tw + q mod tw.  With
// tw = 8 (FP32) or 4 (FP64) a tile's M rows are 64 bytes each and contiguous,
// so a pass along x over tw or more adjacent columns reads and writes whole
// runs of memory.  tw = M * Mzp (one tile) is the row-major [M][M][Mzp]
// layout, kept where Mzp is not a multiple of the tile.  Indices fit 32 bits
// (C < 2^32 for every planned size).
__device__ __forceinline__ long cbase(long q, const Geo& g) {
  const unsigned t = (unsigned)q / (unsigned)g.tw;
  return (long)t * ((long)g.M * g.tw) + (long)((unsigned)q - t * (unsigned)g.tw);
}

// Compact element e of one component: its wavenumbers, or false for row
// padding.
struct ModeK {
  int kx, ky, kz;
};
__device__ __forceinline__ bool mode_of(long e, const Geo& g, ModeK& m) {
  const unsigned tw = (unsigned)g.tw, MT = (unsigned)g.M * tw;
  const unsigned ue = (unsigned)e;
  const unsigned tile = ue / MT;
  const unsigned r = ue - tile * MT;
  const unsigned ix = r / tw;
  const unsigned q = tile * tw + (r - ix * tw);
  const unsigned iy = q / (unsigned)g.Mzp;
  m.kz = (int)(q - iy * (unsigned)g.Mzp);
  if (m.kz >= g.Mz) return false;
  m.kz += g.kz0;
  m.kx = kwave(cpos((int)ix, g), g.N);
  m.ky = kwave(cpos((int)iy, g), g.N);
  return true;
}

// Stores of pass outputs: streamed (non-temporal), since no kernel re-reads
// them while they could still sit in a cache.  (Measured on MI355X: faster
// for the passes that write every row; the compacting forward passes are
// faster with plain stores, see store_out.)
template <typename T>
__device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

template <bool NT, typename T>
__device__ __forceinline__ void store_out(cx<T>* p, cx<T> v) {
  if constexpr (NT) store_stream(p, v);
  else *p = v;
}

// Block barrier that orders LDS accesses only (global loads in flight stay in
// flight across it).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS view for a tile of W interleaved columns (strided passes).  Positions
// are XOR-swizzled in their low two bits by bits 4-5 so that the first-stage
// writes of neighbouring lanes (r positions apart) fall in different banks.
template <typename T, int N, int W>
struct LdsCols {
  cx<T>* base;
  int c;
  static constexpr bool kSwz = (N % 64 == 0);
  __device__ __forceinline__ static int sw(int p) { return kSwz ? (p ^ ((p >> 4) & 3)) : p; }
  __device__ __forceinline__ void put(int pos, cx<T> v) { base[sw(pos) * W + c] = v; }
  __device__ __forceinline__ cx<T> get(int pos) const { return base[sw(pos) * W + c]; }
  __device__ __forceinline__ void sync() { lds_barrier(); }
};

// LDS view for one contiguous line owned by a lane group (inside one wave,
// or whole waves of the block when BLOCK).  First-stage writes of
// neighbouring lanes are 2^SH positions apart: for SH >= 4 bits 0-3 of the
// position are XOR-ed with the low bits of the 2^SH-block index, below that
// one padding slot follows every 2^SH positions.
template <typename T, int SH, bool BLOCK>
struct LdsLine {
  cx<T>* base;
  __device__ __forceinline__ static int sw(int p) {
    // first radix >= 16: a permutation inside each aligned 16-position block
    // (no padding).  Measured on z_cross: a fifth of the bank-conflict cycles
    // of the earlier XOR of bits 1-3, and that one beat padding by 1-3%.
    if constexpr (SH >= 4) return p ^ ((p >> SH) & 15);
    else return p + (p >> SH);
  }
  __device__ __forceinline__ void put(int pos, cx<T> v) { base[sw(pos)] = v; }
  __device__ __forceinline__ cx<T> get(int pos) const { return base[sw(pos)]; }
  __device__ __forceinline__ void sync() {
    if constexpr (BLOCK) lds_barrier();
    else wave_sync();
  }
};

// z kernels run 256-thread blocks; a line is held by Tl lanes that either sit
// inside one wave (floor(64/Tl) lines per wave; leftover lanes idle) or span
// whole waves (block barriers).  Idle lanes work on a private dummy line.
template <class Plan>
struct ZShape {
  static constexpr int Tl = Plan::Tl;
  static_assert(Tl <= 64 || (Tl % 64 == 0 && 256 % Tl == 0), "unsupported z line shape");
  static constexpr bool kBlock = Tl > 64;
  static constexpr int LPW = kBlock ? 1 : 64 / Tl;        // lines per wave
  static constexpr int LPB = kBlock ? 256 / Tl : 4 * LPW;  // lines per block
  static constexpr bool kIdle = !kBlock && LPW * Tl < 64;  // lanes without a line
  static constexpr int SLOTS = LPB + (kIdle ? 4 : 0);      // + one dummy line per wave
  // line slot and lane index of thread tid; live == false for idle lanes
  __device__ __forceinline__ static void place(int tid, int& li, int& j, bool& live) {
    if constexpr (kBlock) {
      li = tid / Tl;
      j = tid % Tl;
      live = true;
    } else {
      const int w = tid >> 6, lane = tid & 63;
      const int l = lane / Tl;
      live = l < LPW;
      li = live ? w * LPW + l : LPB + w;
      j = lane % Tl;
    }
  }
};

// Copy the plan's stage-major twiddles into LDS (once per block).
template <typename T, class Plan>
__device__ __forceinline__ void stage_twiddles(cx<T>* tws) {
  const cx<T>* tab = g_stage_tw<T, Plan>.w;
  for (int e = threadIdx.x; e < Plan::N; e += blockDim.x) tws[e] = tab[e];
}

// The same in two halves for blocks of NT threads: fetch() issues the loads,
// put() writes LDS.  Issuing the pass's data loads in between keeps the two
// sets of loads in flight together.
template <typename T, class Plan, int NT>
struct TwStage {
  static constexpr int K = (Plan::N + NT - 1) / NT;
  cx<T> r[K];
  __device__ __forceinline__ void fetch(int tid) {
    const cx<T>* tab = g_stage_tw<T, Plan>.w;
    static_for<0, K>([&](auto t) {
      const int e = tid + t * NT;
      r[t] = tab[e < Plan::N ? e : 0];
    });
  }
  __device__ __forceinline__ void put(cx<T>* tws, int tid) const {
    static_for<0, K>([&](auto t) {
      const int e = tid + t * NT;
      if (e < Plan::N) tws[e] = r[t];
    });
  }
};

// Tile of block b when PAIR consecutive tiles share one 128-byte row segment:
// the tiles of a segment go to blocks with equal b mod 8 (one XCD, one L2),
// back to back, so the L2 merges their half-line reads and writes.
template <int PAIR>
__device__ __forceinline__ long tile_of_block(long b) {
  if constexpr (PAIR == 1) {
    return b;
  } else {
    const long xcd = b & 7, slot = b >> 3;
    return ((slot / PAIR) * 8 + xcd) * PAIR + (slot % PAIR);
  }
}

// ---------------------------------------------------------------------------
// Strided axis pass: columns are contiguous, lines run along rows.
// The array is a batch of [rows][Qp] blocks (global column gc = b*Qp + q);
// a column is live iff (q mod Mzp) < Mz (the rest is row padding).
// IN_C / OUT_C: rows are compact (retained positions only) or all N.
// otw > 0 (with OUT_C): the output is a compact state array (cbase), its
// columns in tiles of otw and its rows otw apart (ld_out = otw).
// blockIdx.y selects the component (stride cs_*), blockIdx.z the instance of
// a batch of equal-size instances (stride is_*).
// ---------------------------------------------------------------------------
template <typename T, class Plan, int DIR, int W, bool IN_C, bool OUT_C>
__global__ __launch_bounds__(W* Plan::Tl) void k_strided(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                         long ncols, long Qp, long ld_in, long ld_out, long bs_in,
                                                         long bs_out, long cs_in, long cs_out, long is_in,
                                                         long is_out, long otw, Geo g, const int* __restrict__ act) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[N * W];
  __shared__ cx<T> tws[N];
  const long tile = tile_of_block<PAIR>(blockIdx.x);
  if (tile * W >= ncols) return;          // whole block leaves together
  if (act && !act[blockIdx.z]) return;  // instance no longer iterating
  const int tid = threadIdx.x;
  // the stage twiddles go to LDS; the first exchange barrier orders them
  // before their first use
  TwStage<T, Plan, W * Tl> tw;
  tw.fetch(tid);
  const int c = tid % W, j = tid / W;
  const long gc = tile * W + c;
  const long b = gc / Qp;
  const long q = gc - b * Qp;
  const bool valid = gc < ncols && (int)(q % g.Mzp) < g.Mz;
  // blockIdx.y: component, blockIdx.z: instance of a batch
  const long ib = valid ? blockIdx.z * is_in + blockIdx.y * cs_in + b * bs_in + q : 0;
  // otw > 0: the output is a compact state array, its columns in tiles of otw
  // (cbase; ld_out is then otw)
  const long oq = otw > 0 ? (q / otw) * ((long)g.M * otw) + q % otw : q;
  const long ob = valid ? blockIdx.z * is_out + blockIdx.y * cs_out + b * bs_out + oq : 0;
  cx<T> v[R];
  static_for<0, R>([&](auto s) {
    const int p = j + s * Tl;
    // branch-free: load from a valid address, select afterwards
    if (IN_C) {
      const bool kp = valid && kept(p, g);
      const cx<T> x = in[ib + (kp ? (long)crow(p, g) * ld_in : 0)];
      v[s] = kp ? x : cx<T>{T(0), T(0)};
    } else {
      const cx<T> x = in[ib + (valid ? (long)p * ld_in : 0)];
      v[s] = valid ? x : cx<T>{T(0), T(0)};
    }
  });
  tw.put(tws, tid);
  LdsCols<T, N, W> lds{sm, c};
  Plan::template fft<T, DIR>(v, j, lds, TwTab<T>{tws});
  static_for<0, R>([&](auto s) {
    const int p = j + s * Tl;
    if (OUT_C) {
      if (valid && kept(p, g)) store_out<false>(out + ob + (long)crow(p, g) * ld_out, v[s]);
    } else {
      if (valid) store_out<PAIR == 1>(out + ob + (long)p * ld_out, v[s]);
    }
  });
}

// ---------------------------------------------------------------------------
// P1: inverse transform along x of the velocity and of the vorticity
// omega_hat = i k x u_hat (curl fused into the load).  Input compact state
// U[3][M rows (kx)][Q = M*Mzp cols (ky,kz)], output A[6][N rows (x)][Q] with
// components (u_x, u_y, u_z, w_x, w_y, w_z).  Every output carries the factor
// usc = 1/N^3 of the inverse transform of Eq. ffteq, so the z pass multiplies
// nothing (u and w enter its cross product already normalised; they share
// complex lines there, so they must share the scale too).
// One block per (tile, output component); the 6 components of a tile go to
// blocks with equal b mod 8 (one XCD) so that their shared input rows are
// read from HBM once and then served by that XCD's L2.  blockIdx.y is the
// instance of a batch.
// ---------------------------------------------------------------------------
template <typename T, class Plan, int W>
__global__ __launch_bounds__(W* Plan::Tl) void k_x_inv_curl(const cx<T>* __restrict__ U, long csU, long isU,
                                                            cx<T>* __restrict__ A, long csA, long isA,
                                                            int ntiles, Geo g, T usc, const int* __restrict__ act) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[N * W];
  __shared__ cx<T> tws[N];
  const int blk = blockIdx.x;
  const int xcd = blk & 7, slot = blk >> 3;
  const int o = slot % 6;
  const int rest = slot / 6;
  const int tile = ((rest / PAIR) * 8 + xcd) * PAIR + rest % PAIR;
  if (tile >= ntiles) return;           // whole block leaves together
  if (act && !act[blockIdx.y]) return;  // instance no longer iterating
  const int tid = threadIdx.x;
  TwStage<T, Plan, W * Tl> tw;  // to LDS, ordered before use by the first exchange barrier
  tw.fetch(tid);
  const int c = tid % W, j = tid / W;
  const long Q = (long)g.M * g.Mzp;
  const long q = (long)tile * W + c;
  const int iy = (int)(q / g.Mzp);
  const int kz = (int)(q - (long)iy * g.Mzp);
  const bool valid = q < Q && kz < g.Mz;
  const T ky = T(kwave(cpos(valid ? iy : 0, g), N));
  const T kzf = T(kz + g.kz0);
  const long qq = valid ? q : 0;
  U += blockIdx.y * isU;  // instance of a batch
  A += blockIdx.y * isA;
  // Velocity outputs read one component; vorticity outputs two:
  //   w_x = i (ky u_z - kz u_y), w_y = i (kz u_x - kx u_z), w_z = i (kx u_y - ky u_x).
  // Every lane loads from a valid address (row 0 when the position is not
  // retained) and selects afterwards, so that the loads carry no branches and
  // are all in flight together.
  const int ca = o < 3 ? o : (o == 3 ? 2 : (o == 4 ? 0 : 1));
  const int cb = o == 3 ? 1 : (o == 4 ? 2 : 0);
  const long ub = cbase(qq, g);
  const cx<T>* pa = U + ca * csU + ub;
  const cx<T>* pb = U + cb * csU + ub;
  cx<T> v[R];
  if (o < 3) {
    static_for<0, R>([&](auto s) {
      const int p = j + s * Tl;
      const bool kp = valid && kept(p, g);
      const cx<T> x = pa[kp ? (long)crow(p, g) * g.tw : 0];
      v[s] = kp ? x * usc : cx<T>{T(0), T(0)};
    });
  } else {
    static_for<0, R>([&](auto s) {
      const int p = j + s * Tl;
      const bool kp = valid && kept(p, g);
      const long off = kp ? (long)crow(p, g) * g.tw : 0;
      const cx<T> a = pa[off], b = pb[off];
      const T kx = T(kwave(p, N));
      const T fa = (o == 3 ? ky : (o == 4 ? kzf : kx)) * usc;
      const T fb = (o == 3 ? kzf : (o == 4 ? kx : ky)) * usc;
      v[s] = kp ? mul_i(a * fa - b * fb) : cx<T>{T(0), T(0)};
    });
  }
  tw.put(tws, tid);
  LdsCols<T, N, W> lds{sm, c};
  Plan::template fft<T, +1>(v, j, lds, TwTab<T>{tws});
  if (valid) {
    cx<T>* dst = A + o * csA + q;
    static_for<0, R>([&](auto s) { store_out<PAIR == 1>(dst + (long)(j + s * Tl) * Q, v[s]); });
  }
}

// Registers of a column that can hold a retained row: with lo, hi <= KL Tl
// the rows j + s Tl with KL <= s < R - KL lie in [lo, N - hi) for every lane
// j, so they are never loaded and their values are zero at compile time.
template <class Plan, int KL>
constexpr bool col_live(int s) {
  return s < KL || s >= Plan::R - KL;
}

// P1 with three blocks per tile: block m in {0, 1, 2} loads u_m and u_{m+1}
// (indices mod 3) and writes w_{m+2} = i (k_m u_{m+1} - k_{m+1} u_m), then
// u_m (the cyclic form of w = i k x u: w_z = i (kx u_y - ky u_x), w_x =
// i (ky u_z - kz u_y), w_y = i (kz u_x - kx u_z)).  Six component loads per
// tile instead of nine, and half as many blocks as k_x_inv_curl.  The three
// blocks of a tile go to one XCD, so each input row comes from HBM once.
// KL: retained rows reach at most KL registers from either end (col_live).
template <typename T, class Plan, int W, int KL>
__global__ __launch_bounds__(W* Plan::Tl) void k_x_inv_curl3(const cx<T>* __restrict__ U, long csU, long isU,
                                                             cx<T>* __restrict__ A, long csA, long isA,
                                                             int ntiles, Geo g, T usc, const int* __restrict__ act) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[N * W];
  __shared__ cx<T> tws[N];
  const int blk = blockIdx.x;
  const int xcd = blk & 7, slot = blk >> 3;
  const int m = slot % 3;
  const int rest = slot / 3;
  const int tile = ((rest / PAIR) * 8 + xcd) * PAIR + rest % PAIR;
  if (tile >= ntiles) return;           // whole block leaves together
  if (act && !act[blockIdx.y]) return;  // instance no longer iterating
  const int tid = threadIdx.x;
  TwStage<T, Plan, W * Tl> tw;  // to LDS, ordered before use by the first exchange barrier
  tw.fetch(tid);
  const int c = tid % W, j = tid / W;
  const long Q = (long)g.M * g.Mzp;
  const long q = (long)tile * W + c;
  const int iy = (int)(q / g.Mzp);
  const int kz = (int)(q - (long)iy * g.Mzp);
  const bool valid = q < Q && kz < g.Mz;
  const T ky = T(kwave(cpos(valid ? iy : 0, g), N));
  const T kzf = T(kz + g.kz0);
  const long qq = valid ? q : 0;
  U += blockIdx.y * isU;  // instance of a batch
  A += blockIdx.y * isA;
  const int m1 = m == 2 ? 0 : m + 1;
  const long ub = cbase(qq, g);
  const cx<T>* pa = U + m * csU + ub;
  const cx<T>* pb = U + m1 * csU + ub;
  // every lane loads from a valid address (row 0 when the position is not
  // retained) and selects afterwards: no branches around the loads
  cx<T> a[R], v[R];
  static_for<0, R>([&](auto s) {
    if constexpr (col_live<Plan, KL>(s)) {
      const int p = j + s * Tl;
      const bool kp = valid && kept(p, g);
      const long off = kp ? (long)crow(p, g) * g.tw : 0;
      const cx<T> x = pa[off], y = pb[off];
      const T kx = T(kwave(p, N));
      const T km = (m == 0 ? kx : (m == 1 ? ky : kzf)) * usc;
      const T kn = (m == 0 ? ky : (m == 1 ? kzf : kx)) * usc;
      a[s] = kp ? x * usc : cx<T>{T(0), T(0)};
      v[s] = kp ? mul_i(y * km - x * kn) : cx<T>{T(0), T(0)};
    } else {
      a[s] = cx<T>{T(0), T(0)};
      v[s] = cx<T>{T(0), T(0)};
    }
  });
  tw.put(tws, tid);
  LdsCols<T, N, W> lds{sm, c};
  const int ow = m == 0 ? 5 : (m == 1 ? 3 : 4);  // w_z, w_x, w_y
  Plan::template fft<T, +1>(v, j, lds, TwTab<T>{tws});
  if (valid) {
    cx<T>* dst = A + ow * csA + q;
    static_for<0, R>([&](auto s) { store_out<PAIR == 1>(dst + (long)(j + s * Tl) * Q, v[s]); });
  }
  Plan::template fft<T, +1>(a, j, lds, TwTab<T>{tws});
  if (valid) {
    cx<T>* dst = A + m * csA + q;
    static_for<0, R>([&](auto s) { store_out<PAIR == 1>(dst + (long)(j + s * Tl) * Q, a[s]); });
  }
}

// P1 for short lines: one block computes all six outputs of a tile (u_c, then
// w_c = i (k x u)_c) from a single load of the three velocity components,
// transforming them one after another through the same LDS tile.  Six times
// fewer blocks than k_x_inv_curl and three component loads per tile instead
// of nine.  No barrier is needed between two transforms: every exchange ends
// with one after its reads, and the last stage works in registers.
// One tile of instance `inst`, run by the W * Tl threads of a block (tid)
// with sm = N * W + N values of LDS (the exchange tile, then the stage
// twiddles).  k_x_inv_curl6 runs one tile per block; the persistent batch
// kernel calls it for its work items.
template <typename T, class Plan, int W, bool G23 = false>
__device__ __forceinline__ void x_inv_curl6_tile(const cx<T>* __restrict__ U, long csU, long isU,
                                                 cx<T>* __restrict__ A, long csA, long isA, int tile, int inst,
                                                 int tid, const Geo& g_in, T usc, cx<T>* sm) {
  const Geo g = G23 ? geo_two_thirds<Plan::N>(g_in) : g_in;
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  cx<T>* tws = sm + N * W;
  TwStage<T, Plan, W * Tl> tw;  // to LDS, ordered before use by the first exchange barrier
  tw.fetch(tid);
  const int c = tid % W, j = tid / W;
  const long Q = (long)g.M * g.Mzp;
  const long q = (long)tile * W + c;
  const int iy = (int)(q / g.Mzp);
  const int kz = (int)(q - (long)iy * g.Mzp);
  const bool valid = q < Q && kz < g.Mz;
  const T ky = T(kwave(cpos(valid ? iy : 0, g), N));
  const T kzf = T(kz + g.kz0);
  const long qq = valid ? q : 0;
  U += inst * isU;
  A += inst * isA;
  const long ub = cbase(qq, g);
  cx<T> u[3][R];
  static_for<0, 3>([&](auto comp) {
    static_for<0, R>([&](auto s) {
      const int p = j + s * Tl;
      const bool kp = valid && kept(p, g);
      const cx<T> x = U[comp * csU + ub + (kp ? (long)crow(p, g) * g.tw : 0)];
      u[comp][s] = kp ? x * usc : cx<T>{T(0), T(0)};
    });
  });
  tw.put(tws, tid);
  LdsCols<T, N, W> lds{sm, c};
  static_for<0, 6>([&](auto o) {
    cx<T> v[R];
    static_for<0, R>([&](auto s) {
      if constexpr (o < 3) {
        v[s] = u[o][s];
      } else {
        const T kx = T(kwave(j + s * Tl, N));
        // w_x = i (ky u_z - kz u_y), w_y = i (kz u_x - kx u_z), w_z = i (kx u_y - ky u_x)
        if constexpr (o == 3) v[s] = mul_i(u[2][s] * ky - u[1][s] * kzf);
        else if constexpr (o == 4) v[s] = mul_i(u[0][s] * kzf - u[2][s] * kx);
        else v[s] = mul_i(u[1][s] * kx - u[0][s] * ky);
      }
    });
    Plan::template fft<T, +1>(v, j, lds, TwTab<T>{tws});
    if (valid) {
      cx<T>* dst = A + o * csA + q;
      static_for<0, R>([&](auto s) { store_out<PAIR == 1>(dst + (long)(j + s * Tl) * Q, v[s]); });
    }
  });
}

template <typename T, class Plan, int W, bool G23 = false>
__global__ __launch_bounds__(W* Plan::Tl) void k_x_inv_curl6(const cx<T>* __restrict__ U, long csU, long isU,
                                                             cx<T>* __restrict__ A, long csA, long isA,
                                                             int ntiles, Geo g_in, T usc, const int* __restrict__ act) {
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[Plan::N * W + Plan::N];
  const int blk = blockIdx.x;
  const int xcd = blk & 7, rest = blk >> 3;
  const int tile = ((rest / PAIR) * 8 + xcd) * PAIR + rest % PAIR;
  if (tile >= ntiles) return;           // whole block leaves together
  if (act && !act[blockIdx.y]) return;  // instance no longer iterating
  x_inv_curl6_tile<T, Plan, W, G23>(U, csU, isU, A, csA, isA, tile, blockIdx.y, threadIdx.x, g_in, usc, sm);
}

// ---------------------------------------------------------------------------
// z-axis lines.  A group of Tl = N/R lanes owns one line (see ZShape).
// ---------------------------------------------------------------------------

// Number of compact z coefficients a lane loads when Mz coefficients are kept.
template <class Plan>
constexpr int z_loads(int Mz = Plan::N / 2 + 1) {
  return (Mz + Plan::Tl - 1) / Plan::Tl;
}

// Lay out Z_p = a_p + i b_p on the full circle in the line's LDS region from
// the half-spectrum pair (a, b) held as lane j's coefficients k = j + t*Tl:
// Z_k = a_k + i b_k and Z_{N-k} = conj(a_k) + i conj(b_k).  As in a real
// inverse transform, the imaginary parts of the kz = 0 and kz = N/2
// coefficients are dropped.  Positions no coefficient reaches read as zero in
// read_completed().
template <typename T, class Plan, int KL, class L>
__device__ __forceinline__ void put_completed(L& lds, const cx<T> (&la)[KL], const cx<T> (&lb)[KL], int j, int Mz) {
  constexpr int N = Plan::N, Tl = Plan::Tl;
  static_for<0, KL>([&](auto t) {
    const int k = j + t * Tl;
    if (k < Mz) {
      cx<T> x = la[t], y = lb[t];
      if (k == 0 || 2 * k == N) {
        x.y = T(0);
        y.y = T(0);
      }
      lds.put(k, cx<T>{x.x - y.y, x.y + y.x});
      if (k > 0 && 2 * k < N) lds.put(N - k, cx<T>{x.x + y.y, y.x - x.y});
    }
  });
}

// With at most KL coefficients per lane (Mz <= KL Tl), the registers s whose
// positions j + s Tl lie in [KL Tl, N - KL Tl] for every lane are zero
// without a read; the others read their position (inside the line's region)
// and keep it where a coefficient reaches.
template <typename T, class Plan, int KL = Plan::R, class L>
__device__ __forceinline__ void read_completed(const L& lds, cx<T>* v, int j, int Mz) {
  constexpr int N = Plan::N, Tl = Plan::Tl;
  static_for<0, Plan::R>([&](auto s) {
    constexpr bool dead = s * Tl >= KL * Tl && (s + 1) * Tl - 1 <= N - KL * Tl;
    if constexpr (dead) {
      v[s] = cx<T>{T(0), T(0)};
    } else {
      const int p = j + s * Tl;
      const bool live = (p < Mz) || (N - p < Mz);
      const cx<T> t = lds.get(p);
      v[s] = live ? t : cx<T>{T(0), T(0)};
    }
  });
}

// Where coefficient k of a z line sits, relative to the line's first slot.
// ZContig: the line is one row, k at offset k.  ZBlocked: the line arrives in
// chunks of `chunk` coefficients, chunk c in the block written by z-slab
// share c (blocks `blk` elements apart, the line at the same offset in each),
// as an all-to-all between slab shares delivers it.
struct ZContig {
  __device__ __forceinline__ long operator()(int k) const { return k; }
};
struct ZBlocked {
  int chunk;
  float inv;  // 1 / chunk
  long blk;
  __device__ __forceinline__ long operator()(int k) const {
    // exact: k + 1/2 stays at least 1/(2 chunk) away from every multiple of
    // chunk, far beyond the float rounding of the product for k < 2^16
    const int c = (int)((float(k) + 0.5f) * inv);
    return (long)c * blk + (k - c * chunk);
  }
};

// Coalesced load of a compact z line: lane j takes k = j + t*Tl (k < Mz).
template <typename T, class Plan, int KL, class ZA = ZContig>
__device__ __forceinline__ void load_line(cx<T> (&la)[KL], const cx<T>* __restrict__ a, int j, int Mz, bool valid,
                                          ZA za = ZA{}) {
  static_for<0, KL>([&](auto t) {
    const int k = j + t * Plan::Tl;
    la[t] = (valid && k < Mz) ? a[za(k)] : cx<T>{T(0), T(0)};
  });
}

// ---------------------------------------------------------------------------
// P3: per z-line, inverse real transforms of u and omega (three complex FFTs,
// two real lines each), the cross product c = u x omega (component formula of
// Sec. 3.4; both factors already carry the 1/N^3 of Eq. ffteq, applied by
// the x pass), and the forward real transform of c (c0 + i c1 in one FFT,
// c2 in another).
// In place: reads components 0..5 of the line, writes 0..2.  The loads of the
// next component pair are issued before the current pair's FFT.  ZA places
// the coefficients of a line (ZContig: one row; ZBlocked: the chunks of a
// z-slab all-to-all).
// ---------------------------------------------------------------------------
template <typename T, class Plan, int KL, class ZA>
__global__ __launch_bounds__(256) void k_z_cross(cx<T>* __restrict__ A, long csA, long isA, long nlines, Geo g,
                                                 const int* __restrict__ act, ZA za) {
  if (act && !act[blockIdx.y]) return;  // instance no longer iterating
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int LPB = ZShape<Plan>::LPB;
  constexpr int LS = Plan::line_stride;
  __shared__ cx<T> sm[ZShape<Plan>::SLOTS * LS];
  __shared__ cx<T> tws[N];
  TwStage<T, Plan, 256> twst;
  twst.fetch(threadIdx.x);
  int li, j;
  bool live;
  ZShape<Plan>::place(threadIdx.x, li, j, live);
  const long line = (long)blockIdx.x * LPB + li;
  const bool valid = live && line < nlines;
  const int Mz = g.Mz;  // the launcher guarantees Mz <= KL * Tl
  LdsLine<T, Plan::SH, ZShape<Plan>::kBlock> lds{sm + li * LS};
  const TwTab<T> tw{tws};
  const long base = valid ? line * g.Mzp : 0;
  A += blockIdx.y * isA;  // instance of a batch

  cx<T> la[KL], lb[KL];
  load_line<T, Plan, KL>(la, A + base, j, Mz, valid, za);
  load_line<T, Plan, KL>(lb, A + csA + base, j, Mz, valid, za);
  // twiddles to LDS while the line loads are in flight (an LDS-only barrier
  // leaves them in flight)
  twst.put(tws, threadIdx.x);
  lds_barrier();
  cx<T> ph[3][R];
  static_for<0, 3>([&](auto pr) {
    put_completed<T, Plan, KL>(lds, la, lb, j, Mz);
    lds.sync();
    read_completed<T, Plan, KL>(lds, ph[pr], j, Mz);
    lds.sync();
    if constexpr (pr < 2) {
      load_line<T, Plan, KL>(la, A + (2 * pr + 2) * csA + base, j, Mz, valid, za);
      load_line<T, Plan, KL>(lb, A + (2 * pr + 3) * csA + base, j, Mz, valid, za);
    }
    Plan::template fft<T, +1>(ph[pr], j, lds, tw);
  });
  // u = (ph0.x, ph0.y, ph1.x), omega = (ph1.y, ph2.x, ph2.y)
  cx<T> z01[R], z2[R];
  static_for<0, R>([&](auto s) {
    const T u0 = ph[0][s].x, u1 = ph[0][s].y, u2 = ph[1][s].x;
    const T w0 = ph[1][s].y, w1 = ph[2][s].x, w2 = ph[2][s].y;
    z01[s] = {u1 * w2 - u2 * w1, u2 * w0 - u0 * w2};
    z2[s] = {u0 * w1 - u1 * w0, T(0)};
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
        const long ok = za(k);
        store_stream(o0 + ok, cx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)});
        store_stream(o1 + ok, cx<T>{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)});
        store_stream(o2 + ok, z2[s]);
      }
    });
  }
}

// ---------------------------------------------------------------------------
// Packed pair rows.  A real z line f has the half spectrum f_k, k < Mz; two
// real lines a, b travel through one complex transform as Z = a + i b, whose
// spectrum on the full circle is Z_k = a_k + i b_k and Z_{N-k} =
// conj(a_k) + i conj(b_k).  With packed rows the two halves of that circle
// are stored as two rows of the same shape as a half spectrum:
//   row A[k] = Z_k = a_k + i b_k,   row B[k] = Z_{N-k} = conj(a_k) + i conj(b_k),
// k < Mz (at k = 0 the imaginary parts of a_0 and b_0 are dropped, as in any
// real inverse transform).  The y inverse pass writes them for the pairs
// (u_x, u_y), (u_z, w_x), (w_y, w_z) in place of the six components, so the
// z pass loads each complex line straight into its transform registers, with
// no Hermitian completion in LDS; after the forward transform of
// c0 + i c1 the z pass stores the two halves of its circle the same way, and
// the y forward pass separates c0_k = (A_k + conj B_k)/2 and
// c1_k = (A_k - conj B_k)/(2i) on load.  The bytes moved are those of six
// (three) component rows, as before.
// ---------------------------------------------------------------------------

// y inverse on pairs: component pair P = blockIdx.y (inputs 2P, 2P+1 of the
// compact-row array), transformed along the columns' rows, written as the
// packed rows A (component 2P) and B (component 2P + 1).  Arguments as
// k_strided with IN_C = true, OUT_C = false; KL as col_live.
template <typename T, class Plan, int W, int KL>
__global__ __launch_bounds__(W* Plan::Tl) void k_y_inv_pack(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                            long ncols, long Qp, long ld_in, long ld_out, long bs_in,
                                                            long bs_out, long cs_in, long cs_out, long is_in,
                                                            long is_out, Geo g, const int* __restrict__ act) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[N * W];
  __shared__ cx<T> tws[N];
  const long tile = tile_of_block<PAIR>(blockIdx.x);
  if (tile * W >= ncols) return;          // whole block leaves together
  if (act && !act[blockIdx.z]) return;  // instance no longer iterating
  const int tid = threadIdx.x;
  TwStage<T, Plan, W * Tl> tw;
  tw.fetch(tid);
  const int c = tid % W, j = tid / W;
  const long gc = tile * W + c;
  const long b = gc / Qp;
  const long q = gc - b * Qp;
  const int kz = (int)(q % g.Mzp);
  const bool valid = gc < ncols && kz < g.Mz;
  const long pc = 2 * (long)blockIdx.y;
  const long ib = valid ? blockIdx.z * is_in + pc * cs_in + b * bs_in + q : 0;
  const long ob = valid ? blockIdx.z * is_out + pc * cs_out + b * bs_out + q : 0;
  cx<T> va[R], vb[R];
  static_for<0, R>([&](auto s) {
    if constexpr (col_live<Plan, KL>(s)) {
      const int p = j + s * Tl;
      const bool kp = valid && kept(p, g);
      const long off = ib + (kp ? (long)crow(p, g) * ld_in : 0);
      const cx<T> x = in[off], y = in[off + cs_in];
      va[s] = kp ? x : cx<T>{T(0), T(0)};
      vb[s] = kp ? y : cx<T>{T(0), T(0)};
    } else {
      va[s] = cx<T>{T(0), T(0)};
      vb[s] = cx<T>{T(0), T(0)};
    }
  });
  tw.put(tws, tid);
  LdsCols<T, N, W> lds{sm, c};
  Plan::template fft<T, +1>(va, j, lds, TwTab<T>{tws});
  Plan::template fft<T, +1>(vb, j, lds, TwTab<T>{tws});
  if (!valid) return;
  const bool k0 = kz + g.kz0 == 0;  // a real line's k = 0 coefficient is real
  static_for<0, R>([&](auto s) {
    cx<T> a = va[s], e = vb[s];
    if (k0) {
      a.y = T(0);
      e.y = T(0);
    }
    const long o = ob + (long)(j + s * Tl) * ld_out;
    store_out<PAIR == 1>(out + o, cx<T>{a.x - e.y, a.y + e.x});
    store_out<PAIR == 1>(out + o + cs_out, cx<T>{a.x + e.y, e.x - a.y});
  });
}

// y forward from packed rows: blockIdx.y = 0 separates c0, c1 from rows A
// (component 0) and B (component 1) on load and transforms both, into
// components 0 and 1; blockIdx.y = 1 transforms component 2.  Arguments as
// k_strided with IN_C = false, OUT_C = true; KL as col_live (output rows).
template <typename T, class Plan, int W, int KL>
__global__ __launch_bounds__(W* Plan::Tl) void k_y_fwd_unpack(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                              long ncols, long Qp, long ld_in, long ld_out,
                                                              long bs_in, long bs_out, long cs_in, long cs_out,
                                                              long is_in, long is_out, Geo g,
                                                              const int* __restrict__ act) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[N * W];
  __shared__ cx<T> tws[N];
  const long tile = tile_of_block<PAIR>(blockIdx.x);
  if (tile * W >= ncols) return;          // whole block leaves together
  if (act && !act[blockIdx.z]) return;  // instance no longer iterating
  const int tid = threadIdx.x;
  TwStage<T, Plan, W * Tl> tw;
  tw.fetch(tid);
  const int c = tid % W, j = tid / W;
  const long gc = tile * W + c;
  const long b = gc / Qp;
  const long q = gc - b * Qp;
  const bool valid = gc < ncols && (int)(q % g.Mzp) < g.Mz;
  const bool pair = blockIdx.y == 0;
  const long pc = pair ? 0 : 2;
  const long ib = valid ? blockIdx.z * is_in + pc * cs_in + b * bs_in + q : 0;
  const long ob = valid ? blockIdx.z * is_out + pc * cs_out + b * bs_out + q : 0;
  LdsCols<T, N, W> lds{sm, c};
  if (pair) {
    cx<T> va[R], vb[R];
    static_for<0, R>([&](auto s) {
      const long off = ib + (valid ? (long)(j + s * Tl) * ld_in : 0);
      const cx<T> x = in[off], y = in[off + cs_in];
      // c0 = (A + conj B)/2, c1 = (A - conj B)/(2i)
      va[s] = valid ? cx<T>{T(0.5) * (x.x + y.x), T(0.5) * (x.y - y.y)} : cx<T>{T(0), T(0)};
      vb[s] = valid ? cx<T>{T(0.5) * (x.y + y.y), T(0.5) * (y.x - x.x)} : cx<T>{T(0), T(0)};
    });
    tw.put(tws, tid);
    Plan::template fft<T, -1>(va, j, lds, TwTab<T>{tws});
    Plan::template fft<T, -1>(vb, j, lds, TwTab<T>{tws});
    if (!valid) return;
    static_for<0, R>([&](auto s) {
      if constexpr (col_live<Plan, KL>(s)) {
        const int p = j + s * Tl;
        if (kept(p, g)) {
          const long o = ob + (long)crow(p, g) * ld_out;
          store_out<false>(out + o, va[s]);
          store_out<false>(out + o + cs_out, vb[s]);
        }
      }
    });
  } else {
    cx<T> v[R];
    static_for<0, R>([&](auto s) {
      const cx<T> x = in[ib + (valid ? (long)(j + s * Tl) * ld_in : 0)];
      v[s] = valid ? x : cx<T>{T(0), T(0)};
    });
    tw.put(tws, tid);
    Plan::template fft<T, -1>(v, j, lds, TwTab<T>{tws});
    if (!valid) return;
    static_for<0, R>([&](auto s) {
      if constexpr (col_live<Plan, KL>(s)) {
        const int p = j + s * Tl;
        if (kept(p, g)) store_out<false>(out + ob + (long)crow(p, g) * ld_out, v[s]);
      }
    });
  }
}

// The same with one output per block: block o of a tile (0: c0, 1: c1 from
// rows A and B; 2: c2) loads what it needs and runs one transform.  The three
// blocks of a tile are consecutive on one XCD, so the second read of rows A
// and B comes from its L2.  blockIdx.y is the instance of a batch.
template <typename T, class Plan, int W, int KL>
__global__ __launch_bounds__(W* Plan::Tl) void k_y_fwd_unpack3(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                               long ncols, long Qp, long ld_in, long ld_out,
                                                               long bs_in, long bs_out, long cs_in, long cs_out,
                                                               long is_in, long is_out, Geo g,
                                                               const int* __restrict__ act) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[N * W];
  __shared__ cx<T> tws[N];
  const int blk = blockIdx.x;
  const int xcd = blk & 7, slot = blk >> 3;
  const int o = slot % 3;
  const int rest = slot / 3;
  const long tile = ((long)(rest / PAIR) * 8 + xcd) * PAIR + rest % PAIR;
  if (tile * W >= ncols) return;          // whole block leaves together
  if (act && !act[blockIdx.y]) return;  // instance no longer iterating
  const int tid = threadIdx.x;
  TwStage<T, Plan, W * Tl> tw;
  tw.fetch(tid);
  const int c = tid % W, j = tid / W;
  const long gc = tile * W + c;
  const long b = gc / Qp;
  const long q = gc - b * Qp;
  const bool valid = gc < ncols && (int)(q % g.Mzp) < g.Mz;
  const long ib = valid ? blockIdx.y * is_in + (o == 2 ? 2 : 0) * cs_in + b * bs_in + q : 0;
  const long ob = valid ? blockIdx.y * is_out + o * cs_out + b * bs_out + q : 0;
  cx<T> v[R];
  if (o == 2) {
    static_for<0, R>([&](auto s) {
      const cx<T> x = in[ib + (valid ? (long)(j + s * Tl) * ld_in : 0)];
      v[s] = valid ? x : cx<T>{T(0), T(0)};
    });
  } else {
    // c0 = (A + conj B)/2, c1 = (A - conj B)/(2i)
    const T sg = o == 0 ? T(1) : T(-1);
    static_for<0, R>([&](auto s) {
      const long off = ib + (valid ? (long)(j + s * Tl) * ld_in : 0);
      const cx<T> x = in[off], y = in[off + cs_in];
      const cx<T> e = {T(0.5) * (x.x + sg * y.x), T(0.5) * (x.y - sg * y.y)};  // (A +- conj B)/2
      v[s] = valid ? (o == 0 ? e : cx<T>{e.y, -e.x}) : cx<T>{T(0), T(0)};
    });
  }
  tw.put(tws, tid);
  LdsCols<T, N, W> lds{sm, c};
  Plan::template fft<T, -1>(v, j, lds, TwTab<T>{tws});
  if (!valid) return;
  static_for<0, R>([&](auto s) {
    if constexpr (col_live<Plan, KL>(s)) {
      const int p = j + s * Tl;
      if (kept(p, g)) store_out<false>(out + ob + (long)crow(p, g) * ld_out, v[s]);
    }
  });
}

// P3 on packed rows: per z line, the three complex lines (u_x + i u_y,
// u_z + i w_x, w_y + i w_z) load straight into the registers of their inverse
// transforms (lane j, register s holds position p = j + s Tl: row A at p < Mz,
// row B at N - p < Mz, zero between), all nine loads of a lane in flight
// together; then the cross product c = u x w (component formula of Sec. 3.4;
// u and w already carry the 1/N^3 of Eq. ffteq, applied by the x pass), and the
// forward transforms of c0 + i c1 (stored as packed rows A, B in components
// 0, 1) and of c2 (component 2).  In place.  KL: coefficients per lane; ZA
// places coefficient k of a row (ZContig, or ZBlocked for the receive buffer
// of a z-slab all-to-all).  Three waves per SIMD: at 168 VGPRs nothing spills
// for the 2/3 rule.  FORM 0: packed rows in and out.  FORM 1 (SPLIT): store
// c0, c1 and c2 as three half-spectrum rows instead (the two real transforms
// packed in c0 + i c1 separated here, through the line's LDS region), for the
// component-row y forward pass.  FORM 2: also read component rows a, b (the
// six half spectra u_x .. w_z, from the component-row y inverse pass) and pack
// them on load: Z_p = a_p + i b_p for p < Mz, Z_p = conj a_{N-p} + i conj
// b_{N-p} for N - p < Mz, and Z_0 = Re a_0 + i Re b_0 (a real inverse
// transform drops the imaginary part at k = 0); two loads per position, the
// same bytes as the packed rows.
template <typename T, class Plan, int KL, class ZA, int FORM>
__global__ __launch_bounds__(256, 3) void k_z_cross_packed(cx<T>* __restrict__ A, long csA, long isA, long nlines, Geo g,
                                                        const int* __restrict__ act, ZA za) {
  constexpr bool SPLIT = FORM >= 1, CIN = FORM == 2;
  if (act && !act[blockIdx.y]) return;  // instance no longer iterating
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int LPB = ZShape<Plan>::LPB;
  constexpr int LS = Plan::line_stride;
  __shared__ cx<T> sm[ZShape<Plan>::SLOTS * LS];
  __shared__ cx<T> tws[N];
  TwStage<T, Plan, 256> twst;
  twst.fetch(threadIdx.x);
  int li, j;
  bool live;
  ZShape<Plan>::place(threadIdx.x, li, j, live);
  const long line = (long)blockIdx.x * LPB + li;
  const bool valid = live && line < nlines;
  const int Mz = g.Mz;  // the launcher guarantees Mz <= KL * Tl
  LdsLine<T, Plan::SH, ZShape<Plan>::kBlock> lds{sm + li * LS};
  const TwTab<T> tw{tws};
  A += blockIdx.y * isA + (valid ? line * g.Mzp : 0);
  cx<T> ph[3][R];
  static_for<0, 3>([&](auto pr) {
    const cx<T>* ra = A + (2 * pr) * csA;
    const cx<T>* rb = ra + csA;
    static_for<0, R>([&](auto s) {
      constexpr bool lo = s * Tl < KL * Tl;         // can hold a k < Mz
      constexpr bool hi = (s + 1) * Tl > N - KL * Tl;  // can hold an N - k, k < Mz
      if constexpr (lo || hi) {
        const int p = j + s * Tl;
        const bool ina = lo && valid && p < Mz;
        const bool inb = hi && !ina && valid && p > 0 && N - p < Mz;
        if constexpr (CIN) {
          const long o = za(ina ? p : (inb ? N - p : 0));
          const cx<T> a = ra[o], b = rb[o];
          const cx<T> zl = p == 0 ? cx<T>{a.x, b.x} : cx<T>{a.x - b.y, a.y + b.x};  // a + i b
          const cx<T> zh = {a.x + b.y, b.x - a.y};                                  // conj a + i conj b
          ph[pr][s] = ina ? zl : (inb ? zh : cx<T>{T(0), T(0)});
        } else {
          const cx<T> x = ina ? ra[za(p)] : rb[za(inb ? N - p : 0)];
          ph[pr][s] = (ina || inb) ? x : cx<T>{T(0), T(0)};
        }
      } else {
        ph[pr][s] = cx<T>{T(0), T(0)};
      }
    });
  });
  // twiddles to LDS while the line loads are in flight
  twst.put(tws, threadIdx.x);
  lds_barrier();
  static_for<0, 3>([&](auto pr) { Plan::template fft<T, +1>(ph[pr], j, lds, tw); });
  // u = (ph0.x, ph0.y, ph1.x), w = (ph1.y, ph2.x, ph2.y)
  cx<T> z01[R], z2[R];
  static_for<0, R>([&](auto s) {
    const T u0 = ph[0][s].x, u1 = ph[0][s].y, u2 = ph[1][s].x;
    const T w0 = ph[1][s].y, w1 = ph[2][s].x, w2 = ph[2][s].y;
    z01[s] = {u1 * w2 - u2 * w1, u2 * w0 - u0 * w2};
    z2[s] = {u0 * w1 - u1 * w0, T(0)};
  });
  Plan::template fft<T, -1>(z2, j, lds, tw);
  Plan::template fft<T, -1>(z01, j, lds, tw);
  cx<T>* oa = A;
  cx<T>* ob = A + csA;
  cx<T>* o2 = A + 2 * csA;
  if constexpr (SPLIT) {
    // C0_k = (Z_k + conj Z_{N-k})/2, C1_k = (Z_k - conj Z_{N-k})/(2i)
    static_for<0, R>([&](auto s) { lds.put(j + s * Tl, z01[s]); });
    lds.sync();
    if (!valid) return;
    static_for<0, R>([&](auto s) {
      if constexpr (s < KL) {
        const int k = j + s * Tl;
        if (k < Mz) {
          const cx<T> zk = lds.get(k);
          const cx<T> zm = lds.get((N - k) % N);
          const long o = za(k);
          store_stream(oa + o, cx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)});
          store_stream(ob + o, cx<T>{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)});
          store_stream(o2 + o, z2[s]);
        }
      }
    });
    return;
  }
  if (!valid) return;
  static_for<0, R>([&](auto s) {
    constexpr bool lo = s * Tl < KL * Tl;
    constexpr bool hi = (s + 1) * Tl > N - KL * Tl;
    if constexpr (lo || hi) {
      const int p = j + s * Tl;
      if (lo && p < Mz) {
        const long o = za(p);
        store_stream(oa + o, z01[s]);
        store_stream(o2 + o, z2[s]);
        if (p == 0) store_stream(ob + o, z01[s]);  // row B at k = 0 is Z_N = Z_0
      } else if (hi && N - p < Mz) {
        store_stream(ob + za(N - p), z01[s]);
      }
    }
  });
}

// ---------------------------------------------------------------------------
// Plain z transforms (the R2C / C2R operations).  The C2R pass applies the
// 1/N^3 of the inverse transform of Eq. ffteq (scale).
// ---------------------------------------------------------------------------
template <typename T, class Plan>
__global__ __launch_bounds__(256) void k_z_c2r(const cx<T>* __restrict__ in, T* __restrict__ out, long nlines,
                                               Geo g, T scale) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl, KL = z_loads<Plan>();
  constexpr int LPB = ZShape<Plan>::LPB;
  constexpr int LS = Plan::line_stride;
  __shared__ cx<T> sm[ZShape<Plan>::SLOTS * LS];
  __shared__ cx<T> tws[N];
  stage_twiddles<T, Plan>(tws);
  __syncthreads();
  int li, j;
  bool live;
  ZShape<Plan>::place(threadIdx.x, li, j, live);
  const long line = (long)blockIdx.x * LPB + li;
  const bool valid = live && line < nlines;
  LdsLine<T, Plan::SH, ZShape<Plan>::kBlock> lds{sm + li * LS};
  cx<T> la[KL], lb[KL];
  load_line<T, Plan, KL>(la, in + (valid ? line * g.Mzp : 0), j, g.Mz, valid);
  static_for<0, KL>([&](auto t) { lb[t] = {T(0), T(0)}; });
  cx<T> v[R];
  put_completed<T, Plan, KL>(lds, la, lb, j, g.Mz);
  lds.sync();
  read_completed<T, Plan>(lds, v, j, g.Mz);
  lds.sync();
  Plan::template fft<T, +1>(v, j, lds, TwTab<T>{tws});
  if (valid) {
    T* o = out + line * N;
    static_for<0, R>([&](auto s) { o[j + s * Tl] = v[s].x * scale; });
  }
}

template <typename T, class Plan>
__global__ __launch_bounds__(256) void k_z_r2c(const T* __restrict__ in, cx<T>* __restrict__ out, long nlines,
                                               Geo g) {
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  constexpr int LPB = ZShape<Plan>::LPB;
  constexpr int LS = Plan::line_stride;
  __shared__ cx<T> sm[ZShape<Plan>::SLOTS * LS];
  __shared__ cx<T> tws[N];
  stage_twiddles<T, Plan>(tws);
  __syncthreads();
  int li, j;
  bool live;
  ZShape<Plan>::place(threadIdx.x, li, j, live);
  const long line = (long)blockIdx.x * LPB + li;
  const bool valid = live && line < nlines;
  LdsLine<T, Plan::SH, ZShape<Plan>::kBlock> lds{sm + li * LS};
  const T* a = in + (valid ? line * N : 0);
  cx<T> v[R];
  static_for<0, R>([&](auto s) { v[s] = {valid ? a[j + s * Tl] : T(0), T(0)}; });
  Plan::template fft<T, -1>(v, j, lds, TwTab<T>{tws});
  if (valid) {
    cx<T>* o = out + line * g.Mzp;
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
// The stage update in two halves, so that a caller can have the loads of
// several elements in flight before it uses any of them.  RkIn holds what
// stage MODE reads at compact element e (component stride C): the state the
// viscous term acts on (U0 at stages 0 and 4, U1 at 1..3), U0 (stages 1, 2;
// at stage 0 it is the same array as the first) and Acc (stages 1..3).
template <typename T>
struct RkIn {
  cx<T> s[3], a[3], acc[3];
};

template <typename T, int MODE>
__device__ __forceinline__ void rk_load(long e, const cx<T>* __restrict__ U0, const cx<T>* __restrict__ U1,
                                        const cx<T>* __restrict__ Acc, long C, RkIn<T>& r) {
  static_for<0, 3>([&](auto c) {
    r.s[c] = ((MODE == 0 || MODE == 4) ? U0 : U1)[c * C + e];
    if constexpr (MODE == 1 || MODE == 2) r.a[c] = U0[c * C + e];
    if constexpr (MODE >= 1 && MODE <= 3) r.acc[c] = Acc[c * C + e];
  });
}

// n0..n2: the dealiased nonlinear term at element e, with integer
// wavenumbers kxi, kyi, kz; r: what rk_load read there.
template <typename T, int MODE>
__device__ __forceinline__ void rk_apply(long e, cx<T> n0, cx<T> n1, cx<T> n2, int kxi, int kyi, int kz,
                                         const RkIn<T>& r, cx<T>* __restrict__ U0, cx<T>* __restrict__ U1,
                                         cx<T>* __restrict__ Acc, long C, T nu, T dt) {
  const int k2i = kxi * kxi + kyi * kyi + kz * kz;
  const T kx = T(kxi), ky = T(kyi), kzf = T(kz), k2 = T(k2i);
  cx<T> kn = {T(0), T(0)};
  if (k2i != 0) {
    const T inv = T(1) / k2;
    kn = (n0 * kx + n1 * ky + n2 * kzf) * inv;
  }
  const T vk = nu * k2;
  const cx<T> d[3] = {n0 - kn * kx - r.s[0] * vk, n1 - kn * ky - r.s[1] * vk, n2 - kn * kzf - r.s[2] * vk};
  if constexpr (MODE == 4) {
    static_for<0, 3>([&](auto c) { store_stream(Acc + c * C + e, d[c]); });
  } else if constexpr (MODE == 3) {
    const T h = dt / T(6);
    static_for<0, 3>([&](auto c) { store_stream(U0 + c * C + e, r.acc[c] + d[c] * h); });
  } else {
    const T ha = (MODE == 0) ? dt / T(6) : dt / T(3);
    const T hu = (MODE == 2) ? dt : dt / T(2);
    static_for<0, 3>([&](auto c) {
      const cx<T> a = (MODE == 0) ? r.s[c] : r.a[c];
      store_stream(Acc + c * C + e, ((MODE == 0) ? a : r.acc[c]) + d[c] * ha);
      store_stream(U1 + c * C + e, a + d[c] * hu);
    });
  }
}

// One mode of the stage update (runtime mode) at compact element e.
template <typename T>
__device__ __forceinline__ void rk_update(long e, cx<T> n0, cx<T> n1, cx<T> n2, int kxi, int kyi, int kz,
                                          cx<T>* __restrict__ U0, cx<T>* __restrict__ U1, cx<T>* __restrict__ Acc,
                                          long C, int mode, T nu, T dt) {
  RkIn<T> r;
  switch (mode) {
    case 0:
      rk_load<T, 0>(e, U0, U1, Acc, C, r);
      rk_apply<T, 0>(e, n0, n1, n2, kxi, kyi, kz, r, U0, U1, Acc, C, nu, dt);
      break;
    case 1:
      rk_load<T, 1>(e, U0, U1, Acc, C, r);
      rk_apply<T, 1>(e, n0, n1, n2, kxi, kyi, kz, r, U0, U1, Acc, C, nu, dt);
      break;
    case 2:
      rk_load<T, 2>(e, U0, U1, Acc, C, r);
      rk_apply<T, 2>(e, n0, n1, n2, kxi, kyi, kz, r, U0, U1, Acc, C, nu, dt);
      break;
    case 3:
      rk_load<T, 3>(e, U0, U1, Acc, C, r);
      rk_apply<T, 3>(e, n0, n1, n2, kxi, kyi, kz, r, U0, U1, Acc, C, nu, dt);
      break;
    default:
      rk_load<T, 4>(e, U0, U1, Acc, C, r);
      rk_apply<T, 4>(e, n0, n1, n2, kxi, kyi, kz, r, U0, U1, Acc, C, nu, dt);
      break;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_rk_stage(const cx<T>* __restrict__ Nh, cx<T>* __restrict__ U0,
                                                  cx<T>* __restrict__ U1, cx<T>* __restrict__ Acc, long C,
                                                  long is, Geo g, int mode, T nu, T dt) {
  const long stride = (long)gridDim.x * blockDim.x;
  const long ib = blockIdx.y * is;  // instance of a batch (all four arrays share the stride)
  Nh += ib;
  U0 += ib;
  U1 += ib;
  Acc += ib;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < C; e += stride) {
    ModeK m;
    if (!mode_of(e, g, m)) continue;  // row padding
    rk_update(e, Nh[e], Nh[C + e], Nh[2 * C + e], m.kx, m.ky, m.kz, U0, U1, Acc, C, mode, nu, dt);
  }
}

// Register s of the k-th live row of a column (col_live): the first KL and
// the last KL registers, or all of them when those overlap.
template <class Plan, int KL>
constexpr int live_reg(int k) {
  return 2 * KL >= Plan::R ? k : (k < KL ? k : Plan::R - 2 * KL + k);
}
template <class Plan, int KL>
constexpr int live_regs() {
  return 2 * KL >= Plan::R ? Plan::R : 2 * KL;
}

// The stage update of one column of k_x_fwd_rk: v[c][s] holds component c of
// row j + s Tl.  Rows reach at most KL registers from either end (col_live):
// the others are never kept, and their outputs are not computed.  The live
// rows go in groups of GL, the loads of a whole group issued before any of its
// updates, so that a thread waits on memory once per group rather than once
// per row; a row outside the retained set loads from row 0 of its column
// (always valid) and stores nothing.  cb: the column's row 0 in the compact
// state arrays (cbase).
template <typename T, class Plan, int KL, int MODE, int GL = 2>
__device__ __forceinline__ void x_rk_tail(const cx<T> (&v)[3][Plan::R], int j, long cb, int kyi, int kz,
                                          const Geo& g, cx<T>* __restrict__ U0, cx<T>* __restrict__ U1,
                                          cx<T>* __restrict__ Acc, long C, T nu, T dt) {
  constexpr int Tl = Plan::Tl, NL = live_regs<Plan, KL>();
  static_for<0, (NL + GL - 1) / GL>([&](auto gi) {
    RkIn<T> in[GL];
    long e[GL];
    bool kp[GL];
    static_for<0, GL>([&](auto i) {
      constexpr int k = decltype(gi)::value * GL + decltype(i)::value;
      if constexpr (k < NL) {
        const int p = j + live_reg<Plan, KL>(k) * Tl;
        kp[i] = kept(p, g);
        e[i] = cb + (long)(kp[i] ? crow(p, g) : 0) * g.tw;
        rk_load<T, MODE>(e[i], U0, U1, Acc, C, in[i]);
      }
    });
    static_for<0, GL>([&](auto i) {
      constexpr int k = decltype(gi)::value * GL + decltype(i)::value;
      if constexpr (k < NL) {
        constexpr int s = live_reg<Plan, KL>(k);
        if (kp[i])
          rk_apply<T, MODE>(e[i], v[0][s], v[1][s], v[2][s], kwave(j + s * Tl, Plan::N), kyi, kz + g.kz0, in[i], U0,
                            U1, Acc, C, nu, dt);
      }
    });
  });
}

// ---------------------------------------------------------------------------
// P5 fused with the stage update: forward transform along x of the three
// components of a tile (one after the other, the first two kept in
// registers), then the projection, viscous term and RK4 stage update of the
// retained modes, so that the nonlinear term never goes to HBM.  Input
// A[3][N rows (x)][Q = M*Mzp cols (ky, kz)]; the state arrays are compact
// [3][M][Q].  blockIdx.y is the instance of a batch.
// ---------------------------------------------------------------------------
// One tile of instance `inst` (tile * W < M * Mzp), run by the W * Tl
// threads of a block (tid) with sm = N * W + N values of LDS (the exchange
// tile, then the stage twiddles).  k_x_fwd_rk runs one tile per block; the
// persistent batch kernel calls it for its work items.
template <typename T, class Plan, int W, int KL, bool G23 = false, int GL = 2>
__device__ __forceinline__ void x_fwd_rk_tile(const cx<T>* __restrict__ A, long csA, long isA,
                                              cx<T>* __restrict__ U0, cx<T>* __restrict__ U1,
                                              cx<T>* __restrict__ Acc, long C, long isU, const Geo& g_in, int mode,
                                              T nu, T dt, long tile, int inst, int tid, cx<T>* sm) {
  const Geo g = G23 ? geo_two_thirds<Plan::N>(g_in) : g_in;
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl;
  cx<T>* tws = sm + N * W;
  const long Q = (long)g.M * g.Mzp;
  const int c = tid % W, j = tid / W;
  const long q = tile * W + c;
  const int iy = (int)(q / g.Mzp);
  const int kz = (int)(q - (long)iy * g.Mzp);
  const bool valid = q < Q && kz < g.Mz;
  const long qq = valid ? q : 0;
  A += inst * isA;
  U0 += inst * isU;
  U1 += inst * isU;
  Acc += inst * isU;
  TwStage<T, Plan, W * Tl> tw;
  tw.fetch(tid);
  // every component's loads in flight together (their registers hold the
  // transformed values afterwards anyway)
  cx<T> v[3][R];
  static_for<0, 3>([&](auto comp) {
    const cx<T>* a = A + comp * csA + qq;
    static_for<0, R>([&](auto s) {
      const cx<T> x = a[(long)(j + s * Tl) * Q];
      v[comp][s] = valid ? x : cx<T>{T(0), T(0)};
    });
  });
  tw.put(tws, tid);
  static_for<0, 3>([&](auto comp) {
    LdsCols<T, N, W> lds{sm, c};
    Plan::template fft<T, -1>(v[comp], j, lds, TwTab<T>{tws});
  });
  if (!valid) return;
  const int kyi = kwave(cpos(iy, g), N);
  const long cb = cbase(q, g);
  switch (mode) {
    case 0: x_rk_tail<T, Plan, KL, 0, GL>(v, j, cb, kyi, kz, g, U0, U1, Acc, C, nu, dt); break;
    case 1: x_rk_tail<T, Plan, KL, 1, GL>(v, j, cb, kyi, kz, g, U0, U1, Acc, C, nu, dt); break;
    case 2: x_rk_tail<T, Plan, KL, 2, GL>(v, j, cb, kyi, kz, g, U0, U1, Acc, C, nu, dt); break;
    case 3: x_rk_tail<T, Plan, KL, 3, GL>(v, j, cb, kyi, kz, g, U0, U1, Acc, C, nu, dt); break;
    default: x_rk_tail<T, Plan, KL, 4, GL>(v, j, cb, kyi, kz, g, U0, U1, Acc, C, nu, dt); break;
  }
}

template <typename T, class Plan, int W, int KL, bool G23 = false>
__global__ __launch_bounds__(W* Plan::Tl) void k_x_fwd_rk(const cx<T>* __restrict__ A, long csA, long isA,
                                                          cx<T>* __restrict__ U0, cx<T>* __restrict__ U1,
                                                          cx<T>* __restrict__ Acc, long C, long isU, Geo g_in, int mode,
                                                          T nu, T dt) {
  constexpr int PAIR = (W * (int)sizeof(cx<T>) < 128) ? 128 / (W * (int)sizeof(cx<T>)) : 1;
  __shared__ cx<T> sm[Plan::N * W + Plan::N];
  const long tile = tile_of_block<PAIR>(blockIdx.x);
  // whole block leaves together (the launcher's g has the row count M * Mzp)
  if (tile * W >= (long)g_in.M * g_in.Mzp) return;
  x_fwd_rk_tile<T, Plan, W, KL, G23>(A, csA, isA, U0, U1, Acc, C, isU, g_in, mode, nu, dt, tile, blockIdx.y,
                                     threadIdx.x, sm);
}

// ---------------------------------------------------------------------------
// Implicit midpoint step (Crank-Nicolson on the viscous term), an implicit
// alternative to the RK4 integration of Sec. 2, solved by Picard sweeps on the
// increment d = u^{n+1} - u^n:
//   d <- [dt F_NL(u^n + d/2) - 2 a u^n] / (1 + a),   a = dt nu |k|^2 / 2,
// with F_NL = Nh - k (k.Nh)/|k|^2, the right-hand side of Eq. NSfinal without
// its viscous term.  Iterating on d rather than on u^{n+1} keeps the rounding
// relative to the increment, so the stopping test ||d_new - d|| <= tau ||d_new||
// stays decidable in FP32 when the increment is far below the state.  Norms
// are those of the real field: weight 1 on the kz = 0 plane, 2 elsewhere.
// act[b] == 0 marks an instance whose iteration has stopped; every pass
// kernel leaves such an instance alone.
// ---------------------------------------------------------------------------


// Predictor from the increments of earlier steps (H1 newest), the polynomial
// through the last hist of them one step ahead: hist = 0: d = 0; 1: d = H1;
// 2: d = 2 H1 - H2; 3: d = 3 H1 - 3 H2 + H3; 4: d = 4 H1 - 6 H2 + 4 H3 - H4.
// Writes d and the midpoint U1 = U0 + d/2, and marks the instance active.
template <typename T>
__global__ __launch_bounds__(256) void k_imp_predict(const cx<T>* __restrict__ U0, cx<T>* __restrict__ D,
                                                     cx<T>* __restrict__ U1, const cx<T>* __restrict__ H1,
                                                     const cx<T>* __restrict__ H2, const cx<T>* __restrict__ H3,
                                                     const cx<T>* __restrict__ H4, long C, long is, Geo g, int hist,
                                                     int* __restrict__ act) {
  const long ib = blockIdx.y * is;
  if (blockIdx.x == 0 && threadIdx.x == 0) act[blockIdx.y] = 1;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < C; e += stride) {
    ModeK m;
    if (!mode_of(e, g, m)) continue;
    for (int c = 0; c < 3; ++c) {
      const long i = ib + c * C + e;
      cx<T> d = {T(0), T(0)};
      if (hist == 1) d = H1[i];
      if (hist == 2) d = H1[i] * T(2) - H2[i];
      if (hist == 3) d = (H1[i] - H2[i]) * T(3) + H3[i];
      if (hist >= 4) d = (H1[i] + H3[i]) * T(4) - H2[i] * T(6) - H4[i];
      D[i] = d;
      U1[i] = U0[i] + d * T(0.5);
    }
  }
}

// Sum of a double over a 256-thread block (fixed order: deterministic); the
// result is valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// One Picard update of d from the nonlinear term Nh of the midpoint, plus the
// block's partial sums of ||d_new - d||^2 and ||d_new||^2 in part[b][block].
template <typename T>
__global__ __launch_bounds__(256) void k_imp_update(const cx<T>* __restrict__ Nh, const cx<T>* __restrict__ U0,
                                                    cx<T>* __restrict__ D, cx<T>* __restrict__ U1,
                                                    double* __restrict__ part, long C, long is, Geo g, T nu, T dt,
                                                    const int* __restrict__ act) {
  __shared__ double red[4];
  if (!act[blockIdx.y]) return;  // whole block leaves together
  const long ib = blockIdx.y * is;
  const long stride = (long)gridDim.x * blockDim.x;
  double su = 0.0, si = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < C; e += stride) {
    ModeK m;
    if (!mode_of(e, g, m)) continue;
    const long i0 = ib + e, i1 = i0 + C, i2 = i0 + 2 * C;
    const int k2i = m.kx * m.kx + m.ky * m.ky + m.kz * m.kz;
    const T kx = T(m.kx), ky = T(m.ky), kz = T(m.kz);
    const cx<T> n0 = Nh[i0], n1 = Nh[i1], n2 = Nh[i2];
    cx<T> kn = {T(0), T(0)};
    if (k2i != 0) kn = (n0 * kx + n1 * ky + n2 * kz) * (T(1) / T(k2i));
    const T a = T(0.5) * dt * nu * T(k2i);
    const T inv = T(1) / (T(1) + a);
    const cx<T> u0 = U0[i0], u1 = U0[i1], u2 = U0[i2];
    const cx<T> d0 = ((n0 - kn * kx) * dt - u0 * (T(2) * a)) * inv;
    const cx<T> d1 = ((n1 - kn * ky) * dt - u1 * (T(2) * a)) * inv;
    const cx<T> d2 = ((n2 - kn * kz) * dt - u2 * (T(2) * a)) * inv;
    const cx<T> o0 = D[i0], o1 = D[i1], o2 = D[i2];
    const double w = m.kz == 0 ? 1.0 : 2.0;
    const cx<T> e0 = d0 - o0, e1 = d1 - o1, e2 = d2 - o2;
    su += w * ((double)e0.x * e0.x + (double)e0.y * e0.y + (double)e1.x * e1.x + (double)e1.y * e1.y +
               (double)e2.x * e2.x + (double)e2.y * e2.y);
    si += w * ((double)d0.x * d0.x + (double)d0.y * d0.y + (double)d1.x * d1.x + (double)d1.y * d1.y +
               (double)d2.x * d2.x + (double)d2.y * d2.y);
    D[i0] = d0;
    D[i1] = d1;
    D[i2] = d2;
    U1[i0] = u0 + d0 * T(0.5);
    U1[i1] = u1 + d1 * T(0.5);
    U1[i2] = u2 + d2 * T(0.5);
  }
  su = block_sum_256(su, red);
  si = block_sum_256(si, red);
  if (threadIdx.x == 0) {
    double* q = part + 2 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
    q[0] = su;
    q[1] = si;
  }
}

// Stopping test of instance blockIdx.x (one wave): sum its nparts partial
// sums in a fixed order and clear act when ||d_new - d|| <= tau ||d_new||.
// The sweep just run is counted in sweeps[b].
template <int Unused = 0>
__global__ __launch_bounds__(64) void k_imp_decide(const double* __restrict__ part, int nparts, int* __restrict__ act,
                                                   double tau2, int* __restrict__ sweeps) {
  const int b = blockIdx.x;
  if (!act[b]) return;
  double su = 0.0, si = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) {
    su += part[2 * ((long)b * nparts + i)];
    si += part[2 * ((long)b * nparts + i) + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    su += __shfl_xor(su, o, 64);
    si += __shfl_xor(si, o, 64);
  }
  if (threadIdx.x == 0) {
    sweeps[b] += 1;
    if (su <= tau2 * si) act[b] = 0;
  }
}

// After the last allowed sweep of a step: an instance still active stopped
// at max_iter; count it in nonconv[b].
template <int Unused = 0>
__global__ __launch_bounds__(256) void k_imp_close(const int* __restrict__ act, int* __restrict__ nonconv, int nb) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < nb; b += gridDim.x * 256)
    if (act[b]) nonconv[b] += 1;
}

// p[0..n) = v (a fill kernel: graph-safe, unlike a memset node).
template <int Unused = 0>
__global__ __launch_bounds__(256) void k_fill_int(int* __restrict__ p, long n, int v) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = v;
}

// End of a step: U0 += D.
template <typename T>
__global__ __launch_bounds__(256) void k_imp_advance(cx<T>* __restrict__ U0, const cx<T>* __restrict__ D, long C,
                                                     long is, Geo g) {
  const long ib = blockIdx.y * is;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < C; e += stride) {
    ModeK m;
    if (!mode_of(e, g, m)) continue;
    for (int c = 0; c < 3; ++c) {
      const long i = ib + c * C + e;
      U0[i] = U0[i] + D[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Diagnostics of a canonical half-spectrum field [3][N][N][N/2+1]:
//   E   = sum_half w |u_k|^2 / (2 N^6)         kinetic energy (Parseval under Eq. ffteq)
//   eps = nu sum_half w |k|^2 |u_k|^2 / N^6    = nu <|omega|^2>, the rate at which
//                                               the viscous term of Eq. NSfinal removes energy
// with w = 1 on the kz = 0 and kz = N/2 planes and 2 elsewhere.  Per-block FP64
// partial sums part[block][2], summed in a fixed order by k_diag_final.
// One launch per instance.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_diag(const cx<T>* __restrict__ u, int N, double* __restrict__ part) {
  __shared__ double red[4];
  const long Nh = N / 2 + 1, plane = (long)N * Nh, comp = (long)N * plane;
  double se = 0.0, sd = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < comp; e += (long)gridDim.x * 256) {
    const int px = (int)(e / plane);
    const long r = e - px * plane;
    const int py = (int)(r / Nh);
    const int kz = (int)(r - (long)py * Nh);
    const int kx = kwave(px, N), ky = kwave(py, N);
    double a = 0.0;
    for (int c = 0; c < 3; ++c) {
      const cx<T> v = u[c * comp + e];
      a += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double w = (kz == 0 || 2 * kz == N) ? 1.0 : 2.0;
    se += w * a;
    sd += w * (double)(kx * kx + ky * ky + kz * kz) * a;
  }
  se = block_sum_256(se, red);
  sd = block_sum_256(sd, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = se;
    part[2 * blockIdx.x + 1] = sd;
  }
}

// out[0..2) = {E, eps} from one instance's nparts partial sums (one wave).
template <int Unused = 0>
__global__ __launch_bounds__(64) void k_diag_final(const double* __restrict__ part, int nparts, int N, double nu,
                                                   double* __restrict__ out) {
  double se = 0.0, sd = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) {
    se += part[2 * i];
    sd += part[2 * i + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_xor(se, o, 64);
    sd += __shfl_xor(sd, o, 64);
  }
  if (threadIdx.x == 0) {
    const double n6 = (double)N * N * N * N * N * N;
    out[0] = se / (2.0 * n6);
    out[1] = nu * sd / n6;
  }
}

// Per-instance statistics of a call (the hot_stats record of include/hot.h):
// E and eps, as k_diag defines them, of a compact state U [B][3][C] (every
// other mode of the canonical array is zero), plus the implicit step's
// counters.  k_state_sums: per-block FP64 partial sums part[b][block][2];
// k_state_final (one wave per instance) adds them in a fixed order.
struct StatsRec {
  double energy, dissipation;
  int sweeps, nonconv;
};

template <typename T>
__global__ __launch_bounds__(256) void k_state_sums(const cx<T>* __restrict__ U, long C, long is, Geo g,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  U += blockIdx.y * is;
  double se = 0.0, sd = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < C; e += (long)gridDim.x * 256) {
    ModeK m;
    if (!mode_of(e, g, m)) continue;
    double a = 0.0;
    for (int c = 0; c < 3; ++c) {
      const cx<T> v = U[c * C + e];
      a += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double w = (m.kz == 0 || 2 * m.kz == g.N) ? 1.0 : 2.0;
    se += w * a;
    sd += w * (double)(m.kx * m.kx + m.ky * m.ky + m.kz * m.kz) * a;
  }
  se = block_sum_256(se, red);
  sd = block_sum_256(sd, red);
  if (threadIdx.x == 0) {
    double* q = part + 2 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
    q[0] = se;
    q[1] = sd;
  }
}

// Instance blockIdx.x of the group is instance idx[b] of the call (idx NULL:
// the group's single instance is idx0).  sweeps / nonconv NULL: zeros.
template <int Unused = 0>
__global__ __launch_bounds__(64) void k_state_final(const double* __restrict__ part, int nparts, int N, double nu,
                                                    const long* __restrict__ idx, long idx0,
                                                    const int* __restrict__ sweeps, const int* __restrict__ nonconv,
                                                    StatsRec* __restrict__ out) {
  const int b = blockIdx.x;
  double se = 0.0, sd = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) {
    se += part[2 * ((long)b * nparts + i)];
    sd += part[2 * ((long)b * nparts + i) + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_xor(se, o, 64);
    sd += __shfl_xor(sd, o, 64);
  }
  if (threadIdx.x == 0) {
    const double n6 = (double)N * N * N * N * N * N;
    StatsRec r;
    r.energy = se / (2.0 * n6);
    r.dissipation = nu * sd / n6;
    r.sweeps = sweeps ? sweeps[b] : 0;
    r.nonconv = nonconv ? nonconv[b] : 0;
    out[idx ? idx[b] : idx0] = r;
  }
}

// ---------------------------------------------------------------------------
// Canonical <-> compact.  Canonical: [3][N][N][N/2+1].  Compact: the state
// layout of cbase.  Gather drops the modes outside the retained set
// (projection onto the Galerkin space); scatter writes zeros there.
// blockIdx.y is the instance of a batch; the canonical array of instance b
// is tab[b] when a device pointer table is given.
// ---------------------------------------------------------------------------
// Position (c, a, b, z) of a flat index over [3][na][nb][nz], advanced by a
// constant step with carries: the grid-stride loops below divide once per
// thread instead of three times per element (64-bit divisions made them
// VALU-bound).  The host decomposes the grid stride itself.
struct Pos4 {
  int c, a, b, z;
};

__host__ __device__ __forceinline__ Pos4 pos4_of(long e, int na, int nb, int nz) {
  const long row = e / nz;
  const long ab = row / nb;
  Pos4 p;
  p.z = (int)(e - row * nz);
  p.b = (int)(row - ab * nb);
  p.c = (int)(ab / na);
  p.a = (int)(ab - (long)p.c * na);
  return p;
}

// The same for a thread's first index (below 2^31: at most 65535 blocks of
// 256 threads), in 32-bit arithmetic.
__device__ __forceinline__ Pos4 pos4_first(unsigned e, unsigned na, unsigned nb, unsigned nz) {
  const unsigned row = e / nz;
  const unsigned ab = row / nb;
  Pos4 p;
  p.z = (int)(e - row * nz);
  p.b = (int)(row - ab * nb);
  p.c = (int)(ab / na);
  p.a = (int)(ab - (unsigned)p.c * na);
  return p;
}

__device__ __forceinline__ void pos4_add(Pos4& p, const Pos4& s, int na, int nb, int nz) {
  p.z += s.z;
  int k = p.z >= nz;
  p.z -= k ? nz : 0;
  p.b += s.b + k;
  k = p.b >= nb;
  p.b -= k ? nb : 0;
  p.a += s.a + k;
  k = p.a >= na;
  p.a -= k ? na : 0;
  p.c += s.c + k;
}

// Device pointer tables of a batch (the canonical arrays of its instances):
// the pointers travel as kernel arguments, so the tables are written in
// stream order with no host synchronisation, and a call captured into a graph
// records them by value.  One chunk carries the input pointers, the output
// pointers and the instance indices of up to kTabChunk members (3840 bytes of
// the 4096 a kernel's arguments may take); the three tables lie nb entries
// apart.
constexpr int kTabChunk = 160;
struct TabChunk {
  const void* in[kTabChunk];
  const void* out[kTabChunk];
  const void* idx[kTabChunk];
};

template <int Unused = 0>
__global__ __launch_bounds__(256) void k_write_tab(const void** __restrict__ tab, long nb, TabChunk c, int n) {
  const int i = threadIdx.x;
  if (i < n) {
    tab[i] = c.in[i];
    tab[nb + i] = c.out[i];
    tab[2 * nb + i] = c.idx[i];
  }
}

// The elements e0, e0 + stride, ... of one instance (st: stride in the
// digits of the loop).  k_gather runs it as a grid-stride loop; the
// persistent batch kernel as a block-stride loop per work item.
template <typename T>
__device__ __forceinline__ void gather_part(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const Geo& g,
                                            Pos4 st, long e, long stride) {
  const long Nh = g.czp;  // canonical z extent; its kz 0 is local column 0
  if (g.tw == g.M * g.Mzp) {
    // row-major compact [3][M][M][Mzp]; st: the grid stride in the same digits
    Pos4 p = pos4_first((unsigned)e, g.M, g.M, g.Mzp);
    for (; p.c < 3; e += stride, pos4_add(p, st, g.M, g.M, g.Mzp)) {
      if (p.z >= g.Mz) continue;
      const long src = (((long)p.c * g.N + cpos(p.a, g)) * g.N + cpos(p.b, g)) * Nh + p.z;
      store_stream(out + e, in[src]);
    }
  } else {
    // column tiles [3][Q/tw][M][tw] (cbase); st in the same digits
    const int nt = g.M * (g.Mzp / g.tw);
    Pos4 p = pos4_first((unsigned)e, nt, g.M, g.tw);
    for (; p.c < 3; e += stride, pos4_add(p, st, nt, g.M, g.tw)) {
      const unsigned q = (unsigned)p.a * g.tw + p.z;
      const unsigned iy = q / (unsigned)g.Mzp;
      const int kz = (int)(q - iy * (unsigned)g.Mzp);
      if (kz >= g.Mz) continue;
      const long src = (((long)p.c * g.N + cpos(p.b, g)) * g.N + cpos((int)iy, g)) * Nh + kz;
      store_stream(out + e, in[src]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(const cx<T>* __restrict__ in0, const cx<T>* const* __restrict__ in_tab,
                                                cx<T>* __restrict__ out, long C, long is, Geo g, Pos4 st) {
  // instance blockIdx.y: its canonical input from the table (or in0 alone)
  const cx<T>* __restrict__ in = in_tab ? in_tab[blockIdx.y] : in0;
  gather_part(in, out + blockIdx.y * is, g, st, (long)blockIdx.x * blockDim.x + threadIdx.x,
              (long)gridDim.x * blockDim.x);
}

// The elements e0, e0 + stride, ... of one instance's canonical output, as
// gather_part.
template <typename T>
__device__ __forceinline__ void scatter_part(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, long C,
                                             const Geo& g, Pos4 st, long e, long stride) {
  const int Nh = g.czp;
  // canonical [3][N][N][Nh]; st: the stride in the same digits.  Four
  // elements per round, their loads issued before any store (an element
  // outside the retained set loads slot 0 and stores zero).
  Pos4 p = pos4_first((unsigned)e, g.N, g.N, Nh);
  while (p.c < 3) {
    cx<T> v[4];
    long eo[4];
    bool ok[4];
    static_for<0, 4>([&](auto k) {
      ok[k] = p.c < 3;
      const bool live = ok[k] && p.z < g.Mz && kept(p.a, g) && kept(p.b, g);
      const long src =
          live ? (long)p.c * C + cbase((long)crow(p.b, g) * g.Mzp + p.z, g) + (long)crow(p.a, g) * g.tw : 0;
      const cx<T> x = in[src];
      v[k] = live ? x : cx<T>{T(0), T(0)};
      eo[k] = e;
      e += stride;
      pos4_add(p, st, g.N, g.N, Nh);
    });
    static_for<0, 4>([&](auto k) {
      if (ok[k]) store_stream(out + eo[k], v[k]);
    });
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter(const cx<T>* __restrict__ in, cx<T>* out0, cx<T>* const* __restrict__ out_tab,
                                                 long C, long is, Geo g, Pos4 st) {
  cx<T>* __restrict__ out = out_tab ? out_tab[blockIdx.y] : out0;
  scatter_part(in + blockIdx.y * is, out, C, g, st, (long)blockIdx.x * blockDim.x + threadIdx.x,
               (long)gridDim.x * blockDim.x);
}

// Canonical -> column-tiled compact state through LDS (tw < M * Mzp).  A
// block takes RX consecutive compact kx rows of one compact ky row iy
// (blockIdx.y = component * M + iy) and holds them as [RX][Mzp + 1] values
// in LDS: the canonical rows (kx, ky, all retained kz) are read whole, and
// each compact tile of the ky row (tw kz columns, rows kx contiguous) is
// written as RX * tw consecutive values.  k_gather reads the canonical rows
// in 64-byte pieces instead (measured at 1024^3: 2.0 against 1.4 ms).  A
// scatter of the same shape (with the zero rows) measured 4.4 ms against
// 3.9 ms for k_scatter, whose canonical writes are already whole rows.
// blockIdx.z is the instance of a batch.
template <typename T, int RX>
__global__ __launch_bounds__(256) void k_gather_t(const cx<T>* __restrict__ in0, const cx<T>* const* __restrict__ in_tab,
                                                  cx<T>* __restrict__ out, long C, long is, Geo g) {
  extern __shared__ unsigned char gt_smem[];
  cx<T>* sm = reinterpret_cast<cx<T>*>(gt_smem);
  const cx<T>* __restrict__ in = in_tab ? in_tab[blockIdx.z] : in0;
  out += blockIdx.z * is;
  const int tid = threadIdx.x;
  const int c = blockIdx.y / g.M, iy = blockIdx.y - c * g.M;
  const int x0 = blockIdx.x * RX, nr = g.M - x0 < RX ? g.M - x0 : RX;
  const int ky = cpos(iy, g), Nh = g.czp, P = g.Mzp + 1, tpr = g.Mzp / g.tw, Mz = g.Mz;
  // eight loads in flight per thread before their LDS stores
  for (int f0 = 0; f0 < nr * Mz; f0 += 8 * 256) {
    cx<T> v[8];
    int at[8];
    static_for<0, 8>([&](auto k) {
      const int f = f0 + k * 256 + tid;
      const bool ok = f < nr * Mz;
      const int r = ok ? f / Mz : 0, kz = ok ? f - r * Mz : 0;
      v[k] = in[(((long)c * g.N + cpos(x0 + r, g)) * g.N + ky) * Nh + kz];
      at[k] = ok ? r * P + kz : -1;
    });
    static_for<0, 8>([&](auto k) {
      if (at[k] >= 0) sm[at[k]] = v[k];
    });
  }
  __syncthreads();
  const int tile = nr * g.tw;
  for (int f = tid; f < tpr * tile; f += 256) {
    const int t = f / tile, rem = f - t * tile, r = rem / g.tw, zz = rem - r * g.tw;
    const int kz = t * g.tw + zz;
    if (kz < Mz) store_stream(out + c * C + ((long)(iy * tpr + t) * g.M + x0 + r) * g.tw + zz, sm[r * P + kz]);
  }
}

}  // namespace hot
