// Kernel launchers of libhot for one (element type, N): line plans, tile
// shapes and the Ops table.  Each (type, N) is instantiated in its own
// translation unit (generated at build time) so the library builds in
// parallel; hot.hip only sees the Ops tables.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"
#include "yz_fused.hpp"

namespace hot {

// ---------------------------------------------------------------------------
// line plans per length (per-thread count R and radix sequence)
// ---------------------------------------------------------------------------
template <int N>
struct LP;
template <> struct LP<8> { using P = LinePlan<8, 8, 8>; };
template <> struct LP<16> { using P = LinePlan<16, 16, 16>; };
template <> struct LP<32> { using P = LinePlan<32, 8, 8, 4>; };
template <> struct LP<64> { using P = LinePlan<64, 8, 8, 8>; };
template <> struct LP<128> { using P = LinePlan<128, 16, 16, 8>; };
template <> struct LP<256> { using P = LinePlan<256, 16, 16, 16>; };
template <> struct LP<512> { using P = LinePlan<512, 16, 16, 16, 2>; };
template <> struct LP<1024> { using P = LinePlan<1024, 16, 16, 16, 4>; };
template <> struct LP<2048> { using P = LinePlan<2048, 16, 16, 16, 8>; };
// 2^a 3^b lengths of the batched workloads
template <> struct LP<18> { using P = LinePlan<18, 6, 6, 3>; };
template <> struct LP<24> { using P = LinePlan<24, 12, 4, 6>; };
template <> struct LP<36> { using P = LinePlan<36, 6, 6, 6>; };
template <> struct LP<48> { using P = LinePlan<48, 12, 4, 4, 3>; };
template <> struct LP<54> { using P = LinePlan<54, 6, 6, 3, 3>; };

// line plans of the x forward pass fused with the stage update: it holds three
// components per thread, so long lines spread over twice the lanes (half the
// registers per component, one more exchange)
template <int N>
struct LPf {
  using P = typename LP<N>::P;
};
template <> struct LPf<1024> { using P = LinePlan<1024, 8, 8, 8, 4, 4>; };

// line plans of the z passes (one line per Tl lanes; see ZShape)
template <int N>
struct LPz {
  using P = typename LP<N>::P;
};
// FP32 z lines of the short lengths: LDS slots per line picked with a model of
// the 64 four-byte LDS banks (8-byte accesses served 32 lanes at a time) so
// that the lines of a wave fall on different banks in the z pass's exchanges
// (Stockham stages, Hermitian completion and split): the summed conflict
// degree drops from 1935 / 108 / 213 / 147 / 109 / 333 / 291 / 227 to
// 0 / 72 / 9 / 4 / 105 / 21 / 168 / 11 at N = 16 / 18 / 24 / 32 / 36 / 48 / 54 / 64
// (the bank model tests/zline_banks.py, checked by tests/test_line_strides.py).
template <int N>
struct LPz32 {
  using P = typename LPz<N>::P;
};
template <> struct LPz32<16> { using P = StridedLines<LP<16>::P, 17>; };
template <> struct LPz32<18> { using P = StridedLines<LP<18>::P, 35>; };
template <> struct LPz32<24> { using P = StridedLines<LP<24>::P, 34>; };
template <> struct LPz32<32> { using P = StridedLines<LP<32>::P, 44>; };
template <> struct LPz32<36> { using P = StridedLines<LP<36>::P, 58>; };
template <> struct LPz32<48> { using P = StridedLines<LP<48>::P, 68>; };
template <> struct LPz32<54> { using P = StridedLines<LP<54>::P, 70>; };
template <> struct LPz32<64> { using P = StridedLines<LP<64>::P, 88>; };

// Columns per block of a strided pass: at least one 128-byte segment per row
// (16 FP32 / 8 FP64 complex values), more while the LDS tile stays within
// 64 KB; never above 1024 threads or a 128 KB tile.
template <typename T, int N>
constexpr int cols_per_block() {
  constexpr int tl = LP<N>::P::Tl;
  constexpr int seg = int(128 / sizeof(cx<T>));
  int w = int(65536 / (N * sizeof(cx<T>)));
  if (w > 64) w = 64;
  if (w < seg) w = seg;
  while (w > 1 && (w * tl > 1024 || (long)N * w * (long)sizeof(cx<T>) > 131072)) w /= 2;
  return w;
}

// Kernel launchers for one (element type, N).  Every function enqueues one
// kernel on the stream for nb instances of a batch (instance strides is*)
// and returns hipGetLastError().
struct Ops {
  // act: per-instance flags of an implicit step (NULL: every instance runs)
  hipError_t (*strided)(hipStream_t, int variant, int dir, bool inc, bool outc, const void* in, void* out,
                        long ncols, long Qp, long ld_in, long ld_out, long bs_in, long bs_out, long cs_in,
                        long cs_out, int ncomp, long is_in, long is_out, long otw, int nb, const Geo&,
                        const int* act);
  hipError_t (*x_inv_curl)(hipStream_t, int variant, const void* U, long csU, long isU, void* A, long csA, long isA,
                           int nb, const Geo&, const int* act);
  hipError_t (*z_cross)(hipStream_t, void* A, long csA, long isA, long nlines, int nb, const Geo&, const int* act);
  // the y inverse, z and y forward passes on packed pair rows (k_y_inv_pack,
  // k_z_cross_packed, k_y_fwd_unpack); strided-pass arguments without the
  // direction, row kinds and component count
  hipError_t (*y_inv_pack)(hipStream_t, int variant, const void* in, void* out, long ncols, long Qp, long ld_in,
                           long ld_out, long bs_in, long bs_out, long cs_in, long cs_out, long is_in, long is_out,
                           int nb, const Geo&, const int* act);
  // form: 0 packed rows in and out, 1 packed in and component rows out, 2
  // component rows in (packed on load) and out
  hipError_t (*z_cross_packed)(hipStream_t, void* A, long csA, long isA, long nlines, int nb, const Geo&,
                               const int* act, int form);
  hipError_t (*y_fwd_unpack)(hipStream_t, int variant, const void* in, void* out, long ncols, long Qp, long ld_in,
                             long ld_out, long bs_in, long bs_out, long cs_in, long cs_out, long is_in, long is_out,
                             int nb, const Geo&, const int* act);
  // z_cross on lines that arrive in chunks of `chunk` coefficients, blocks blk
  // elements apart (the receive buffer of a z-slab all-to-all)
  hipError_t (*z_cross_blocked)(hipStream_t, void* A, long csA, long nlines, const Geo&, int chunk, long blk);
  hipError_t (*z_cross_packed_blocked)(hipStream_t, void* A, long csA, long nlines, const Geo&, int chunk, long blk,
                                       int form);
  // y inverse, z pass and y forward in one kernel, in place on A1 (NULL where
  // the six planes of an x-plane do not fit in LDS)
  hipError_t (*yz_fused)(hipStream_t, void* A, long csA, long isA, int nb, const Geo&, const int* act);
  hipError_t (*z_c2r)(hipStream_t, const void* in, void* out, long nlines, const Geo&);
  hipError_t (*z_r2c)(hipStream_t, const void* in, void* out, long nlines, const Geo&);
  hipError_t (*rk_stage)(hipStream_t, const void* Nh, void* U0, void* U1, void* Acc, long C, long is, int nb,
                         const Geo&, int mode, double nu, double dt);
  // x forward transform fused with the stage update (replaces x_fwd + rk_stage)
  hipError_t (*x_fwd_rk)(hipStream_t, int variant, const void* A, long csA, long isA, void* U0, void* U1, void* Acc,
                         long C, long isU, int nb, const Geo&, int mode, double nu, double dt);
  hipError_t (*gather)(hipStream_t, const void* in0, const void* const* in_tab, void* out, long C, long is, int nb,
                       const Geo&);
  hipError_t (*scatter)(hipStream_t, const void* in, void* out0, void* const* out_tab, long C, long is, int nb,
                        const Geo&);
  // implicit midpoint step
  hipError_t (*imp_predict)(hipStream_t, const void* U0, void* D, void* U1, const void* H1, const void* H2,
                            const void* H3, const void* H4, long C, long is, int nb, const Geo&, int hist, int* act);
  hipError_t (*imp_update)(hipStream_t, const void* Nh, const void* U0, void* D, void* U1, double* part, long C,
                           long is, int nb, const Geo&, double nu, double dt, const int* act);
  hipError_t (*imp_advance)(hipStream_t, void* U0, const void* D, long C, long is, int nb, const Geo&);
  int strided_variants;       // number of column widths the autotuner may pick from
  int strided_width[3];       // columns per block of each variant
  int fused_width[3];         // columns per block of the x_fwd_rk variants 0, 1, 2
};

static inline unsigned grid_1d(long work, int block) {
  long g = (work + block - 1) / block;
  const long cap = 256L * 64;  // grid-stride loops: a few waves per SIMD
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T, int N>
struct Impl {
  using P = typename LP<N>::P;
  static constexpr int W = cols_per_block<T, N>();
  static constexpr int Tl = P::Tl;

  // strided column widths the autotuner chooses from: W/2, W, 2W when the
  // block stays within 1024 threads, at least one wave and 160 KB of LDS
  static constexpr bool fits(int w) {
    return w >= 1 && w * Tl <= 1024 && w * Tl >= 64 && (long)N * (w + 1) * (long)sizeof(cx<T>) <= 163840;
  }
  static constexpr int WV0 = fits(W / 2) ? W / 2 : W;
  static constexpr int WV2 = fits(2 * W) ? 2 * W : W;

  template <int WW, int DIR, bool IC, bool OC>
  static void go(hipStream_t s, const void* in, void* out, long ncols, long Qp, long ld_in, long ld_out, long bs_in,
                 long bs_out, long cs_in, long cs_out, int ncomp, long is_in, long is_out, long otw, int nb,
                 const Geo& g, const int* act) {
    constexpr int pair = (WW * (int)sizeof(cx<T>) < 128) ? 128 / (WW * (int)sizeof(cx<T>)) : 1;
    const long ntiles = (ncols + WW - 1) / WW;
    const long group = 8L * pair;
    dim3 grid((unsigned)((ntiles + group - 1) / group * group), (unsigned)ncomp, (unsigned)nb);
    hipLaunchKernelGGL((k_strided<T, P, DIR, WW, IC, OC>), grid, dim3(WW * Tl), 0, s, (const cx<T>*)in, (cx<T>*)out,
                       ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, is_in, is_out, otw, g, act);
  }
  template <int WW>
  static hipError_t strided_w(hipStream_t s, int dir, bool inc, bool outc, const void* in, void* out, long ncols,
                              long Qp, long ld_in, long ld_out, long bs_in, long bs_out, long cs_in, long cs_out,
                              int ncomp, long is_in, long is_out, long otw, int nb, const Geo& g, const int* act) {
#define HOT_GO(D, I, O)                                                                                          \
  go<WW, D, I, O>(s, in, out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, ncomp, is_in, is_out, otw, nb, g, \
                  act)
    if (dir > 0) {
      if (inc && !outc) HOT_GO(+1, true, false);
      else if (!inc && !outc) HOT_GO(+1, false, false);
      else return hipErrorInvalidValue;
    } else {
      if (!inc && outc) HOT_GO(-1, false, true);
      else if (!inc && !outc) HOT_GO(-1, false, false);
      else return hipErrorInvalidValue;
    }
#undef HOT_GO
    return hipGetLastError();
  }
  static hipError_t strided(hipStream_t s, int variant, int dir, bool inc, bool outc, const void* in, void* out,
                            long ncols, long Qp, long ld_in, long ld_out, long bs_in, long bs_out, long cs_in,
                            long cs_out, int ncomp, long is_in, long is_out, long otw, int nb, const Geo& g,
                            const int* act) {
    switch (variant) {
      case 0: return strided_w<WV0>(s, dir, inc, outc, in, out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in,
                                    cs_out, ncomp, is_in, is_out, otw, nb, g, act);
      case 2: return strided_w<WV2>(s, dir, inc, outc, in, out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in,
                                    cs_out, ncomp, is_in, is_out, otw, nb, g, act);
      default: return strided_w<W>(s, dir, inc, outc, in, out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in,
                                   cs_out, ncomp, is_in, is_out, otw, nb, g, act);
    }
  }
  // g is the 2/3-rule geometry of N with no row padding (geo_two_thirds):
  // kernels instantiated for it take the geometry at compile time
  static bool is_g23(const Geo& g) {
    constexpr int K = (N - 1) / 3;
    return g.N == N && g.lo == K + 1 && g.hi == K && g.M == 2 * K + 1 && g.Mz == K + 1 && g.Mzp == K + 1 &&
           g.kz0 == 0 && g.tw == g.M * g.Mzp;
  }
  // short FP32 lines: all six outputs of a tile in one block (k_x_inv_curl6)
  static constexpr bool kCurl6 = std::is_same_v<T, float> && N <= 64;
  // 1/N^3 of the inverse transform (Eq. ffteq), applied to u and w by the x pass
  static constexpr double kUsc = 1.0 / (double(N) * N * N);
  // SIX (large N): one output per block (k_x_inv_curl, six blocks per tile)
  // instead of two (k_x_inv_curl3)
  template <int WW, bool SIX = false>
  static hipError_t x_inv_curl_w(hipStream_t s, const void* U, long csU, long isU, void* A, long csA, long isA,
                                 int nb, const Geo& g, const int* act) {
    const T usc = T(kUsc);
    const long Q = (long)g.M * g.Mzp;
    const int ntiles = (int)((Q + WW - 1) / WW);
    constexpr int pair = (WW * (int)sizeof(cx<T>) < 128) ? 128 / (WW * (int)sizeof(cx<T>)) : 1;
    const unsigned ngrp = (unsigned)((ntiles + 8 * pair - 1) / (8 * pair) * pair);
    if constexpr (kCurl6) {
      if (is_g23(g))
        hipLaunchKernelGGL((k_x_inv_curl6<T, P, WW, true>), dim3(8u * ngrp, (unsigned)nb), dim3(WW * Tl), 0, s,
                           (const cx<T>*)U, csU, isU, (cx<T>*)A, csA, isA, ntiles, g, usc, act);
      else
        hipLaunchKernelGGL((k_x_inv_curl6<T, P, WW>), dim3(8u * ngrp, (unsigned)nb), dim3(WW * Tl), 0, s,
                           (const cx<T>*)U, csU, isU, (cx<T>*)A, csA, isA, ntiles, g, usc, act);
    } else if constexpr (SIX) {
      hipLaunchKernelGGL((k_x_inv_curl<T, P, WW>), dim3(8u * 6u * ngrp, (unsigned)nb), dim3(WW * Tl), 0, s,
                         (const cx<T>*)U, csU, isU, (cx<T>*)A, csA, isA, ntiles, g, usc, act);
    } else {
      // registers that can hold a retained row: the 2/3-rule count, or all
      constexpr int KL23 = (((N - 1) / 3 + 1) + Tl - 1) / Tl;
      if (g.lo <= KL23 * Tl && g.hi <= KL23 * Tl)
        hipLaunchKernelGGL((k_x_inv_curl3<T, P, WW, KL23>), dim3(8u * 3u * ngrp, (unsigned)nb), dim3(WW * Tl), 0, s,
                           (const cx<T>*)U, csU, isU, (cx<T>*)A, csA, isA, ntiles, g, usc, act);
      else
        hipLaunchKernelGGL((k_x_inv_curl3<T, P, WW, P::R>), dim3(8u * 3u * ngrp, (unsigned)nb), dim3(WW * Tl), 0,
                           s, (const cx<T>*)U, csU, isU, (cx<T>*)A, csA, isA, ntiles, g, usc, act);
    }
    return hipGetLastError();
  }
  static hipError_t x_inv_curl(hipStream_t s, int variant, const void* U, long csU, long isU, void* A, long csA,
                               long isA, int nb, const Geo& g, const int* act) {
    // variants 0..2: widths W/2, W, 2W; 3..5: the same with one output per block
    switch (variant) {
      case 0: return x_inv_curl_w<WV0>(s, U, csU, isU, A, csA, isA, nb, g, act);
      case 2: return x_inv_curl_w<WV2>(s, U, csU, isU, A, csA, isA, nb, g, act);
      case 3: return x_inv_curl_w<WV0, true>(s, U, csU, isU, A, csA, isA, nb, g, act);
      case 4: return x_inv_curl_w<W, true>(s, U, csU, isU, A, csA, isA, nb, g, act);
      case 5: return x_inv_curl_w<WV2, true>(s, U, csU, isU, A, csA, isA, nb, g, act);
      default: return x_inv_curl_w<W>(s, U, csU, isU, A, csA, isA, nb, g, act);
    }
  }
  using PZ = std::conditional_t<std::is_same_v<T, float>, typename LPz32<N>::P, typename LPz<N>::P>;
  static constexpr int lines_per_block() { return ZShape<PZ>::LPB; }
  template <class ZA>
  static hipError_t z_cross_za(hipStream_t s, void* A, long csA, long isA, long nlines, int nb, const Geo& g,
                               const int* act, ZA za) {
    const unsigned nblk = (unsigned)((nlines + lines_per_block() - 1) / lines_per_block());
    const dim3 grid(nblk, (unsigned)nb);
    // coefficients per lane: the 2/3-rule count, or the all-but-Nyquist one
    constexpr int KL23 = z_loads<PZ>((N - 1) / 3 + 1), KLall = z_loads<PZ>(N / 2);
    if (g.Mz <= KL23 * PZ::Tl)
      hipLaunchKernelGGL((k_z_cross<T, PZ, KL23, ZA>), grid, dim3(256), 0, s, (cx<T>*)A, csA, isA, nlines, g, act,
                         za);
    else if (g.Mz <= KLall * PZ::Tl)
      hipLaunchKernelGGL((k_z_cross<T, PZ, KLall, ZA>), grid, dim3(256), 0, s, (cx<T>*)A, csA, isA, nlines, g, act,
                         za);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  static hipError_t z_cross(hipStream_t s, void* A, long csA, long isA, long nlines, int nb, const Geo& g,
                            const int* act) {
    return z_cross_za(s, A, csA, isA, nlines, nb, g, act, ZContig{});
  }
  template <class ZA, int FORM>
  static hipError_t z_cross_packed_za(hipStream_t s, void* A, long csA, long isA, long nlines, int nb, const Geo& g,
                                      const int* act, ZA za) {
    const unsigned nblk = (unsigned)((nlines + lines_per_block() - 1) / lines_per_block());
    const dim3 grid(nblk, (unsigned)nb);
    constexpr int KL23 = z_loads<PZ>((N - 1) / 3 + 1), KLall = z_loads<PZ>(N / 2);
    if (g.Mz <= KL23 * PZ::Tl)
      hipLaunchKernelGGL((k_z_cross_packed<T, PZ, KL23, ZA, FORM>), grid, dim3(256), 0, s, (cx<T>*)A, csA, isA,
                         nlines, g, act, za);
    else if (g.Mz <= KLall * PZ::Tl)
      hipLaunchKernelGGL((k_z_cross_packed<T, PZ, KLall, ZA, FORM>), grid, dim3(256), 0, s, (cx<T>*)A, csA, isA,
                         nlines, g, act, za);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  // form 0: packed rows in and out; 1: c0, c1, c2 stored as half-spectrum rows
  // (for the component-row y forward pass); 2: component rows in as well
  // (from the component-row y inverse pass), packed on load
  static hipError_t z_cross_packed(hipStream_t s, void* A, long csA, long isA, long nlines, int nb, const Geo& g,
                                   const int* act, int form) {
    if (form == 2) return z_cross_packed_za<ZContig, 2>(s, A, csA, isA, nlines, nb, g, act, ZContig{});
    return form == 1 ? z_cross_packed_za<ZContig, 1>(s, A, csA, isA, nlines, nb, g, act, ZContig{})
                     : z_cross_packed_za<ZContig, 0>(s, A, csA, isA, nlines, nb, g, act, ZContig{});
  }
  // the y passes on packed rows: a grid like k_strided's, with blockIdx.y
  // the component pair (3 for the inverse, 2 for the forward)
  template <int WW, bool INV>
  static hipError_t ypack_w(hipStream_t s, const void* in, void* out, long ncols, long Qp, long ld_in, long ld_out,
                            long bs_in, long bs_out, long cs_in, long cs_out, long is_in, long is_out, int nb,
                            const Geo& g, const int* act, bool single) {
    constexpr int pair = (WW * (int)sizeof(cx<T>) < 128) ? 128 / (WW * (int)sizeof(cx<T>)) : 1;
    const long ntiles = (ncols + WW - 1) / WW;
    const long group = 8L * pair;
    if (!INV && single) {  // one output per block, the three blocks of a tile consecutive on one XCD
      constexpr int KL23 = (((N - 1) / 3 + 1) + Tl - 1) / Tl;
      const dim3 grid3((unsigned)(3 * ((ntiles + group - 1) / group * group)), (unsigned)nb);
      if (g.lo <= KL23 * Tl && g.hi <= KL23 * Tl)
        hipLaunchKernelGGL((k_y_fwd_unpack3<T, P, WW, KL23>), grid3, dim3(WW * Tl), 0, s, (const cx<T>*)in,
                           (cx<T>*)out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, is_in, is_out, g, act);
      else
        hipLaunchKernelGGL((k_y_fwd_unpack3<T, P, WW, P::R>), grid3, dim3(WW * Tl), 0, s, (const cx<T>*)in,
                           (cx<T>*)out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, is_in, is_out, g, act);
      return hipGetLastError();
    }
    const dim3 grid((unsigned)((ntiles + group - 1) / group * group), INV ? 3u : 2u, (unsigned)nb);
    constexpr int KL23 = (((N - 1) / 3 + 1) + Tl - 1) / Tl;
    const bool cut = g.lo <= KL23 * Tl && g.hi <= KL23 * Tl;
#define HOT_YP(K)                                                                                                  \
  hipLaunchKernelGGL((INV ? k_y_inv_pack<T, P, WW, K> : k_y_fwd_unpack<T, P, WW, K>), grid, dim3(WW * Tl), 0, s, \
                     (const cx<T>*)in, (cx<T>*)out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, is_in,  \
                     is_out, g, act)
    if (cut) HOT_YP(KL23);
    else HOT_YP(P::R);
#undef HOT_YP
    return hipGetLastError();
  }
  template <bool INV>
  static hipError_t ypack(hipStream_t s, int variant, const void* in, void* out, long ncols, long Qp, long ld_in,
                          long ld_out, long bs_in, long bs_out, long cs_in, long cs_out, long is_in, long is_out,
                          int nb, const Geo& g, const int* act) {
    const bool single = variant >= 3;  // y forward: one output per block
    switch (variant % 3) {
      case 0: return ypack_w<WV0, INV>(s, in, out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, is_in,
                                       is_out, nb, g, act, single);
      case 2: return ypack_w<WV2, INV>(s, in, out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, is_in,
                                       is_out, nb, g, act, single);
      default: return ypack_w<W, INV>(s, in, out, ncols, Qp, ld_in, ld_out, bs_in, bs_out, cs_in, cs_out, is_in,
                                      is_out, nb, g, act, single);
    }
  }
  static hipError_t z_cross_blocked(hipStream_t s, void* A, long csA, long nlines, const Geo& g, int chunk,
                                    long blk) {
    if (chunk < 1) return hipErrorInvalidValue;
    return z_cross_za(s, A, csA, 0, nlines, 1, g, nullptr, ZBlocked{chunk, 1.0f / (float)chunk, blk});
  }
  static hipError_t z_cross_packed_blocked(hipStream_t s, void* A, long csA, long nlines, const Geo& g, int chunk,
                                           long blk, int form) {
    if (chunk < 1) return hipErrorInvalidValue;
    const ZBlocked za{chunk, 1.0f / (float)chunk, blk};
    if (form == 2) return z_cross_packed_za<ZBlocked, 2>(s, A, csA, 0, nlines, 1, g, nullptr, za);
    return form == 1 ? z_cross_packed_za<ZBlocked, 1>(s, A, csA, 0, nlines, 1, g, nullptr, za)
                     : z_cross_packed_za<ZBlocked, 0>(s, A, csA, 0, nlines, 1, g, nullptr, za);
  }
  static constexpr bool kYz = N <= 64 && YzShape<T, PZ>::kFits;
  static hipError_t yz_fused(hipStream_t s, void* A, long csA, long isA, int nb, const Geo& g, const int* act) {
    if constexpr (kYz) {
      const size_t lds = (size_t)YzShape<T, PZ>::lds_bytes(g.Mz);
      const dim3 grid((unsigned)N, (unsigned)nb);
      constexpr int K = (N - 1) / 3;
      constexpr int KL23 = z_loads<PZ>(K + 1), KLall = z_loads<PZ>(N / 2);
      if (is_g23(g)) {  // the 2/3 rule: the geometry at compile time
        (void)hipFuncSetAttribute((const void*)k_yz_fused<T, PZ, KL23, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_yz_fused<T, PZ, KL23, true>), grid, dim3(YzShape<T, PZ>::NT), lds, s, (cx<T>*)A, csA,
                           isA, g, act);
      } else if (g.Mz <= KL23 * PZ::Tl) {
        (void)hipFuncSetAttribute((const void*)k_yz_fused<T, PZ, KL23, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_yz_fused<T, PZ, KL23, false>), grid, dim3(YzShape<T, PZ>::NT), lds, s, (cx<T>*)A, csA,
                           isA, g, act);
      } else if (g.Mz <= KLall * PZ::Tl) {
        (void)hipFuncSetAttribute((const void*)k_yz_fused<T, PZ, KLall, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_yz_fused<T, PZ, KLall, false>), grid, dim3(YzShape<T, PZ>::NT), lds, s, (cx<T>*)A, csA,
                           isA, g, act);
      } else {
        return hipErrorInvalidValue;
      }
      return hipGetLastError();
    } else {
      (void)s, (void)A, (void)csA, (void)isA, (void)nb, (void)g, (void)act;
      return hipErrorInvalidValue;
    }
  }
  static hipError_t z_c2r(hipStream_t s, const void* in, void* out, long nlines, const Geo& g) {
    const unsigned nblk = (unsigned)((nlines + lines_per_block() - 1) / lines_per_block());
    const T scale = T(1.0 / (double(N) * N * N));
    hipLaunchKernelGGL((k_z_c2r<T, PZ>), dim3(nblk), dim3(256), 0, s, (const cx<T>*)in, (T*)out, nlines, g, scale);
    return hipGetLastError();
  }
  static hipError_t z_r2c(hipStream_t s, const void* in, void* out, long nlines, const Geo& g) {
    const unsigned nblk = (unsigned)((nlines + lines_per_block() - 1) / lines_per_block());
    hipLaunchKernelGGL((k_z_r2c<T, PZ>), dim3(nblk), dim3(256), 0, s, (const T*)in, (cx<T>*)out, nlines, g);
    return hipGetLastError();
  }
  static hipError_t rk_stage(hipStream_t s, const void* Nh, void* U0, void* U1, void* Acc, long C, long is, int nb,
                             const Geo& g, int mode, double nu, double dt) {
    hipLaunchKernelGGL((k_rk_stage<T>), dim3(grid_1d(C, 256), (unsigned)nb), dim3(256), 0, s, (const cx<T>*)Nh,
                       (cx<T>*)U0, (cx<T>*)U1, (cx<T>*)Acc, C, is, g, mode, T(nu), T(dt));
    return hipGetLastError();
  }
  using PF = typename LPf<N>::P;
  static constexpr int TlF = PF::Tl;
  template <int WW>
  static hipError_t x_fwd_rk_w(hipStream_t s, const void* A, long csA, long isA, void* U0, void* U1, void* Acc,
                               long C, long isU, int nb, const Geo& g, int mode, double nu, double dt) {
    constexpr int pair = (WW * (int)sizeof(cx<T>) < 128) ? 128 / (WW * (int)sizeof(cx<T>)) : 1;
    const long Q = (long)g.M * g.Mzp;
    const long ntiles = (Q + WW - 1) / WW;
    const long group = 8L * pair;
    const dim3 grid((unsigned)((ntiles + group - 1) / group * group), (unsigned)nb);
    // registers that can hold a retained row: the 2/3-rule count, or all
    constexpr int KL23 = (((N - 1) / 3 + 1) + TlF - 1) / TlF;
    if constexpr (N <= 64) {  // the batch sizes: the geometry at compile time where it is the 2/3 rule's
      if (is_g23(g)) {
        hipLaunchKernelGGL((k_x_fwd_rk<T, PF, WW, KL23, true>), grid, dim3(WW * TlF), 0, s, (const cx<T>*)A, csA,
                           isA, (cx<T>*)U0, (cx<T>*)U1, (cx<T>*)Acc, C, isU, g, mode, T(nu), T(dt));
        return hipGetLastError();
      }
    }
    if (g.lo <= KL23 * TlF && g.hi <= KL23 * TlF)
      hipLaunchKernelGGL((k_x_fwd_rk<T, PF, WW, KL23>), grid, dim3(WW * TlF), 0, s, (const cx<T>*)A, csA, isA,
                         (cx<T>*)U0, (cx<T>*)U1, (cx<T>*)Acc, C, isU, g, mode, T(nu), T(dt));
    else
      hipLaunchKernelGGL((k_x_fwd_rk<T, PF, WW, PF::R>), grid, dim3(WW * TlF), 0, s, (const cx<T>*)A, csA, isA,
                         (cx<T>*)U0, (cx<T>*)U1, (cx<T>*)Acc, C, isU, g, mode, T(nu), T(dt));
    return hipGetLastError();
  }
  // fused variants: W/2, W and W/4 columns per block (three components in
  // registers), within 1024 threads and at least one wave
  static constexpr bool fitsF(int w) { return w >= 1 && w * TlF <= 1024 && w * TlF >= 64; }
  static constexpr int WF = fitsF(W) ? W : W / 2;
  static constexpr int WF0 = fitsF(WF / 2) ? WF / 2 : WF;
  static constexpr int WQ = fitsF(WF / 4) ? WF / 4 : WF0;
  static hipError_t x_fwd_rk(hipStream_t s, int variant, const void* A, long csA, long isA, void* U0, void* U1,
                             void* Acc, long C, long isU, int nb, const Geo& g, int mode, double nu, double dt) {
    if (variant == 0) return x_fwd_rk_w<WF0>(s, A, csA, isA, U0, U1, Acc, C, isU, nb, g, mode, nu, dt);
    if (variant == 2) return x_fwd_rk_w<WQ>(s, A, csA, isA, U0, U1, Acc, C, isU, nb, g, mode, nu, dt);
    return x_fwd_rk_w<WF>(s, A, csA, isA, U0, U1, Acc, C, isU, nb, g, mode, nu, dt);
  }
  // the grid stride of k_gather in the digits of its loop
  static Pos4 gather_step(long stride, const Geo& g) {
    if (g.tw == g.M * g.Mzp) return pos4_of(stride, g.M, g.M, g.Mzp);
    return pos4_of(stride, g.M * (g.Mzp / g.tw), g.M, g.tw);
  }
  // compact rows per block of the transposing gather: about 22 KB of LDS
  // at N = 1024
  static constexpr int kRX = std::is_same_v<T, float> ? 8 : 4;
  static size_t transpose_lds(const Geo& g) { return (size_t)kRX * (g.Mzp + 1) * sizeof(cx<T>); }
  static hipError_t gather(hipStream_t s, const void* in0, const void* const* in_tab, void* out, long C, long is,
                           int nb, const Geo& g) {
    if (g.tw < g.M * g.Mzp) {  // column-tiled state: through LDS
      const size_t lds = transpose_lds(g);
      hipError_t e = hipFuncSetAttribute((const void*)k_gather_t<T, kRX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
      if (e != hipSuccess) return e;
      const dim3 grid((unsigned)((g.M + kRX - 1) / kRX), (unsigned)(3 * g.M), (unsigned)nb);
      hipLaunchKernelGGL((k_gather_t<T, kRX>), grid, dim3(256), lds, s, (const cx<T>*)in0,
                         (const cx<T>* const*)in_tab, (cx<T>*)out, C, is, g);
      return hipGetLastError();
    }
    const unsigned grid = grid_1d((3 * C + 3) / 4, 256);  // a few elements per thread
    hipLaunchKernelGGL((k_gather<T>), dim3(grid, (unsigned)nb), dim3(256), 0, s, (const cx<T>*)in0,
                       (const cx<T>* const*)in_tab, (cx<T>*)out, C, is, g, gather_step(256L * grid, g));
    return hipGetLastError();
  }
  static hipError_t scatter(hipStream_t s, const void* in, void* out0, void* const* out_tab, long C, long is, int nb,
                            const Geo& g) {
    const long total = 3L * g.N * g.N * g.czp;
    const unsigned grid = grid_1d((total + 3) / 4, 256);  // a few elements per thread
    hipLaunchKernelGGL((k_scatter<T>), dim3(grid, (unsigned)nb), dim3(256), 0, s, (const cx<T>*)in,
                       (cx<T>*)out0, (cx<T>* const*)out_tab, C, is, g, pos4_of(256L * grid, g.N, g.N, g.czp));
    return hipGetLastError();
  }
  static hipError_t imp_predict(hipStream_t s, const void* U0, void* D, void* U1, const void* H1, const void* H2,
                                const void* H3, const void* H4, long C, long is, int nb, const Geo& g, int hist,
                                int* act) {
    hipLaunchKernelGGL((k_imp_predict<T>), dim3(grid_1d(C, 256), (unsigned)nb), dim3(256), 0, s, (const cx<T>*)U0,
                       (cx<T>*)D, (cx<T>*)U1, (const cx<T>*)H1, (const cx<T>*)H2, (const cx<T>*)H3,
                       (const cx<T>*)H4, C, is, g, hist, act);
    return hipGetLastError();
  }
  static hipError_t imp_update(hipStream_t s, const void* Nh, const void* U0, void* D, void* U1, double* part, long C,
                               long is, int nb, const Geo& g, double nu, double dt, const int* act) {
    hipLaunchKernelGGL((k_imp_update<T>), dim3(grid_1d(C, 256), (unsigned)nb), dim3(256), 0, s, (const cx<T>*)Nh,
                       (const cx<T>*)U0, (cx<T>*)D, (cx<T>*)U1, part, C, is, g, T(nu), T(dt), act);
    return hipGetLastError();
  }
  static hipError_t imp_advance(hipStream_t s, void* U0, const void* D, long C, long is, int nb, const Geo& g) {
    hipLaunchKernelGGL((k_imp_advance<T>), dim3(grid_1d(C, 256), (unsigned)nb), dim3(256), 0, s, (cx<T>*)U0,
                       (const cx<T>*)D, C, is, g);
    return hipGetLastError();
  }
  static Ops ops() {
    return Ops{&strided,     &x_inv_curl, &z_cross,    &ypack<true>, &z_cross_packed, &ypack<false>, &z_cross_blocked, &z_cross_packed_blocked,
               kYz ? &yz_fused : nullptr,   &z_c2r,      &z_r2c,      &rk_stage,
               &x_fwd_rk,    &gather,     &scatter,    &imp_predict,
               &imp_update,  &imp_advance, 3,          {WV0, W, WV2}, {WF0, WF, WQ}};
  }
};

#define HOT_SIZES(X) X(8) X(16) X(18) X(24) X(32) X(36) X(48) X(54) X(64) X(128) X(256) X(512) X(1024) X(2048)

#define HOT_DECLARE_OPS(n)  \
  Ops make_ops_f32_##n();   \
  Ops make_ops_f64_##n();
HOT_SIZES(HOT_DECLARE_OPS)
#undef HOT_DECLARE_OPS

}  // namespace hot
