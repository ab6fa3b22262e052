// Kernels of the per-mode MLP surrogate that warm-starts the Picard
// iteration of the implicit-midpoint step: 32 -> 256 -> 256 -> 256 -> 6,
// tanh on the hidden layers, BF16 MFMA operands (v_mfma_f32_16x16x32_bf16)
// with FP32 accumulation, FP32 master weights.
//
// MFMA 16x16x32 operand layout (lane l of a wave):
//   A (16 x 32): row l % 16, k = 8 (l / 16) .. +8   (8 bf16 per lane)
//   B (32 x 16): col l % 16, k = 8 (l / 16) .. +8
//   D (16 x 16): col l % 16, rows 4 (l / 16) .. +4  (4 fp32 per lane)
// The training GEMM puts activations in A and weights in B; the fused
// inference kernel the other way round (D = W x act^T), so that a lane's
// four results are consecutive features of one row.
//
// Parameters (one FP32 vector, weights W[out][in]):
//   W1[256][32] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[6][256] b4[6]
// Packed inference copy (bytes): BF16 W1[256][32], W2[256][256],
//   W3[256][256], W4[16][256] (rows 6..15 zero), then FP32 b1[256], b2[256],
//   b3[256], b4[16] (entries 6..15 zero).
//
// Surrogate features of a retained mode (per mode, FP32), with D1, D2 the
// increments of the two previous steps (newest first), s = ||D1_k|| over the
// three complex components, a = dt nu |k|^2 / 2:
//   f[0:6] D1/s, f[6:12] D2/s, f[12:18] ((1 - a) D1 + 2 a u)/s (the previous
//   step's dt F_NL at its fixed point), f[18:24] u/||u_k||, f[24] s/||u_k||,
//   f[25:28] k/N, f[28] a, f[29:32] 0; all zero when s = 0.
// Prediction: d = 2 D1 - D2 + s y, y = MLP(f).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hot {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 32, kHid = 256, kOut = 6, kOutPad = 16;
constexpr long kParamCount = (long)kHid * kIn + kHid + 2L * (kHid * kHid + kHid) + (long)kOut * kHid + kOut;
// offsets (floats) of the parameter blocks
constexpr long kW1 = 0, kB1 = kW1 + kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid, kW3 = kB2 + kHid,
               kB3 = kW3 + kHid * kHid, kW4 = kB3 + kHid, kB4 = kW4 + kOut * kHid;
// offsets (bytes) of the packed copy
constexpr long kPW1 = 0, kPW2 = kPW1 + 2L * kHid * kIn, kPW3 = kPW2 + 2L * kHid * kHid,
               kPW4 = kPW3 + 2L * kHid * kHid, kPB1 = kPW4 + 2L * kOutPad * kHid, kPB2 = kPB1 + 4L * kHid,
               kPB3 = kPB2 + 4L * kHid, kPB4 = kPB3 + 4L * kHid, kPackedBytes = kPB4 + 4L * kOutPad;

// FP32 -> BF16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ unsigned pack2(float a, float b) {
  const bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}
__device__ __forceinline__ unsigned short bf16_bits(float f) { return (unsigned short)(pack2(f, 0.f) & 0xFFFFu); }

// tanh(x) = 1 - 2 / (1 + e^{2x}) on the hardware exp2 and reciprocal; its
// absolute error (a few 1e-7) is far below the BF16 rounding the result
// then takes.  Saturates to +-1 for large |x|.
__device__ __forceinline__ float fast_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // e^{2x}
  return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + e);
}
__device__ __forceinline__ bf16x8 lds_frag(const unsigned short* p) { return *(const bf16x8*)p; }
__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Training GEMM: C(m, n) = epi(sum_k A(m, k) B(k, n)) for FP32 operands with
// arbitrary strides, rounded to BF16 while staged into LDS.  64 x 64 tile per
// 256-thread block (2 x 2 waves of 32 x 32), k-steps of 32.  Split K:
// blockIdx.z sums k in [z kchunk, (z + 1) kchunk) into C + z csz (EPI_NONE;
// k_split_sum adds the pieces).
//   EPI_NONE: C = acc
//   EPI_BIAS: C = acc + bias[n]
//   EPI_BIAS_TANH: C = tanh(acc + bias[n])
//   EPI_DTANH: C = acc * (1 - H(m, n)^2)   (backward through tanh)
// ---------------------------------------------------------------------------
enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3 };

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, long sam, long sak,
                                              const float* __restrict__ B, long sbk, long sbn,
                                              float* __restrict__ C, long scm, long scn,
                                              const float* __restrict__ bias, const float* __restrict__ H, long shm,
                                              long shn, int kchunk, long csz) {
  constexpr int LD = 40;  // 32 + 8: rows 80 bytes apart, conflict-free 16-byte fragment reads
  __shared__ __attribute__((aligned(16))) unsigned short As[64 * LD];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[64 * LD];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int sr = t >> 2, sk = (t & 3) * 8;  // staging: row (of A) or column (of B), k chunk
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  C += blockIdx.z * csz;
  for (int k0 = kb; k0 < ke; k0 += 32) {
    float av[8], bv[8];
    const int m = m0 + sr, n = n0 + sr;
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + sk + i;
      av[i] = (m < M && k < ke) ? A[m * sam + k * sak] : 0.f;
      bv[i] = (n < N && k < ke) ? B[k * sbk + n * sbn] : 0.f;
    }
    __syncthreads();  // the previous step's fragments have been read
    *(uint4*)&As[sr * LD + sk] = uint4{pack2(av[0], av[1]), pack2(av[2], av[3]), pack2(av[4], av[5]), pack2(av[6], av[7])};
    *(uint4*)&Bs[sr * LD + sk] = uint4{pack2(bv[0], bv[1]), pack2(bv[2], bv[3]), pack2(bv[4], bv[5]), pack2(bv[6], bv[7])};
    __syncthreads();
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i) a[i] = lds_frag(&As[(wm + 16 * i + (l & 15)) * LD + 8 * (l >> 4)]);
    for (int j = 0; j < 2; ++j) b[j] = lds_frag(&Bs[(wn + 16 * j + (l & 15)) * LD + 8 * (l >> 4)]);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (l >> 4) + r, n = n0 + wn + 16 * j + (l & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i][j][r];
        if (EPI == EPI_BIAS || EPI == EPI_BIAS_TANH) v += bias[n];
        if (EPI == EPI_BIAS_TANH) v = tanhf(v);
        if (EPI == EPI_DTANH) {
          const float h = H[m * shm + n * shn];
          v *= 1.f - h * h;
        }
        C[m * scm + n * scn] = v;
      }
}

// C(m, n) = sum over z < nz of P[z][m][n] (fixed order), P of [nz][M][N].
__global__ __launch_bounds__(256) void k_split_sum(const float* __restrict__ P, int nz, int M, int N,
                                                   float* __restrict__ C, long scm, long scn) {
  const long MN = (long)M * N;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < MN; i += (long)gridDim.x * 256) {
    float s = 0.f;
    for (int z = 0; z < nz; ++z) s += P[z * MN + i];
    const int m = (int)(i / N), n = (int)(i - (long)m * N);
    C[m * scm + n * scn] = s;
  }
}

// Loss and output gradient: R = Y - T, dY = 2 R / (rows * 6); part[block] =
// the block's sum of R^2 (summed in a fixed order).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             float* __restrict__ dY, double* __restrict__ part, long count) {
  __shared__ double red[4];
  double acc = 0.0;
  const float sc = 2.f / (float)count;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) {
    const float r = Y[i] - T[i];
    dY[i] = sc * r;
    acc += (double)r * r;
  }
  acc = block_sum_256(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// loss = sum(part[0..n)) / count, one wave, fixed order.
__global__ __launch_bounds__(64) void k_loss_final(const double* __restrict__ part, int n, long count,
                                                   float* __restrict__ loss) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += part[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) *loss = (float)(s / (double)count);
}

// Column sums (bias gradients): g[n] = sum_m Z(m, n), Z row-major [rows][ncol];
// one block per column, fixed order.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ Z, int rows, int ncol, float* __restrict__ g) {
  __shared__ double red[4];
  const int n = blockIdx.x;
  double s = 0.0;
  for (int m = threadIdx.x; m < rows; m += 256) s += Z[(long)m * ncol + n];
  s = block_sum_256(s, red);
  if (threadIdx.x == 0) g[n] = (float)s;
}

// Adam (Kingma and Ba, 2015) with bias correction; step counts from 1.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// FP32 parameters -> packed inference copy.
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ th, unsigned char* __restrict__ pk) {
  unsigned short* w1 = (unsigned short*)(pk + kPW1);
  unsigned short* w2 = (unsigned short*)(pk + kPW2);
  unsigned short* w3 = (unsigned short*)(pk + kPW3);
  unsigned short* w4 = (unsigned short*)(pk + kPW4);
  float* b1 = (float*)(pk + kPB1);
  float* b2 = (float*)(pk + kPB2);
  float* b3 = (float*)(pk + kPB3);
  float* b4 = (float*)(pk + kPB4);
  const long stride = (long)gridDim.x * 256;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < (long)kHid * kHid; i += stride) {
    w2[i] = bf16_bits(th[kW2 + i]);
    w3[i] = bf16_bits(th[kW3 + i]);
    if (i < (long)kHid * kIn) w1[i] = bf16_bits(th[kW1 + i]);
    if (i < (long)kOutPad * kHid) w4[i] = i < (long)kOut * kHid ? bf16_bits(th[kW4 + i]) : (unsigned short)0;
    if (i < kHid) {
      b1[i] = th[kB1 + i];
      b2[i] = th[kB2 + i];
      b3[i] = th[kB3 + i];
    }
    if (i < kOutPad) b4[i] = i < kOut ? th[kB4 + i] : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Fused inference: 256 rows per 512-thread block, 8 waves of 32 rows.  The
// activations of a row stay in LDS (BF16) through all layers; each wave owns
// its 32 rows, so only the weight slices staged into LDS (256 x 32 per
// k-step, shared by the 8 waves) need block barriers.
// ---------------------------------------------------------------------------
constexpr int kRows = 256, kThreads = 512, kActLd = 264, kWLd = 40;

template <int NT>
__device__ __forceinline__ void mlp_layer(const unsigned short* __restrict__ Wg, int K,
                                          const unsigned short* __restrict__ act, unsigned short* __restrict__ Ws,
                                          int row0, f32x4 (&acc)[2][NT]) {
  const int t = threadIdx.x, l = t & 63;
  for (int i = 0; i < 2; ++i)
    for (int n = 0; n < NT; ++n) acc[i][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    __syncthreads();  // every wave is done with the previous slice
    for (int c = t; c < NT * 16 * 4; c += kThreads) {
      const int n = c >> 2, q = c & 3;
      *(uint4*)&Ws[n * kWLd + q * 8] = *(const uint4*)&Wg[(long)n * K + k0 + q * 8];
    }
    __syncthreads();
    const bf16x8 a0 = lds_frag(&act[(row0 + (l & 15)) * kActLd + k0 + 8 * (l >> 4)]);
    const bf16x8 a1 = lds_frag(&act[(row0 + 16 + (l & 15)) * kActLd + k0 + 8 * (l >> 4)]);
    // weights as the A operand, activations as B: lane l then holds output
    // features 4 (l / 16) .. +4 of row l % 16, written back as one 8-byte store
    for (int n = 0; n < NT; ++n) {
      const bf16x8 w = lds_frag(&Ws[(n * 16 + (l & 15)) * kWLd + 8 * (l >> 4)]);
      acc[0][n] = mfma16(w, a0, acc[0][n]);
      acc[1][n] = mfma16(w, a1, acc[1][n]);
    }
  }
}

// Hidden-layer epilogue: the wave's rows <- bf16(tanh(acc + b)); acc[i][n]
// holds features n*16 + 4 (l / 16) .. +4 of row row0 + 16 i + l % 16.
__device__ __forceinline__ void mlp_hidden_out(const f32x4 (&acc)[2][16], const float* __restrict__ bias,
                                               unsigned short* __restrict__ act, int row0) {
  const int l = threadIdx.x & 63;
  for (int n = 0; n < 16; ++n) {
    const int f0 = n * 16 + 4 * (l >> 4);
    const float4 bb = *(const float4*)&bias[f0];
    for (int i = 0; i < 2; ++i) {
      const int row = row0 + 16 * i + (l & 15);
      const f32x4 v = acc[i][n];
      *(uint2*)&act[row * kActLd + f0] = uint2{pack2(fast_tanh(v[0] + bb.x), fast_tanh(v[1] + bb.y)),
                                               pack2(fast_tanh(v[2] + bb.z), fast_tanh(v[3] + bb.w))};
    }
  }
}

// Features of one retained mode (see the top of this file) from the state u
// and the increments d1 (newest), d2, as (re, im) x 3 FP32 values; returns s.
__device__ __forceinline__ float surrogate_features(const float (&u)[6], const float (&d1)[6], const float (&d2)[6],
                                                    const ModeK& m, int N, float nu, float dt, float (&f)[kIn]) {
  for (int i = 0; i < kIn; ++i) f[i] = 0.f;
  float ss = 0.f, su = 0.f;
  for (int i = 0; i < 6; ++i) {
    ss += d1[i] * d1[i];
    su += u[i] * u[i];
  }
  const float s = sqrtf(ss);
  if (s > 0.f) {
    const float inv = 1.f / s;
    const float a = 0.5f * dt * nu * (float)(m.kx * m.kx + m.ky * m.ky + m.kz * m.kz);
    const float nrm = sqrtf(su), invu = nrm > 0.f ? 1.f / nrm : 0.f;
    for (int i = 0; i < 6; ++i) {
      f[i] = d1[i] * inv;
      f[6 + i] = d2[i] * inv;
      f[12 + i] = ((1.f - a) * d1[i] + 2.f * a * u[i]) * inv;
      f[18 + i] = u[i] * invu;
    }
    f[24] = s * invu;
    const float invN = 1.f / (float)N;
    f[25] = (float)m.kx * invN;
    f[26] = (float)m.ky * invN;
    f[27] = (float)m.kz * invN;
    f[28] = a;
  }
  return s;
}

// Feature source / result sink of the fused kernel.
//   MLP_ARRAYS:  X[rows][32] FP32 in, Y[rows][6] FP32 out.
//   MLP_PREDICT: the implicit step's compact state of one group, U0, H1, H2
//                [B][3][C] of element type T; out: d and U1 = U0 + d/2.
enum { MLP_ARRAYS = 0, MLP_PREDICT = 1 };

template <typename T>
struct MlpState {
  const cx<T>* U0;
  const cx<T>* H1;
  const cx<T>* H2;
  cx<T>* D;
  cx<T>* U1;
  int* act;
  long C, is;  // slots per component, stride between instances
  int B;       // instances
  Geo g;
  float nu, dt;
};

template <typename T>
__device__ __forceinline__ bool mlp_row(const MlpState<T>& st, long gr, long& ib, long& e, ModeK& m) {
  const long b = gr / st.C;
  e = gr - b * st.C;
  ib = b * st.is;
  return b < st.B && mode_of(e, st.g, m);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_mlp_fused(const unsigned char* __restrict__ pk, long rows,
                                                        const float* __restrict__ X, float* __restrict__ Y,
                                                        MlpState<T> st) {
  __shared__ __attribute__((aligned(16))) unsigned short act[kRows * kActLd];
  __shared__ __attribute__((aligned(16))) unsigned short Ws[kHid * kWLd];  // also the FP32 outputs at the end
  __shared__ float srow[kRows];
  const int t = threadIdx.x, w = t >> 6;
  const long tile0 = (long)blockIdx.x * kRows;
  const int row0 = w * 32;
  // features -> act[:, 0:32]
  if (t < kRows) {
    const long gr = tile0 + t;
    float f[kIn];
    for (int i = 0; i < kIn; ++i) f[i] = 0.f;
    float s = 0.f;
    if (MODE == MLP_ARRAYS) {
      if (gr < rows)
        for (int i = 0; i < kIn; ++i) f[i] = X[gr * kIn + i];
    } else {
      long ib, e;
      ModeK m;
      if (gr < rows && mlp_row(st, gr, ib, e, m)) {
        if (e == 0) st.act[gr / st.C] = 1;
        float u[6], d1[6], d2[6];
        for (int c = 0; c < 3; ++c) {
          const long i = ib + c * st.C + e;
          const cx<T> a = st.U0[i], b = st.H1[i], q = st.H2[i];
          u[2 * c] = (float)a.x;
          u[2 * c + 1] = (float)a.y;
          d1[2 * c] = (float)b.x;
          d1[2 * c + 1] = (float)b.y;
          d2[2 * c] = (float)q.x;
          d2[2 * c + 1] = (float)q.y;
        }
        s = surrogate_features(u, d1, d2, m, st.g.N, st.nu, st.dt, f);
      }
    }
    srow[t] = s;
    uint4* dst = (uint4*)&act[t * kActLd];
    for (int q = 0; q < 4; ++q)
      dst[q] = uint4{pack2(f[8 * q], f[8 * q + 1]), pack2(f[8 * q + 2], f[8 * q + 3]), pack2(f[8 * q + 4], f[8 * q + 5]),
                     pack2(f[8 * q + 6], f[8 * q + 7])};
  }
  __syncthreads();
  f32x4 acc[2][16];
  mlp_layer<16>((const unsigned short*)(pk + kPW1), kIn, act, Ws, row0, acc);
  mlp_hidden_out(acc, (const float*)(pk + kPB1), act, row0);
  mlp_layer<16>((const unsigned short*)(pk + kPW2), kHid, act, Ws, row0, acc);
  mlp_hidden_out(acc, (const float*)(pk + kPB2), act, row0);
  mlp_layer<16>((const unsigned short*)(pk + kPW3), kHid, act, Ws, row0, acc);
  mlp_hidden_out(acc, (const float*)(pk + kPB3), act, row0);
  f32x4 out[2][1];
  mlp_layer<1>((const unsigned short*)(pk + kPW4), kHid, act, Ws, row0, out);
  __syncthreads();  // every wave is done with the last weight slice
  float* yl = (float*)Ws;  // [256 rows][8]
  {
    const int l = t & 63;
    const float* b4 = (const float*)(pk + kPB4);
    for (int i = 0; i < 2; ++i)
      for (int r = 0; r < 4; ++r) {
        const int f = 4 * (l >> 4) + r;  // output feature; lane l % 16 is the row
        if (f < kOut) yl[(row0 + 16 * i + (l & 15)) * 8 + f] = out[i][0][r] + b4[f];
      }
  }
  __syncthreads();
  if (t < kRows) {
    const long gr = tile0 + t;
    if (MODE == MLP_ARRAYS) {
      if (gr < rows)
        for (int c = 0; c < kOut; ++c) Y[gr * kOut + c] = yl[t * 8 + c];
    } else {
      long ib, e;
      ModeK m;
      if (gr < rows && mlp_row(st, gr, ib, e, m)) {
        const T s = (T)srow[t];
        for (int c = 0; c < 3; ++c) {
          const long i = ib + c * st.C + e;
          const cx<T> y = {(T)yl[t * 8 + 2 * c], (T)yl[t * 8 + 2 * c + 1]};
          const cx<T> d = st.H1[i] * T(2) - st.H2[i] + y * s;
          st.D[i] = d;
          st.U1[i] = st.U0[i] + d * T(0.5);
        }
      }
    }
  }
}

// Training rows of one N^3 field (2/3 rule), one thread per retained mode in
// canonical (kx, ky, kz) order: x[row][32] features, t[row][6] targets
// (d - (2 d1 - d2)) / s (0 where s = 0) when d is given, sc[row] = s when
// sc is given.  Canonical layout
// [3][N][N][N/2+1].
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_dataset(const cx<T>* __restrict__ u, const cx<T>* __restrict__ d1,
                                                     const cx<T>* __restrict__ d2, const cx<T>* __restrict__ d,
                                                     Geo g, float nu, float dt, float* __restrict__ x,
                                                     float* __restrict__ t, float* __restrict__ sc) {
  const long rows = (long)g.M * g.M * g.Mz;
  const long Nh = g.N / 2 + 1, comp = (long)g.N * g.N * Nh;
  for (long r = (long)blockIdx.x * 256 + threadIdx.x; r < rows; r += (long)gridDim.x * 256) {
    const int ix = (int)(r / ((long)g.M * g.Mz));
    const long rr = r - (long)ix * g.M * g.Mz;
    const int iy = (int)(rr / g.Mz);
    ModeK m;
    m.kz = (int)(rr - (long)iy * g.Mz);
    const int px = cpos(ix, g), py = cpos(iy, g);
    m.kx = kwave(px, g.N);
    m.ky = kwave(py, g.N);
    const long at = ((long)px * g.N + py) * Nh + m.kz;
    float fu[6], f1[6], f2[6];
    for (int c = 0; c < 3; ++c) {
      const cx<T> a = u[c * comp + at], b = d1[c * comp + at], q = d2[c * comp + at];
      fu[2 * c] = (float)a.x;
      fu[2 * c + 1] = (float)a.y;
      f1[2 * c] = (float)b.x;
      f1[2 * c + 1] = (float)b.y;
      f2[2 * c] = (float)q.x;
      f2[2 * c + 1] = (float)q.y;
    }
    float f[kIn];
    const float s = surrogate_features(fu, f1, f2, m, g.N, nu, dt, f);
    for (int i = 0; i < kIn; ++i) x[r * kIn + i] = f[i];
    if (sc) sc[r] = s;
    if (t) {
      for (int c = 0; c < 3; ++c) {
        const cx<T> e = d[c * comp + at] - (d1[c * comp + at] * T(2) - d2[c * comp + at]);
        t[r * kOut + 2 * c] = s > 0.f ? (float)(e.x / (T)s) : 0.f;
        t[r * kOut + 2 * c + 1] = s > 0.f ? (float)(e.y / (T)s) : 0.f;
      }
    }
  }
}

}  // namespace hot
