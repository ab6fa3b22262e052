// libhot: C ABI of the per-mode MLP surrogate (include/hot.h) and the
// warm-start launcher used by the implicit step.  Arithmetic: mlp.hpp.
#include <hip/hip_runtime.h>

#include "../../include/hot.h"
#include "mlp.hpp"
#include "mlp_launch.hpp"

namespace hot {

static inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <typename T>
hipError_t mlp_predict(hipStream_t s, const void* packed, const void* U0, const void* H1, const void* H2, void* D,
                       void* U1, int* act, long C, long is, int nb, const Geo& g, double nu, double dt) {
  MlpState<T> st;
  st.U0 = (const cx<T>*)U0;
  st.H1 = (const cx<T>*)H1;
  st.H2 = (const cx<T>*)H2;
  st.D = (cx<T>*)D;
  st.U1 = (cx<T>*)U1;
  st.act = act;
  st.C = C;
  st.is = is;
  st.B = nb;
  st.g = g;
  st.nu = (float)nu;
  st.dt = (float)dt;
  const long rows = (long)nb * C;
  const long blocks = (rows + kRows - 1) / kRows;
  hipLaunchKernelGGL((k_mlp_fused<T, MLP_PREDICT>), dim3((unsigned)blocks), dim3(kThreads), 0, s,
                     (const unsigned char*)packed, rows, (const float*)nullptr, (float*)nullptr, st);
  return hipGetLastError();
}

template hipError_t mlp_predict<float>(hipStream_t, const void*, const void*, const void*, const void*, void*, void*,
                                       int*, long, long, int, const Geo&, double, double);
template hipError_t mlp_predict<double>(hipStream_t, const void*, const void*, const void*, const void*, void*, void*,
                                        int*, long, long, int, const Geo&, double, double);

}  // namespace hot

using namespace hot;

namespace {

// Training workspace (floats unless noted): H1, H2, H3, dZa, dZb [rows][256],
// Y, dY [rows][6], the loss partial sums (doubles), then the split-K pieces
// of the weight gradients [nsplit][256][256].
constexpr int kSplitRows = 512;  // rows summed per split-K piece
struct TrainLayout {
  size_t h1, h2, h3, za, zb, y, dy, part, split, bytes;
  int nparts, nsplit;
  explicit TrainLayout(long rows) {
    const size_t big = (size_t)rows * kHid * sizeof(float), small = (size_t)rows * kOut * sizeof(float);
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    h1 = 0;
    h2 = h1 + up(big);
    h3 = h2 + up(big);
    za = h3 + up(big);
    zb = za + up(big);
    y = zb + up(big);
    dy = y + up(small);
    part = dy + up(small);
    long n = ((long)rows * kOut + 255) / 256;
    nparts = (int)(n > 1024 ? 1024 : n);
    split = part + up((size_t)nparts * sizeof(double));
    nsplit = (int)((rows + kSplitRows - 1) / kSplitRows);
    if (nsplit > 64) nsplit = 64;
    bytes = split + up((size_t)nsplit * kHid * kHid * sizeof(float));
  }
};

template <int EPI>
hipError_t gemm(hipStream_t s, int M, int N, int K, const float* A, long sam, long sak, const float* B, long sbk,
                long sbn, float* C, long scm, long scn, const float* bias = nullptr, const float* H = nullptr,
                long shm = 0, long shn = 0) {
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
  hipLaunchKernelGGL((k_gemm<EPI>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, bias, H,
                     shm, shn, K, 0L);
  return hipGetLastError();
}

// A weight gradient (M, N <= 256, K = rows): K split into nsplit pieces of
// whole 32-row steps, summed afterwards in a fixed order.
hipError_t gemm_wgrad(hipStream_t s, int M, int N, int K, const float* A, long sam, long sak, const float* B,
                      long sbk, long sbn, float* C, long scm, long scn, float* pieces, int nsplit) {
  const int kchunk = ((K + nsplit - 1) / nsplit + 31) / 32 * 32;
  const int nz = (K + kchunk - 1) / kchunk;
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)nz);
  hipLaunchKernelGGL((k_gemm<EPI_NONE>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, pieces, (long)N,
                     1L, (const float*)nullptr, (const float*)nullptr, 0L, 0L, kchunk, (long)M * N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long MN = (long)M * N;
  hipLaunchKernelGGL(k_split_sum, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, s, (const float*)pieces, nz, M,
                     N, C, scm, scn);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int32_t hot_mlp_param_count(void) { return (int32_t)kParamCount; }

size_t hot_mlp_packed_bytes(void) { return (size_t)kPackedBytes; }

int hot_mlp_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed || !aligned16(params) || !aligned16(packed)) return HOT_E_INVALID;
  hipLaunchKernelGGL(k_mlp_pack, dim3(256), dim3(256), 0, (hipStream_t)stream, params, (unsigned char*)packed);
  return hipGetLastError() == hipSuccess ? HOT_OK : HOT_E_HIP;
}

int hot_mlp_forward(const void* packed, const float* x, float* y, int64_t rows, void* stream) {
  if (!packed || !x || !y || rows < 0 || !aligned16(packed)) return HOT_E_INVALID;
  if (rows == 0) return HOT_OK;
  const long blocks = (long)((rows + kRows - 1) / kRows);
  if (blocks > 0x7fffffffL) return HOT_E_UNSUPPORTED;
  MlpState<float> none{};
  hipLaunchKernelGGL((k_mlp_fused<float, MLP_ARRAYS>), dim3((unsigned)blocks), dim3(kThreads), 0,
                     (hipStream_t)stream, (const unsigned char*)packed, (long)rows, x, y, none);
  return hipGetLastError() == hipSuccess ? HOT_OK : HOT_E_HIP;
}

size_t hot_mlp_train_bytes(int32_t rows) { return rows > 0 ? TrainLayout(rows).bytes : 0; }

int hot_mlp_grad(const float* th, const float* x, const float* t, int32_t rows, float* grad, float* loss, void* ws,
                 void* stream) {
  if (!th || !x || !t || !grad || !loss || !ws || rows < 1) return HOT_E_INVALID;
  if (((uintptr_t)ws & 255) != 0) return HOT_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const TrainLayout L(rows);
  char* base = (char*)ws;
  float *H1 = (float*)(base + L.h1), *H2 = (float*)(base + L.h2), *H3 = (float*)(base + L.h3);
  float *Za = (float*)(base + L.za), *Zb = (float*)(base + L.zb), *Y = (float*)(base + L.y);
  float* dY = (float*)(base + L.dy);
  double* part = (double*)(base + L.part);
  float* pieces = (float*)(base + L.split);
  const long R = rows, H = kHid;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t v) {
    if (e == hipSuccess) e = v;
  };
  // forward, keeping the activations
  ok(gemm<EPI_BIAS_TANH>(s, rows, kHid, kIn, x, kIn, 1, th + kW1, 1, kIn, H1, H, 1, th + kB1));
  ok(gemm<EPI_BIAS_TANH>(s, rows, kHid, kHid, H1, H, 1, th + kW2, 1, H, H2, H, 1, th + kB2));
  ok(gemm<EPI_BIAS_TANH>(s, rows, kHid, kHid, H2, H, 1, th + kW3, 1, H, H3, H, 1, th + kB3));
  ok(gemm<EPI_BIAS>(s, rows, kOut, kHid, H3, H, 1, th + kW4, 1, H, Y, kOut, 1, th + kB4));
  // loss and dL/dY
  hipLaunchKernelGGL(k_mse, dim3(L.nparts), dim3(256), 0, s, Y, t, dY, part, R * kOut);
  ok(hipGetLastError());
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, part, L.nparts, R * kOut, loss);
  ok(hipGetLastError());
  // output layer
  ok(gemm_wgrad(s, kOut, kHid, rows, dY, 1, kOut, H3, H, 1, grad + kW4, H, 1, pieces, L.nsplit));
  hipLaunchKernelGGL(k_colsum, dim3(kOut), dim3(256), 0, s, dY, rows, kOut, grad + kB4);
  ok(hipGetLastError());
  ok(gemm<EPI_DTANH>(s, rows, kHid, kOut, dY, kOut, 1, th + kW4, H, 1, Za, H, 1, nullptr, H3, H, 1));
  // hidden layers 3, 2, 1
  ok(gemm_wgrad(s, kHid, kHid, rows, Za, 1, H, H2, H, 1, grad + kW3, H, 1, pieces, L.nsplit));
  hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, Za, rows, kHid, grad + kB3);
  ok(hipGetLastError());
  ok(gemm<EPI_DTANH>(s, rows, kHid, kHid, Za, H, 1, th + kW3, H, 1, Zb, H, 1, nullptr, H2, H, 1));
  ok(gemm_wgrad(s, kHid, kHid, rows, Zb, 1, H, H1, H, 1, grad + kW2, H, 1, pieces, L.nsplit));
  hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, Zb, rows, kHid, grad + kB2);
  ok(hipGetLastError());
  ok(gemm<EPI_DTANH>(s, rows, kHid, kHid, Zb, H, 1, th + kW2, H, 1, Za, H, 1, nullptr, H1, H, 1));
  ok(gemm_wgrad(s, kHid, kIn, rows, Za, 1, H, x, kIn, 1, grad + kW1, kIn, 1, pieces, L.nsplit));
  hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, Za, rows, kHid, grad + kB1);
  ok(hipGetLastError());
  return e == hipSuccess ? HOT_OK : HOT_E_HIP;
}

int64_t hot_mlp_dataset_rows(int32_t N) {
  if (N < 8 || (N & 1)) return HOT_E_INVALID;
  const long K = (N - 1) / 3;
  return (2 * K + 1) * (2 * K + 1) * (K + 1);
}

int hot_mlp_dataset(int32_t N, int32_t dtype, const void* u, const void* d1, const void* d2, const void* d, double nu,
                    double dt, float* x, float* t, float* s_out, void* stream) {
  if (N < 8 || (N & 1) || !u || !d1 || !d2 || !x || (d && !t) || (dtype != HOT_F64 && dtype != HOT_F32))
    return HOT_E_INVALID;
  Geo g{};
  const int K = (N - 1) / 3;
  g.N = N;
  g.lo = K + 1;
  g.hi = K;
  g.M = 2 * K + 1;
  g.Mz = g.Mzp = K + 1;
  g.czp = N / 2 + 1;
  g.tw = g.M * g.Mzp;
  const long rows = (long)g.M * g.M * g.Mz;
  long blocks = (rows + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipStream_t s = (hipStream_t)stream;
  if (dtype == HOT_F64)
    hipLaunchKernelGGL(k_mlp_dataset<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const cx<double>*)u,
                       (const cx<double>*)d1, (const cx<double>*)d2, (const cx<double>*)d, g, (float)nu, (float)dt, x,
                       d ? t : nullptr, s_out);
  else
    hipLaunchKernelGGL(k_mlp_dataset<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const cx<float>*)u,
                       (const cx<float>*)d1, (const cx<float>*)d2, (const cx<float>*)d, g, (float)nu, (float)dt, x,
                       d ? t : nullptr, s_out);
  return hipGetLastError() == hipSuccess ? HOT_OK : HOT_E_HIP;
}

int hot_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                 float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || step < 1 || !(lr > 0.f)) return HOT_E_INVALID;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, (hipStream_t)stream, params, grad, m, v, (long)kParamCount,
                     lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? HOT_OK : HOT_E_HIP;
}

}  // extern "C"
