// Result checks outside the hot path: a scan of the retained modes for values
// that are not finite.  Kept apart from the pass kernels so that it never
// changes their code.
#pragma once

#include "kernels.hpp"

namespace hot {

// ---------------------------------------------------------------------------
// Finite check of a compact result [B][3][C] (row padding skipped): any NaN or
// infinity sets *flag to 1 (every writer stores the same value).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite(const cx<T>* __restrict__ X, long C, long is, Geo g,
                                                   int* __restrict__ flag) {
  const cx<T>* x = X + blockIdx.y * is;
  const long stride = (long)gridDim.x * blockDim.x;
  bool bad = false;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < 3 * C; e += stride) {
    ModeK m;
    if (!mode_of(e % C, g, m)) continue;
    const cx<T> v = x[e];
    bad = bad || !isfinite(v.x) || !isfinite(v.y);
  }
  if (bad) *flag = 1;
}

template <int Unused = 0>
__global__ void k_set_int(int* __restrict__ p, int v) {
  *p = v;
}

}  // namespace hot
