// Warm-start launcher of the MLP surrogate, shared by the implicit step
// (hot.hip) and its definition (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hot {

// For every instance of a group (compact [B][3][C] buffers of element type
// T): d = 2 H1 - H2 + s MLP(features), U1 = U0 + d/2, act[b] = 1.
template <typename T>
hipError_t mlp_predict(hipStream_t s, const void* packed, const void* U0, const void* H1, const void* H2, void* D,
                       void* U1, int* act, long C, long is, int nb, const Geo& g, double nu, double dt);

}  // namespace hot
