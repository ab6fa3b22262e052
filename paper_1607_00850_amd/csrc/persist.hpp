// The persistent batch kernel: every pass of an RK4 call over a batch of
// uneven FP32 instances (the 2/3 rule, N up to 64) in one launch.  Host-side
// declarations; the kernel is in persist.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hot {

// sizes per launch.  The control block in the workspace holds the queue
// head, an error flag and one completion counter per size, each in a
// 256-byte line of its own (int offsets below).
constexpr int kPersistMaxGroups = 8;
constexpr int kPersistLine = 64;
constexpr int kPersistHead = 0, kPersistErr = kPersistLine, kPersistDone = 2 * kPersistLine;
constexpr int kPersistCtlInts = (2 + kPersistMaxGroups) * kPersistLine;

// One size of the batch.  The host fills N, nb, C, D1, g and the pointers;
// persist_fill the item counts and strides.
struct PersistGroup {
  int N, nb;
  int nt_c, nt_x;   // tiles per instance of the x inverse (curl) and x forward (stage update) passes
  int nv_g, nv_s;   // work items per instance of the gather and the scatter
  Pos4 st_g, st_s;  // their element strides in the digits of the loops
  long C, D1;       // compact state and x-pass slots per component
  Geo g;
  const void* in0;  // canonical input of the first member, or the table of all members' inputs
  const void* const* in_tab;
  void* out0;
  void* const* out_tab;
  void *U0, *U1, *Acc, *A1;  // the group's workspace arrays (batch-major)
};

struct PersistArgs {
  int ng, nsteps;
  float nu, dt;
  int spin;  // polls of a wait before the error flag (0: the default bound)
  int* ctl;  // the control block: queue head, error flag, items of size g completed
  PersistGroup G[kPersistMaxGroups];
};

// Device bytes of the kernel's control block and its copy of the arguments
// (in the workspace).
constexpr size_t kPersistCtlBytes = kPersistCtlInts * sizeof(int);
constexpr size_t kPersistAreaBytes = kPersistCtlBytes + (sizeof(PersistArgs) + 255) / 256 * 256;

// Whether the kernel has a body for N with geometry g (FP32, the 2/3 rule
// without row padding); if so, fill G's item counts and strides and return
// the LDS bytes its items need, else 0.
size_t persist_fill(PersistGroup& G);

// Enqueue the kernel on the kPersistAreaBytes at `area` (device memory,
// 256-byte aligned): a one-block kernel zeroes the control block and copies
// the arguments there (with ctl pointing at the control block), then the persistent kernel runs one
// block per resident slot, at most one per work item.
hipError_t persist_launch(hipStream_t s, const PersistArgs& a, void* area, size_t lds_bytes);

}  // namespace hot
