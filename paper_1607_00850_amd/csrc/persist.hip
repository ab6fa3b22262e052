// The persistent batch kernel.  One launch runs a whole RK4 call (Sec. 2's
// classical RK4 on the right-hand side of Eq. NSfinal) for a batch of
// instances of several sizes: per size the gather, then per stage the x
// inverse with the curl, the fused y-z pass and the x forward pass with the
// stage update, then the scatter -- the passes and arithmetic of the
// launch-per-pass schedule for these sizes, as device functions of one
// kernel.
//
// Work items are (pass, size, instance, tile or plane), numbered pass-level
// by pass-level (every size's items of one level before the next level's).
// A block takes the next kPersistChunk numbers from a queue head in the
// control block and runs those items in order; before an item starts, the
// block waits until every item of the same size in earlier levels has
// completed (one completion counter per size: a level-l item needs the
// counter at the number of items in levels < l).  A block adds its completed
// items to the counters before it waits and at the end of each chunk, so a
// waiting block holds none back.  An item waits only on lower numbers, which
// running blocks already hold, so the wait always ends.  A wait is still
// bounded: past the bound the kernel raises the error flag, no item waits
// any more, and every scatter item from then on writes NaN.
//
// One block shape serves every pass: 576 threads (nine waves), which every
// line length of the batch sizes divides, so that a tile of the x passes is
// 576 / Tl columns and the fused y-z pass runs nine waves of z lines.  The
// LDS is that of the largest item of the launch's sizes.
#include <hip/hip_runtime.h>

#include "impl.hpp"
#include "persist.hpp"

namespace hot {

constexpr int kPersistNT = 576;
constexpr int kPersistNW = kPersistNT / 64;
// elements per thread of a gather or scatter item
constexpr int kPersistElems = 16;
// polls of a wait before the error flag (about a second with the sleeps)
constexpr int kPersistSpin = 1 << 21;
// consecutive work items a block takes per access to the queue head
constexpr int kPersistChunk = 8;

template <int N>
struct PSize {
  static constexpr int K = (N - 1) / 3;
  using P = typename LP<N>::P;  // x inverse
  static constexpr int WC = kPersistNT / P::Tl;
  using PZ = typename LPz32<N>::P;  // z lines of the fused y-z pass
  static constexpr int KLZ = z_loads<PZ>(K + 1);
  using YS = YzShape<float, PZ, kPersistNW>;
  using PF = typename LPf<N>::P;  // x forward with the stage update
  static constexpr int WF = kPersistNT / PF::Tl;
  static constexpr int KLF = ((K + 1) + PF::Tl - 1) / PF::Tl;
  // rows of the stage update with their loads in flight together: one for
  // the plans of 12 and 16 values per thread (their three components fill
  // most of the registers a 576-thread block allows)
  static constexpr int GLF = PF::R >= 12 ? 1 : 2;
  static_assert(WC * P::Tl == kPersistNT && WF * PF::Tl == kPersistNT && YS::NT == kPersistNT,
                "every pass of the persistent kernel runs the block's threads");
  static constexpr size_t lds_x(int W) { return (size_t)(N * W + N) * sizeof(cx<float>); }
  static size_t lds(const Geo& g) {
    size_t b = lds_x(WC);
    if (lds_x(WF) > b) b = lds_x(WF);
    const size_t y = (size_t)YS::lds_bytes(g.Mz);
    return y > b ? y : b;
  }
};

// work item kinds, in level order within a stage
enum : int { IT_GATHER = 0, IT_CURL, IT_YZ, IT_XF, IT_SCATTER };

__device__ __forceinline__ long items_of(const PersistGroup& G, int kind) {
  switch (kind) {
    case IT_GATHER: return (long)G.nb * G.nv_g;
    case IT_CURL: return (long)G.nb * G.nt_c;
    case IT_YZ: return (long)G.nb * G.N;
    case IT_XF: return (long)G.nb * G.nt_x;
    default: return (long)G.nb * G.nv_s;
  }
}

// One work item of size N and kind KIND.  Not inlined: each (size, kind)
// gets its own register allocation, within the kernel's budget.
template <int N, int KIND>
__device__ __noinline__ void run_item(const PersistGroup& G, float nu, float dt, int stage, long li, int tid,
                                      cx<float>* lds, bool failed) {
  using S = PSize<N>;
  constexpr int kind = KIND;
  const long C = G.C, D1 = G.D1;
  switch (kind) {
    case IT_GATHER: {
      const long inst = li / G.nv_g, vb = li - inst * G.nv_g;
      const cx<float>* in = G.in_tab ? (const cx<float>*)G.in_tab[inst] : (const cx<float>*)G.in0;
      gather_part(in, (cx<float>*)G.U0 + inst * 3 * C, G.g, G.st_g, vb * kPersistNT + tid,
                  (long)G.nv_g * kPersistNT);
      break;
    }
    case IT_CURL: {
      const long inst = li / G.nt_c, tile = li - inst * G.nt_c;
      const cx<float>* src = (const cx<float>*)((stage & 3) == 0 ? G.U0 : G.U1);
      x_inv_curl6_tile<float, typename S::P, S::WC, true>(src, C, 3 * C, (cx<float>*)G.A1, D1, 6 * D1, (int)tile,
                                                          (int)inst, tid, G.g, float(1.0 / (double(N) * N * N)),
                                                          lds);
      break;
    }
    case IT_YZ: {
      const long inst = li / N, x = li - inst * N;
      yz_fused_plane<float, typename S::PZ, S::KLZ, true, kPersistNW>((cx<float>*)G.A1, D1, 6 * D1, G.g, x,
                                                                      (int)inst, tid, lds);
      break;
    }
    case IT_XF: {
      const long inst = li / G.nt_x, tile = li - inst * G.nt_x;
      x_fwd_rk_tile<float, typename S::PF, S::WF, S::KLF, true, S::GLF>(
          (const cx<float>*)G.A1, D1, 6 * D1, (cx<float>*)G.U0, (cx<float>*)G.U1, (cx<float>*)G.Acc, C, 3 * C, G.g,
          stage & 3, nu, dt, tile, (int)inst, tid, lds);
      break;
    }
    default: {
      const long inst = li / G.nv_s, vb = li - inst * G.nv_s;
      cx<float>* out = G.out_tab ? (cx<float>*)G.out_tab[inst] : (cx<float>*)G.out0;
      if (!failed) {
        scatter_part((const cx<float>*)G.U0 + inst * 3 * C, out, C, G.g, G.st_s, vb * kPersistNT + tid,
                     (long)G.nv_s * kPersistNT);
      } else {
        const long total = 3L * G.N * G.N * G.g.czp;
        const float nan = __builtin_nanf("");
        for (long e = vb * kPersistNT + tid; e < total; e += (long)G.nv_s * kPersistNT)
          store_stream(out + e, cx<float>{nan, nan});
      }
      break;
    }
  }
}

// The arguments in device memory (the sizes are indexed at run time, and
// the item functions take them by reference), the control block zeroed.
__global__ __launch_bounds__(256) void k_persist_setup(const PersistArgs a, PersistArgs* __restrict__ dst) {
  const int tid = threadIdx.x;
  for (int i = tid; i < kPersistCtlInts; i += 256) a.ctl[i] = 0;
  const int* src = reinterpret_cast<const int*>(&a);
  int* d = reinterpret_cast<int*>(dst);
  for (int i = tid; i < (int)(sizeof(PersistArgs) / sizeof(int)); i += 256) d[i] = src[i];
}

__global__ __launch_bounds__(kPersistNT) void k_persist_rk4(const PersistArgs* __restrict__ pa) {
  const PersistArgs& a = *pa;
  extern __shared__ unsigned char persist_smem[];
  __shared__ int s_item;
  __shared__ int s_seen[kPersistMaxGroups];  // completion counts this block has seen
  cx<float>* lds = reinterpret_cast<cx<float>*>(persist_smem);
  const int tid = threadIdx.x;
  // the queue head, the error flag and each size's completion counter sit
  // in cache lines of their own (the polls of one do not slow the others)
  int* head = a.ctl + kPersistHead;
  int* err = a.ctl + kPersistErr;
  // items per kind over all sizes
  long S[5];
  for (int k = 0; k < 5; ++k) {
    S[k] = 0;
    for (int g = 0; g < a.ng; ++g) S[k] += items_of(a.G[g], k);
  }
  const long nst = 4L * a.nsteps;  // stages of the call
  const long T3 = S[IT_CURL] + S[IT_YZ] + S[IT_XF];
  const long total = S[IT_GATHER] + nst * T3 + S[IT_SCATTER];
  // The loop has no per-lane branch: the queue and the counters are handled
  // by the whole first wave (a wave-uniform condition), only lane 0 adding,
  // and every value that steers the loop goes through readfirstlane.  With
  // a per-lane `if (tid == 0)` around the dequeue the compiler may split the
  // loop into two exec-masked levels, with lane 0's dequeue on the outer one,
  // so that the other lanes re-enter the barrier and re-read the slot before
  // lane 0 has taken the next item.
  const int spin_max = a.spin > 0 ? a.spin : kPersistSpin;
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) < 64;
  const int lane0 = tid == 0 ? 1 : 0;
  if (tid < kPersistMaxGroups) s_seen[tid] = 0;
  // wave 0: items completed by this block not yet added to the counter of
  // size pend_g.  They are added before the block waits on any counter (a
  // wait may need them) and at the end of each chunk, so a waiting block
  // holds none back.
  int pend_g = 0, pend_n = 0;
  for (;;) {
    // a chunk of consecutive items per queue access
    if (wave0) s_item = __builtin_amdgcn_readfirstlane(atomicAdd(head, lane0 * kPersistChunk));
    __syncthreads();
    const long i0 = __builtin_amdgcn_readfirstlane(s_item);
    if (i0 >= total) break;
    const long iend = i0 + kPersistChunk < total ? i0 + kPersistChunk : total;
    for (long i = i0; i < iend; ++i) {
      // level of item i: kind, stage, and the offset within the kind's items
      int kind, stage = 0;
      long off;
      if (i < S[IT_GATHER]) {
        kind = IT_GATHER;
        off = i;
      } else if (i - S[IT_GATHER] < nst * T3) {
        const long r0 = i - S[IT_GATHER];
        stage = (int)(r0 / T3);
        off = r0 - (long)stage * T3;
        kind = IT_CURL;
        if (off >= S[IT_CURL]) {
          off -= S[IT_CURL];
          kind = IT_YZ;
          if (off >= S[IT_YZ]) {
            off -= S[IT_YZ];
            kind = IT_XF;
          }
        }
      } else {
        kind = IT_SCATTER;
        off = i - S[IT_GATHER] - nst * T3;
      }
      int gi = 0;
      for (; gi < a.ng - 1; ++gi) {
        const long n = items_of(a.G[gi], kind);
        if (off < n) break;
        off -= n;
      }
      const PersistGroup& G = a.G[gi];
      int* done = a.ctl + kPersistDone + gi * kPersistLine;
      // completed items of this size that the level needs
      if (kind != IT_GATHER) {
        const long per_stage = items_of(G, IT_CURL) + items_of(G, IT_YZ) + items_of(G, IT_XF);
        long need = items_of(G, IT_GATHER);
        if (kind == IT_SCATTER) {
          need += nst * per_stage;
        } else {
          need += (long)stage * per_stage;
          if (kind >= IT_YZ) need += items_of(G, IT_CURL);
          if (kind == IT_XF) need += items_of(G, IT_YZ);
        }
        if (wave0 && __builtin_amdgcn_readfirstlane(s_seen[gi]) < need) {
          if (pend_n > 0) {
            __hip_atomic_fetch_add(a.ctl + kPersistDone + pend_g * kPersistLine, lane0 * pend_n, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            pend_n = 0;
          }
          int d = 0;
          for (int spins = 0;; ++spins) {
            d = __builtin_amdgcn_readfirstlane(__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (d >= need) break;
            if (spins >= spin_max) {
              __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            // once any wait has timed out, no other waits: the call's results
            // are lost anyway, and the kernel drains at once
            if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) !=
                0)
              break;
            __builtin_amdgcn_s_sleep(8);
          }
          s_seen[gi] = d;
          // what the completed items wrote, from any XCD
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
      }
      const bool failed =
          kind == IT_SCATTER &&
          __builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0;
#define HOT_PK(n)                                                                                   \
  case n:                                                                                           \
    switch (kind) {                                                                                 \
      case IT_GATHER: run_item<n, IT_GATHER>(G, a.nu, a.dt, stage, off, tid, lds, failed); break; \
      case IT_CURL: run_item<n, IT_CURL>(G, a.nu, a.dt, stage, off, tid, lds, failed); break;     \
      case IT_YZ: run_item<n, IT_YZ>(G, a.nu, a.dt, stage, off, tid, lds, failed); break;         \
      case IT_XF: run_item<n, IT_XF>(G, a.nu, a.dt, stage, off, tid, lds, failed); break;         \
      default: run_item<n, IT_SCATTER>(G, a.nu, a.dt, stage, off, tid, lds, failed); break;       \
    }                                                                                               \
    break;
      switch (G.N) {
        HOT_PK(16)
        HOT_PK(18)
        HOT_PK(24)
        HOT_PK(32)
        HOT_PK(36)
        HOT_PK(48)
        HOT_PK(54)
        HOT_PK(64)
        default: break;
      }
#undef HOT_PK
      // the item's stores are complete before the barrier (the barrier alone
      // does not wait for them), and wave 0's device-scope release after it
      // writes the L2's dirty lines back for every wave of the block (one
      // write-back per item: a release in each of the nine waves measured
      // 200 against 130 ms per batch step); the barrier also frees the LDS
      // for the next item
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (wave0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (pend_n > 0 && pend_g != gi) {
          __hip_atomic_fetch_add(a.ctl + kPersistDone + pend_g * kPersistLine, lane0 * pend_n, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          pend_n = 0;
        }
        pend_g = gi;
        ++pend_n;
      }
    }
    if (wave0 && pend_n > 0) {
      __hip_atomic_fetch_add(a.ctl + kPersistDone + pend_g * kPersistLine, lane0 * pend_n, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      pend_n = 0;
    }
  }
}

template <int N>
static size_t fill_n(PersistGroup& G) {
  using S = PSize<N>;
  if (!Impl<float, N>::is_g23(G.g)) return 0;
  const long Q = (long)G.g.M * G.g.Mzp;
  G.nt_c = (int)((Q + S::WC - 1) / S::WC);
  G.nt_x = (int)((Q + S::WF - 1) / S::WF);
  const long per = (long)kPersistNT * kPersistElems;
  const long ng = 3 * G.C, ns = 3L * N * N * G.g.czp;
  G.nv_g = (int)((ng + per - 1) / per);
  G.nv_s = (int)((ns + per - 1) / per);
  G.st_g = pos4_of((long)G.nv_g * kPersistNT, G.g.M, G.g.M, G.g.Mzp);
  G.st_s = pos4_of((long)G.nv_s * kPersistNT, N, N, G.g.czp);
  return S::lds(G.g);
}

size_t persist_fill(PersistGroup& G) {
  switch (G.N) {
    case 16: return fill_n<16>(G);
    case 18: return fill_n<18>(G);
    case 24: return fill_n<24>(G);
    case 32: return fill_n<32>(G);
    case 36: return fill_n<36>(G);
    case 48: return fill_n<48>(G);
    case 54: return fill_n<54>(G);
    case 64: return fill_n<64>(G);
    default: return 0;
  }
}

hipError_t persist_launch(hipStream_t s, const PersistArgs& a, void* area, size_t lds_bytes) {
  static_assert(kPersistCtlInts * sizeof(int) == kPersistCtlBytes, "control block");
  if (a.ng < 1 || a.ng > kPersistMaxGroups || a.nsteps < 0 || !area) return hipErrorInvalidValue;
  int* ctl = (int*)area;
  PersistArgs* args = (PersistArgs*)((char*)area + kPersistCtlBytes);
  hipError_t e = hipFuncSetAttribute((const void*)k_persist_rk4, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_bytes);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist_rk4, kPersistNT, lds_bytes);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  long items = 0;
  for (int g = 0; g < a.ng; ++g) {
    const PersistGroup& G = a.G[g];
    items += (long)G.nb * (G.nv_g + G.nv_s + 4L * a.nsteps * (G.nt_c + G.N + G.nt_x));
  }
  long grid = (long)cus * per_cu;
  if (grid > items) grid = items;
  if (grid < 1) grid = 1;
  PersistArgs b = a;
  b.ctl = ctl;
  hipLaunchKernelGGL(k_persist_setup, dim3(1), dim3(256), 0, s, b, args);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_persist_rk4, dim3((unsigned)grid), dim3(kPersistNT), lds_bytes, s, (const PersistArgs*)args);
  return hipGetLastError();
}

}  // namespace hot
