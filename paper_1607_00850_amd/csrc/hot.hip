// libhot host side: plan validation, workspace layout, pass schedule and the
// C ABI of include/hot.h.  All arithmetic runs in the kernels of kernels.hpp
// (and, for the surrogate warm start, mlp.hpp).
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/hot.h"
#include "checks.hpp"
#include "impl.hpp"
#include "mlp_launch.hpp"
#include "persist.hpp"

namespace hot {

enum Pass : int {
  PASS_GATHER = 0,
  PASS_X_INV_CURL,
  PASS_Y_INV,
  PASS_Z_CROSS,
  PASS_Y_FWD,
  PASS_X_FWD,
  PASS_RK_STAGE,
  PASS_SCATTER,
  PASS_Z_R2C,
  PASS_Z_C2R,
  PASS_X_INV,
  PASS_IMP_PREDICT,
  PASS_IMP_UPDATE,
  PASS_IMP_DECIDE,
  PASS_IMP_ADVANCE,
  PASS_X_FWD_RK,
  PASS_YZ_FUSED,
  PASS_TABLES,
  PASS_STATS,
  PASS_GRAPH,  // no kernel: the batch schedule (hot_set_variant)
  PASS_PERSIST,  // the persistent batch kernel (every pass of an RK4 call)
  NUM_PASSES
};

static const char* kPassNames[NUM_PASSES] = {
    "gather", "x_inv_curl", "y_inv", "z_cross", "y_fwd", "x_fwd", "rk_stage", "scatter", "z_r2c", "z_c2r", "x_inv",
    "imp_predict", "imp_update", "imp_decide", "imp_advance", "x_fwd_rk", "yz_fused", "tables", "stats", "graph",
    "persistent",
};

template <typename T>
static bool ops_for(int N, Ops* o) {
  const bool f = std::is_same<T, float>::value;
  switch (N) {
#define HOT_CASE(n)                                    \
  case n:                                              \
    *o = f ? make_ops_f32_##n() : make_ops_f64_##n(); \
    return true;
    HOT_SIZES(HOT_CASE)
#undef HOT_CASE
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
// mode: 0 = 2/3 rule, 1 = all but Nyquist, 2 = every mode (plain transforms).
// elem: bytes per complex value; the z pitch is padded to whole 128-byte rows
// once rows are long enough for the padding to be cheap.
// Column tile of the compact state arrays (cbase in kernels.hpp): 64 bytes of
// a row where the z pitch is a multiple of it and holds whole 128-byte rows,
// else one tile of all M*Mzp columns (row-major).
static int state_tile(const Geo& g, int elem) {
  const int tw = 64 / elem, seg = 128 / elem;
  return (g.Mzp % seg == 0 && g.Mzp >= 4 * seg) ? tw : g.M * g.Mzp;
}

static Geo make_geo(int N, int mode, int elem) {
  Geo g{};
  g.N = N;
  if (mode == 0) {  // 2/3 rule: |k| <= K = floor((N-1)/3)
    const int K = (N - 1) / 3;
    g.lo = K + 1;
    g.hi = K;
    g.Mz = K + 1;
  } else if (mode == 1) {  // all but Nyquist
    g.lo = N / 2;
    g.hi = N / 2 - 1;
    g.Mz = N / 2;
  } else {  // every mode (plain transforms)
    g.lo = N / 2 + 1;
    g.hi = N / 2 - 1;
    g.Mz = N / 2 + 1;
  }
  g.M = g.lo + g.hi;
  const int seg = 128 / elem;
  g.Mzp = (mode != 2 && g.Mz >= 4 * seg) ? (g.Mz + seg - 1) / seg * seg : g.Mz;
  g.kz0 = 0;
  g.czp = N / 2 + 1;
  g.tw = state_tile(g, elem);
  return g;
}

static const size_t kAlign = 256;
static const int kStatParts = 64;  // blocks of partial sums per instance (hot_stats)
static inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// All instances of one N.  For the right-hand side, RK4 and the implicit step
// their workspace is one region laid out batch-major: U0, U1, Acc, Nh =
// [B][3][C] each, A1 = [B][6][D1], A2 = [B][6][D2], then for B > 1 the device
// tables of the members' input and output pointers.  The implicit step adds
// two increment histories H1, H2 = [B][3][C] (its iterate d lives in Acc),
// the stopping flags act[B], the partial sums part[B][nparts][2] and the
// per-instance counters cnt[2][B] (sweeps, steps stopped at max_iter).  Every
// such group also keeps the partial sums of its statistics diag[B][64][2]
// (hot_stats).  Plain
// transforms run one instance at a time in a shared region.
struct Group {
  int N = 0;
  Geo g{};
  Ops ops{};
  std::vector<int> members;  // instance indices in descriptor order
  long C = 0, D1 = 0, D2 = 0;       // slots per component (row pitch Mzp)
  double lC = 0, lD1 = 0, lD2 = 0;  // live values per component (Mz)
  size_t off = 0;                   // byte offset of the group's region
  size_t oU0 = 0, oU1 = 0, oAcc = 0, oNh = 0, oA1 = 0, oA2 = 0, oTab = 0;
  size_t oH[4] = {0, 0, 0, 0}, oAct = 0, oPart = 0, oCnt = 0;  // implicit step only
  size_t oDiag = 0;                                      // statistics partial sums
  size_t oZ = 0;                              // z-slab share: receive buffer of the all-to-all
  int nparts = 0;                             // blocks of the implicit update
  int rot = 0, hist = 0;                      // implicit step: buffer rotation, history depth
  int fused = -1;  // RK4/RHS: x_fwd_rk variant fusing the x pass with the stage update, -1 = separate passes
  int yz = -1;     // 0: the y and z passes fused (k_yz_fused), -1: y_inv, z_cross, y_fwd
  // row form of the y and z passes: 0 six component rows (the z pass completes
  // the Hermitian halves in LDS); 1 packed pairs in and out (default); 2 packed
  // pairs in, c0 c1 c2 component rows out; 3 component rows in and out, the z
  // pass packing its lines on load
  int zpack = 0;
  bool packed_y_inv() const { return zpack == 1 || zpack == 2; }
  size_t bytes = 0;
  int variant[NUM_PASSES];  // strided column-width variant per pass (autotuned)
  int B() const { return (int)members.size(); }
};

}  // namespace hot

using namespace hot;

struct hot_plan_s {
  int op, dtype, dealias;
  double nu, dt;
  double tol;    // implicit step: stopping tolerance
  int max_iter;  // implicit step: sweeps per step at most
  std::vector<int> imp_sweeps, imp_nonconv;  // implicit step: last call, per instance
  int flags = 0;
  // z-slab share (hot_plan_slab): nranks > 1 splits kz over the shares in
  // chunks of `chunk` retained values and x over them in nx planes each
  bool slab = false;
  int nranks = 1, rank = 0, chunk = 0, nx = 0;
  Geo gz{};  // geometry of the exchanged z lines (all retained kz, pitch of the blocks)
  size_t o_finite = 0;              // HOT_FLAG_CHECK_FINITE: byte offset of the flag in the workspace
  size_t o_persist = 0;             // FP32 RK4 with the 2/3 rule: the persistent kernel's control block
  const void* surrogate = nullptr;  // packed MLP for the implicit warm start
  void* hist_ws = nullptr;          // workspace holding the kept history
  void* cnt_ws = nullptr;           // implicit step: workspace and stream of the last call (its counters)
  hipStream_t cnt_stream = nullptr;
  size_t elem;  // bytes per complex element
  int batch;
  std::vector<int> n;
  std::vector<Group> groups;
  size_t ws_bytes;
  int last_hip;
  // profiling
  bool prof;
  struct Rec {
    int pass;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  // graph capture of several sizes: one side stream per group (a branch of the
  // graph each) and the events of the fork and the join
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_ev;
  bool graph_branches = true;  // hot_set_variant(graph): 1 branch per group, 0 one chain
  bool persistent = false;     // hot_set_variant(graph) 2: the persistent kernel (RK4)
  int persist_spin = 0;        // hot_set_variant(persistent): polls of a wait before its error path (0: default)
  int imp_check = 2;           // implicit step: sweeps between the host's looks at the flags (0: never)
  std::vector<int> act_host;   // implicit step: the flags read back, per instance
};

struct hot_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* hot_error_string(int code) {
  switch (code) {
    case HOT_OK: return "ok";
    case HOT_E_INVALID: return "invalid argument";
    case HOT_E_UNSUPPORTED: return "unsupported request";
    case HOT_E_WORKSPACE: return "workspace missing or misaligned";
    case HOT_E_HIP: return "HIP error";
    case HOT_E_NOCONVERGE: return "implicit step stopped at max_iter sweeps";
    case HOT_E_NONFINITE: return "result holds a NaN or an infinity";
    case HOT_E_TOOBIG: return "plan needs more than the library's static scratch (hot_run_noalloc)";
    default: return "unknown error";
  }
}

// Workspace layout of every group (offsets and sizes from the groups'
// geometry); sets p->ws_bytes.
static int layout_groups(hot_plan_s* p, int op) {
  const bool plain = op == HOT_OP_R2C || op == HOT_OP_C2R;
  p->ws_bytes = 0;
  size_t off = 0;
  for (auto& G : p->groups) {
    if (G.B() > 65535) return HOT_E_UNSUPPORTED;  // one grid dimension per batch
    const long N = G.N;
    G.C = (long)G.g.M * G.g.M * G.g.Mzp;
    G.D1 = N * G.g.M * G.g.Mzp;
    G.D2 = N * N * G.g.Mzp;
    G.lC = (double)G.g.M * G.g.M * G.g.Mz;
    G.lD1 = (double)N * G.g.M * G.g.Mz;
    G.lD2 = (double)N * N * G.g.Mz;
    const size_t e = p->elem, B = (size_t)G.B();
    if (plain) {
      G.bytes = 2 * align_up(3 * (size_t)G.D2 * e);  // shared by all instances, one at a time
      if (G.bytes > p->ws_bytes) p->ws_bytes = G.bytes;
      continue;
    }
    const size_t sC = align_up(B * 3 * (size_t)G.C * e);
    G.off = off;
    G.oU0 = 0;
    G.oU1 = sC;
    G.oAcc = 2 * sC;
    G.oNh = 3 * sC;
    G.oA1 = 4 * sC;
    G.oA2 = G.oA1 + align_up(B * 6 * (size_t)G.D1 * e);
    G.oTab = G.oA2 + align_up(B * 6 * (size_t)G.D2 * e);
    // for B > 1: the in and out pointer tables and the members' instance indices
    G.oDiag = G.oTab + (B > 1 ? align_up(3 * B * sizeof(void*)) : 0);
    G.bytes = G.oDiag + align_up(B * (size_t)kStatParts * 2 * sizeof(double));
    if (p->slab) {
      G.oZ = G.bytes;
      G.bytes += align_up(B * 6 * (size_t)G.D2 * e);
    }
    if (op == HOT_OP_IMPLICIT) {
      G.nparts = (int)grid_1d(G.C, 256);
      G.oH[0] = G.bytes;
      G.oH[1] = G.oH[0] + sC;
      G.oH[2] = G.oH[1] + sC;
      G.oH[3] = G.oH[2] + sC;
      G.oAct = G.oH[3] + sC;
      G.oPart = G.oAct + align_up(B * sizeof(int));
      G.oCnt = G.oPart + align_up(B * (size_t)G.nparts * 2 * sizeof(double));
      G.bytes = G.oCnt + align_up(2 * B * sizeof(int));
    }
    off += G.bytes;
  }
  if (!plain) p->ws_bytes = off;
  if (p->flags & HOT_FLAG_CHECK_FINITE) {
    p->o_finite = p->ws_bytes;
    p->ws_bytes += kAlign;
  }
  if (op == HOT_OP_RK4 && p->elem == 8 && p->dealias == HOT_DEALIAS_TWO_THIRDS && !p->slab) {
    p->o_persist = p->ws_bytes;
    p->ws_bytes += align_up(kPersistAreaBytes);
  }
  return HOT_OK;
}

int hot_plan(const hot_desc* d, hot_plan_t* out, size_t* workspace_bytes) {
  if (out) *out = nullptr;
  if (!d || !out || !workspace_bytes) return HOT_E_INVALID;
  if (d->abi_version != HOT_ABI_VERSION) return HOT_E_INVALID;
  if (d->batch < 1 || !d->n) return HOT_E_INVALID;
  if (d->dtype != HOT_F64 && d->dtype != HOT_F32) return HOT_E_INVALID;
  if (d->op < HOT_OP_R2C || d->op > HOT_OP_IMPLICIT) return HOT_E_INVALID;
  if (d->dealias != HOT_DEALIAS_TWO_THIRDS && d->dealias != HOT_DEALIAS_NONE) return HOT_E_INVALID;
  if (d->reserved != 0) return HOT_E_INVALID;
  if (d->flags & ~(HOT_FLAG_KEEP_HISTORY | HOT_FLAG_CHECK_FINITE)) return HOT_E_INVALID;
  if ((d->flags & HOT_FLAG_KEEP_HISTORY) && d->op != HOT_OP_IMPLICIT) return HOT_E_INVALID;
  if ((d->flags & HOT_FLAG_CHECK_FINITE) && (d->op == HOT_OP_R2C || d->op == HOT_OP_C2R)) return HOT_E_INVALID;
  if (!(d->nu >= 0.0)) return HOT_E_INVALID;  // also rejects NaN
  if ((d->op == HOT_OP_RK4 || d->op == HOT_OP_IMPLICIT) && !(d->dt > 0.0)) return HOT_E_INVALID;
  if (d->op == HOT_OP_IMPLICIT && (!(d->tol > 0.0) || d->max_iter < 1)) return HOT_E_INVALID;
  for (int i = 0; i < d->batch; ++i) {
    const int N = d->n[i];
    if (N < 8 || (N & 1)) return HOT_E_INVALID;
  }
  hot_plan_s* p = new (std::nothrow) hot_plan_s();
  if (!p) return HOT_E_INVALID;
  p->op = d->op;
  p->dtype = d->dtype;
  p->dealias = d->dealias;
  p->nu = d->nu;
  p->dt = d->dt;
  p->tol = d->tol;
  p->max_iter = d->max_iter;
  p->flags = d->flags;
  p->elem = d->dtype == HOT_F64 ? 16 : 8;
  p->batch = d->batch;
  p->n.assign(d->n, d->n + d->batch);
  p->act_host.assign(d->batch, 0);
  p->last_hip = 0;
  p->prof = false;
  p->ws_bytes = 0;
  const bool plain = d->op == HOT_OP_R2C || d->op == HOT_OP_C2R;
  // group the instances by N, in order of first appearance
  for (int i = 0; i < d->batch; ++i) {
    const int N = d->n[i];
    Group* gp = nullptr;
    for (auto& G : p->groups)
      if (G.N == N) gp = &G;
    if (!gp) {
      Group G;
      G.N = N;
      const bool ok = d->dtype == HOT_F64 ? ops_for<double>(N, &G.ops) : ops_for<float>(N, &G.ops);
      if (!ok) {
        delete p;
        return HOT_E_UNSUPPORTED;
      }
      G.g = make_geo(N, plain ? 2 : d->dealias, (int)p->elem);
      G.zpack = plain ? 0 : 1;
      for (int k = 0; k < NUM_PASSES; ++k) G.variant[k] = 1;
      p->groups.push_back(G);
      gp = &p->groups.back();
    }
    gp->members.push_back(i);
  }
  if (layout_groups(p, d->op) != HOT_OK) {
    delete p;
    return HOT_E_UNSUPPORTED;
  }
  *out = p;
  *workspace_bytes = p->ws_bytes;
  return HOT_OK;
}

int hot_destroy(hot_plan_t p) {
  if (!p) return HOT_OK;
  for (auto& r : p->recs) {
    (void)hipEventSynchronize(r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : p->pool) (void)hipEventDestroy(e);
  for (auto e : p->side_ev) (void)hipEventDestroy(e);
  for (auto st : p->side) (void)hipStreamDestroy(st);
  delete p;
  return HOT_OK;
}

int hot_last_hip_error(hot_plan_t p) { return p ? p->last_hip : 0; }

int hot_profile_enable(hot_plan_t p, int enable) {
  if (!p) return HOT_E_INVALID;
  p->prof = enable != 0;
  return HOT_OK;
}

int hot_profile_read(hot_plan_t p, int32_t max_passes, double* ms, int64_t* launches) {
  if (!p || max_passes < 0 || (max_passes > 0 && (!ms || !launches))) return HOT_E_INVALID;
  for (int i = 0; i < max_passes; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  int rc = HOT_OK;
  for (auto& r : p->recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) {
      p->last_hip = (int)e;
      rc = HOT_E_HIP;
    } else if (r.pass < max_passes) {
      ms[r.pass] += t;
      launches[r.pass] += 1;
    }
    p->pool.push_back(r.a);
    p->pool.push_back(r.b);
  }
  p->recs.clear();
  return rc == HOT_OK ? (int)NUM_PASSES : rc;
}

const char* hot_pass_name(int32_t pass) {
  return (pass >= 0 && pass < NUM_PASSES) ? kPassNames[pass] : "";
}

int hot_pass_bytes(hot_plan_t p, int32_t instance, int32_t pass, double* bytes) {
  if (!p || !bytes || instance < 0 || instance >= p->batch) return HOT_E_INVALID;
  const Group* Gp = nullptr;
  for (const auto& G : p->groups)
    if (G.N == p->n[instance]) Gp = &G;
  const Group& I = *Gp;
  const double e = (double)p->elem, C = I.lC, D1 = I.lD1, D2 = I.lD2;
  const double N = I.g.N, canon = 3.0 * N * N * I.g.czp;
  double b = 0;
  const bool plain = p->op == HOT_OP_R2C || p->op == HOT_OP_C2R;
  switch (pass) {
    case PASS_GATHER: b = plain ? 0 : 6 * C; break;  // read the 3C retained values, write 3C
    case PASS_X_INV_CURL: b = plain ? 0 : 3 * C + 6 * D1; break;
    case PASS_Y_INV: b = plain ? (p->op == HOT_OP_C2R ? 6 * D2 : 0) : 6 * D1 + 6 * D2; break;
    // a slab share transforms nx x-planes of lines with every retained kz
    case PASS_Z_CROSS: b = plain ? 0 : (p->slab ? 9.0 * p->nx * N * p->gz.Mz : 6 * D2 + 3 * D2); break;
    case PASS_Y_FWD: b = plain ? (p->op == HOT_OP_R2C ? 6 * D2 : 0) : 3 * D2 + 3 * D1; break;
    case PASS_X_FWD: b = plain ? (p->op == HOT_OP_R2C ? 6 * D2 : 0) : 3 * D1 + 3 * C; break;
    // RK4 stages move 12C, 18C, 18C, 12C (mean 15C); the plain RHS 9C
    case PASS_RK_STAGE: b = (p->op == HOT_OP_RHS ? 9 * C : (p->op == HOT_OP_RK4 ? 15 * C : 0)); break;
    case PASS_SCATTER: b = plain ? 0 : 3 * C + canon; break;
    case PASS_Z_R2C: b = p->op == HOT_OP_R2C ? 3 * D2 + 3 * N * N * N / 2 : 0; break;  // reals count half
    case PASS_Z_C2R: b = p->op == HOT_OP_C2R ? 3 * D2 + 3 * N * N * N / 2 : 0; break;
    case PASS_X_INV: b = p->op == HOT_OP_C2R ? 6 * D2 : 0; break;
    // implicit step: the predictor at its widest (reads U0, H1, H2; writes d, U1),
    // the update (reads Nh, U0, d; writes d, U1), the advance (U0 += d)
    case PASS_IMP_PREDICT: b = p->op == HOT_OP_IMPLICIT ? 15 * C : 0; break;
    case PASS_IMP_UPDATE: b = p->op == HOT_OP_IMPLICIT ? 15 * C : 0; break;
    case PASS_IMP_DECIDE: b = 0; break;
    case PASS_IMP_ADVANCE: b = p->op == HOT_OP_IMPLICIT ? 9 * C : 0; break;
    // the x pass fused with the stage update: the stage traffic without the
    // nonlinear term (which stays in registers)
    case PASS_X_FWD_RK: b = p->op == HOT_OP_RK4 ? 3 * D1 + 12 * C : (p->op == HOT_OP_RHS ? 3 * D1 + 6 * C : 0); break;
    // the y and z passes in one: six components of A1 in, three out
    case PASS_YZ_FUSED: b = plain ? 0 : 6 * D1 + 3 * D1; break;
    case PASS_TABLES: b = 0; break;  // a few pointers per instance
    case PASS_STATS: b = plain ? 0 : 3 * C; break;  // reads the compact state once
    case PASS_GRAPH: b = 0; break;
    // the persistent kernel over a one-step RK4 call: the gather, four stages
    // of the x inverse, the fused y-z pass and the fused x forward, the scatter
    case PASS_PERSIST:
      b = p->op == HOT_OP_RK4 ? 6 * C + 4 * ((3 * C + 6 * D1) + 9 * D1 + (3 * D1 + 12 * C)) + 3 * C + canon : 0;
      break;
    default: return HOT_E_INVALID;
  }
  *bytes = b * e;
  return HOT_OK;
}

}  // extern "C"

namespace {

static_assert(sizeof(StatsRec) == sizeof(hot_stats) && offsetof(StatsRec, sweeps) == offsetof(hot_stats, sweeps) &&
                  offsetof(StatsRec, nonconv) == offsetof(hot_stats, nonconv),
              "device statistics record must match hot_stats");

struct Runner {
  hot_plan_s* p;
  hipStream_t s;
  bool record = true;  // profiling events (off while a graph is captured)
  int rc = HOT_OK;

  hipEvent_t ev() {
    if (!p->pool.empty()) {
      hipEvent_t e = p->pool.back();
      p->pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }

  template <class F>
  void pass(int id, F&& launch) {
    if (rc != HOT_OK) return;
    hipEvent_t a = nullptr, b = nullptr;
    const bool prof = p->prof && record;
    if (prof) {
      a = ev();
      b = ev();
      if (a && b) (void)hipEventRecord(a, s);
    }
    hipError_t e = launch();
    if (prof && a && b) {
      (void)hipEventRecord(b, s);
      p->recs.push_back({id, a, b});
    }
    if (e != hipSuccess) {
      p->last_hip = (int)e;
      rc = HOT_E_HIP;
    }
  }
};

struct GroupPtrs {
  char *U0, *U1, *Acc, *Nh, *A1, *A2, *Z;
  char* H[4];  // implicit step: increment histories
  int* act;
  double* part;
  int* cnt;  // implicit step: sweeps[B], then nonconv[B]
  double* diag;
  const void* const* in_tab;
  void* const* out_tab;
  const long* idx_tab;  // instance index of each member (B > 1)
};

GroupPtrs group_ptrs(const Group& G, void* workspace) {
  char* base = (char*)workspace + G.off;
  GroupPtrs q;
  q.U0 = base + G.oU0;
  q.U1 = base + G.oU1;
  q.Acc = base + G.oAcc;
  q.Nh = base + G.oNh;
  q.A1 = base + G.oA1;
  q.A2 = base + G.oA2;
  q.Z = base + G.oZ;
  q.H[0] = base + G.oH[0];
  q.H[1] = base + G.oH[1];
  q.H[2] = base + G.oH[2];
  q.H[3] = base + G.oH[3];
  q.act = (int*)(base + G.oAct);
  q.part = (double*)(base + G.oPart);
  q.cnt = (int*)(base + G.oCnt);
  q.diag = (double*)(base + G.oDiag);
  q.in_tab = G.B() > 1 ? (const void* const*)(base + G.oTab) : nullptr;
  q.out_tab = G.B() > 1 ? (void* const*)(base + G.oTab + G.B() * sizeof(void*)) : nullptr;
  q.idx_tab = G.B() > 1 ? (const long*)(base + G.oTab + 2 * G.B() * sizeof(void*)) : nullptr;
  return q;
}

// The y inverse pass of a group (A1 -> A2), the z pass (in place on A2) and
// the y forward pass (A2 -> A1): on packed pair rows where the group uses them.
void y_inv_pass(Runner& r, const Group& G, const GroupPtrs& q, const int* act) {
  const long N = G.N, M = G.g.M, P = G.g.Mzp;
  r.pass(PASS_Y_INV, [&] {
    if (G.packed_y_inv())
      return G.ops.y_inv_pack(r.s, G.variant[PASS_Y_INV], q.A1, q.A2, N * P, P, P, P, M * P, N * P, G.D1, G.D2,
                              6 * G.D1, 6 * G.D2, G.B(), G.g, act);
    return G.ops.strided(r.s, G.variant[PASS_Y_INV], +1, true, false, q.A1, q.A2, N * P, P, P, P, M * P, N * P, G.D1,
                         G.D2, 6, 6 * G.D1, 6 * G.D2, 0, G.B(), G.g, act);
  });
}

void z_pass(Runner& r, const Group& G, const GroupPtrs& q, const int* act) {
  r.pass(PASS_Z_CROSS, [&] {
    return G.zpack > 0
               ? G.ops.z_cross_packed(r.s, q.A2, G.D2, 6 * G.D2, G.N * (long)G.N, G.B(), G.g, act, G.zpack - 1)
               : G.ops.z_cross(r.s, q.A2, G.D2, 6 * G.D2, G.N * (long)G.N, G.B(), G.g, act);
  });
}

void y_fwd_pass(Runner& r, const Group& G, const GroupPtrs& q, const int* act) {
  const long N = G.N, M = G.g.M, P = G.g.Mzp;
  r.pass(PASS_Y_FWD, [&] {
    if (G.zpack == 1)
      return G.ops.y_fwd_unpack(r.s, G.variant[PASS_Y_FWD], q.A2, q.A1, N * P, P, P, P, N * P, M * P, G.D2, G.D1,
                                6 * G.D2, 6 * G.D1, G.B(), G.g, act);
    return G.ops.strided(r.s, G.variant[PASS_Y_FWD] % 3, -1, false, true, q.A2, q.A1, N * P, P, P, P, N * P, M * P, G.D2,
                         G.D1, 3, 6 * G.D2, 6 * G.D1, 0, G.B(), G.g, act);
  });
}

// The inverse half of a right-hand side for every instance of a group: the x
// pass (curl fused) from compact state `src`, then the y pass, into A2.
void inverse_passes(Runner& r, const Group& G, const GroupPtrs& q, const char* src, const int* act) {
  const Geo& g = G.g;
  const long N = g.N, M = g.M, P = g.Mzp;
  const Ops& o = G.ops;
  const int nb = G.B();
  const long isU = 3 * G.C, isA1 = 6 * G.D1, isA2 = 6 * G.D2;
  r.pass(PASS_X_INV_CURL, [&] {
    return o.x_inv_curl(r.s, G.variant[PASS_X_INV_CURL], src, G.C, isU, q.A1, G.D1, isA1, nb, g, act);
  });
  // y inverse: 6 components, batch over x, rows ky (compact) -> y (all N)
  y_inv_pass(r, G, q, act);
}

// The forward half after the z pass: the y pass from A2, then (x_fwd) the x
// pass into Nh.
void forward_passes(Runner& r, const Group& G, const GroupPtrs& q, const int* act, bool x_fwd) {
  const Geo& g = G.g;
  const long N = g.N, M = g.M, P = g.Mzp;
  const Ops& o = G.ops;
  const int nb = G.B();
  const long isU = 3 * G.C, isA1 = 6 * G.D1, isA2 = 6 * G.D2;
  // y forward: 3 components, y (all N) -> ky (compact)
  y_fwd_pass(r, G, q, act);
  // x forward: rows x (all N) -> kx (compact), columns (ky, kz)
  if (!x_fwd) return;
  r.pass(PASS_X_FWD, [&] {
    const long Q = M * P;
    return o.strided(r.s, G.variant[PASS_X_FWD], -1, false, true, q.A1, q.Nh, Q, Q, Q, g.tw, 0, 0, G.D1, G.C, 3,
                     isA1, isU, g.tw, nb, g, act);
  });
}

// One evaluation of the right-hand side for every instance of a group, from
// compact state `src` into Nh.
void rhs_passes(Runner& r, const Group& G, const GroupPtrs& q, const char* src, const int* act = nullptr,
                bool x_fwd = true) {
  if (G.yz < 0) {
    inverse_passes(r, G, q, src, act);
    z_pass(r, G, q, act);
    forward_passes(r, G, q, act, x_fwd);
    return;
  }
  // small N: x inverse, then the y and z passes in one kernel on A1, then x forward
  const int nb = G.B();
  r.pass(PASS_X_INV_CURL, [&] {
    return G.ops.x_inv_curl(r.s, G.variant[PASS_X_INV_CURL], src, G.C, 3 * G.C, q.A1, G.D1, 6 * G.D1, nb, G.g, act);
  });
  r.pass(PASS_YZ_FUSED, [&] { return G.ops.yz_fused(r.s, q.A1, G.D1, 6 * G.D1, nb, G.g, act); });
  if (!x_fwd) return;
  r.pass(PASS_X_FWD, [&] {
    const long Q = (long)G.g.M * G.g.Mzp;
    return G.ops.strided(r.s, G.variant[PASS_X_FWD], -1, false, true, q.A1, q.Nh, Q, Q, Q, G.g.tw, 0, 0, G.D1, G.C,
                         3, 6 * G.D1, 3 * G.C, G.g.tw, nb, G.g, act);
  });
}

// The stage update after the forward y pass (mode 0..3 RK4 stage, 4 plain
// right-hand side into Acc): the x pass and the update fused or separate.
void stage_update(Runner& r, const Group& G, const GroupPtrs& q, int mode, double nu, double dt) {
  const Ops& o = G.ops;
  const long isU = 3 * G.C;
  const int nb = G.B();
  if (G.fused < 0)
    r.pass(PASS_RK_STAGE, [&] { return o.rk_stage(r.s, q.Nh, q.U0, q.U1, q.Acc, G.C, isU, nb, G.g, mode, nu, dt); });
  else
    r.pass(PASS_X_FWD_RK, [&] {
      return o.x_fwd_rk(r.s, G.fused, q.A1, G.D1, 6 * G.D1, q.U0, q.U1, q.Acc, G.C, isU, nb, G.g, mode, nu, dt);
    });
}

// One right-hand side plus stage update.
void stage_passes(Runner& r, const Group& G, const GroupPtrs& q, const char* src, int mode, double nu, double dt) {
  rhs_passes(r, G, q, src, nullptr, G.fused < 0);
  stage_update(r, G, q, mode, nu, dt);
}

// Write a batched group's tables of its members' canonical input and output
// pointers into the workspace, in stream order (k_write_tab).  Every call
// writes them, so no earlier call, graph or plan sharing the workspace can
// leave stale pointers behind.
void write_tables(Runner& r, const Group& G, const GroupPtrs& q, void* const* in, void* const* out) {
  const int nb = G.B();
  if (nb < 2) return;
  // the in pointers, out pointers and instance indices (as pointer-sized
  // integers) lie nb entries apart from in_tab on
  static_assert(sizeof(TabChunk) + 2 * sizeof(void*) + sizeof(int) <= 4096, "kernel argument size");
  const void** tab = (const void**)q.in_tab;
  for (int m0 = 0; m0 < nb && r.rc == HOT_OK; m0 += kTabChunk) {
    TabChunk c{};
    const int n = nb - m0 < kTabChunk ? nb - m0 : kTabChunk;
    for (int m = 0; m < n; ++m) {
      const int i = G.members[m0 + m];
      c.in[m] = in[i];
      c.out[m] = out[i];
      c.idx[m] = (const void*)(intptr_t)i;
    }
    r.pass(PASS_TABLES, [&] {
      hipLaunchKernelGGL(k_write_tab<>, dim3(1), dim3(256), 0, r.s, tab + m0, (long)nb, c, n);
      return hipGetLastError();
    });
  }
}

// hot_stats of every instance of a group from its compact state X (and, for
// the implicit step, its counters), written to stats[instance].
void state_stats(Runner& r, const hot_plan_s* p, const Group& G, const GroupPtrs& q, const char* X, StatsRec* stats,
                 bool counters) {
  const int nb = G.B();
  r.pass(PASS_STATS, [&] {
    const dim3 grid((unsigned)kStatParts, (unsigned)nb);
    if (p->dtype == HOT_F64)
      hipLaunchKernelGGL(k_state_sums<double>, grid, dim3(256), 0, r.s, (const cx<double>*)X, G.C, 3 * G.C, G.g,
                         q.diag);
    else
      hipLaunchKernelGGL(k_state_sums<float>, grid, dim3(256), 0, r.s, (const cx<float>*)X, G.C, 3 * G.C, G.g,
                         q.diag);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_state_final<>, dim3(nb), dim3(64), 0, r.s, (const double*)q.diag, kStatParts, G.N, p->nu,
                       q.idx_tab, (long)G.members[0], counters ? (const int*)q.cnt : nullptr,
                       counters ? (const int*)q.cnt + nb : nullptr, stats);
    return hipGetLastError();
  });
}

// Branches: when `fork` is set and the plan has several groups, every group
// runs on its own side stream, forked from and joined back into the calling
// stream with events.  Under graph capture this gives one branch per size, so
// the passes of small sizes run beside those of large ones.
hipError_t fork_groups(hot_plan_s* p, hipStream_t s) {
  const size_t ng = p->groups.size();
  hipError_t e = hipSuccess;
  while (e == hipSuccess && p->side.size() < ng) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);  // default priority
    if (e == hipSuccess) p->side.push_back(st);
  }
  while (e == hipSuccess && p->side_ev.size() < ng + 1) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) p->side_ev.push_back(ev);
  }
  if (e == hipSuccess) e = hipEventRecord(p->side_ev[ng], s);
  for (size_t g = 0; g < ng && e == hipSuccess; ++g) e = hipStreamWaitEvent(p->side[g], p->side_ev[ng], 0);
  return e;
}

hipError_t join_groups(hot_plan_s* p, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (size_t g = 0; g < p->groups.size() && e == hipSuccess; ++g) {
    e = hipEventRecord(p->side_ev[g], p->side[g]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->side_ev[g], 0);
  }
  return e;
}

// The order in which the branches are enqueued: sorted by work (N^3 times the
// instances), the smaller half from the smallest up, then the larger half from
// the largest down.  On the batch of 4096 uneven instances (N 16-64) the
// replay took 19.65 ms in this order, 20.0 ms in order of first appearance,
// 19.8 ms smallest first and 20.4 ms largest first.
std::vector<size_t> branch_order(const hot_plan_s* p) {
  std::vector<size_t> o(p->groups.size());
  for (size_t i = 0; i < o.size(); ++i) o[i] = i;
  const auto work = [p](size_t i) {
    const double N = p->groups[i].N;
    return N * N * N * (double)p->groups[i].members.size();
  };
  std::stable_sort(o.begin(), o.end(), [&](size_t a, size_t b) { return work(a) < work(b); });
  const size_t h = o.size() / 2;
  std::reverse(o.begin() + h, o.end());
  return o;
}

int check_run_args(hot_plan_s* p, void* const* in, void* const* out, void* workspace, int32_t nsteps,
                   const void* stats) {
  if (!p || !in || !out || nsteps < 0) return HOT_E_INVALID;
  if (stats && (p->op == HOT_OP_R2C || p->op == HOT_OP_C2R || ((uintptr_t)stats % 8) != 0)) return HOT_E_INVALID;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return HOT_E_WORKSPACE;
  for (int i = 0; i < p->batch; ++i) {
    if (!in[i] || !out[i]) return HOT_E_INVALID;
    if (((uintptr_t)in[i] % kAlign) != 0 || ((uintptr_t)out[i] % kAlign) != 0) return HOT_E_INVALID;
  }
  return HOT_OK;
}

// Whether the persistent kernel has every size of the plan: FP32 RK4 with
// the 2/3 rule, at most kPersistMaxGroups sizes, each a batch size of the
// fused y-z pass in its compile-time geometry.
bool persist_ok(const hot_plan_s* p) {
  if (p->op != HOT_OP_RK4 || p->elem != 8 || p->dealias != HOT_DEALIAS_TWO_THIRDS || p->slab) return false;
  if (p->groups.empty() || p->groups.size() > (size_t)kPersistMaxGroups) return false;
  for (const auto& G : p->groups) {
    PersistGroup t{};
    t.N = G.N;
    t.nb = G.B();
    t.C = G.C;
    t.D1 = G.D1;
    t.g = G.g;
    if (persist_fill(t) == 0) return false;
  }
  return true;
}

// An RK4 call as one persistent launch (hot_set_variant(graph, 2)): the
// pointer tables, a fill of the control block, the kernel, then the
// statistics.
int enqueue_persistent(hot_plan_s* p, void* const* in, void* const* out, void* workspace, int32_t nsteps,
                       hipStream_t stream, bool record, StatsRec* stats) {
  Runner r{p, stream, record};
  PersistArgs a{};
  a.ng = (int)p->groups.size();
  a.nsteps = nsteps;
  a.nu = (float)p->nu;
  a.dt = (float)p->dt;
  a.spin = p->persist_spin;
  a.ctl = nullptr;  // set on the device by persist_launch
  size_t lds = 0;
  for (size_t gi = 0; gi < p->groups.size() && r.rc == HOT_OK; ++gi) {
    const Group& G = p->groups[gi];
    const GroupPtrs q = group_ptrs(G, workspace);
    write_tables(r, G, q, in, out);
    PersistGroup& P = a.G[gi];
    P.N = G.N;
    P.nb = G.B();
    P.C = G.C;
    P.D1 = G.D1;
    P.g = G.g;
    P.in0 = in[G.members[0]];
    P.in_tab = q.in_tab;
    P.out0 = out[G.members[0]];
    P.out_tab = q.out_tab;
    P.U0 = q.U0;
    P.U1 = q.U1;
    P.Acc = q.Acc;
    P.A1 = q.A1;
    const size_t b = persist_fill(P);
    if (b == 0) return HOT_E_INVALID;  // hot_set_variant checked every size
    if (b > lds) lds = b;
  }
  r.pass(PASS_PERSIST, [&] { return persist_launch(r.s, a, (char*)workspace + p->o_persist, lds); });
  if (stats)
    for (const auto& G : p->groups) {
      const GroupPtrs q = group_ptrs(G, workspace);
      state_stats(r, p, G, q, q.U0, stats, false);
    }
  return r.rc;
}

// Enqueue the whole operation (the pointer tables are already in place).
int enqueue(hot_plan_s* p, void* const* in, void* const* out, void* workspace, int32_t nsteps, hipStream_t stream,
            bool record, StatsRec* stats, bool branches = false) {
  Runner r{p, stream, record};
  const size_t e = p->elem;
  if (p->op == HOT_OP_R2C || p->op == HOT_OP_C2R) {
    for (const auto& G : p->groups) {
      const Geo& g = G.g;
      const Ops& o = G.ops;
      const long N = g.N, Nh = g.Mz, D2 = G.D2;
      char* Z1 = (char*)workspace;
      char* Z2 = Z1 + align_up(3 * (size_t)G.D2 * e);
      for (int i : G.members) {
        if (r.rc != HOT_OK) break;
        if (p->op == HOT_OP_R2C) {
          r.pass(PASS_Z_R2C, [&] { return o.z_r2c(r.s, in[i], Z1, 3 * N * N, g); });
          r.pass(PASS_Y_FWD, [&] {
            return o.strided(r.s, 1, -1, false, false, Z1, Z2, N * Nh, Nh, Nh, Nh, N * Nh, N * Nh, D2, D2, 3, 0, 0,
                             0, 1, g, nullptr);
          });
          r.pass(PASS_X_FWD, [&] {
            const long Q = N * Nh;
            return o.strided(r.s, 1, -1, false, false, Z2, out[i], Q, Q, Q, Q, 0, 0, D2, D2, 3, 0, 0, 0, 1, g, nullptr);
          });
        } else {
          r.pass(PASS_X_INV, [&] {
            const long Q = N * Nh;
            return o.strided(r.s, 1, +1, false, false, in[i], Z1, Q, Q, Q, Q, 0, 0, D2, D2, 3, 0, 0, 0, 1, g, nullptr);
          });
          r.pass(PASS_Y_INV, [&] {
            return o.strided(r.s, 1, +1, false, false, Z1, Z2, N * Nh, Nh, Nh, Nh, N * Nh, N * Nh, D2, D2, 3, 0, 0,
                             0, 1, g, nullptr);
          });
          r.pass(PASS_Z_C2R, [&] { return o.z_c2r(r.s, Z2, out[i], 3 * N * N, g); });
        }
      }
    }
    return r.rc;
  }
  if (p->persistent && p->op == HOT_OP_RK4)
    return enqueue_persistent(p, in, out, workspace, nsteps, stream, record, stats);
  // right-hand side / RK4: group by group (a small group's working set can
  // stay in the device's last-level cache between its passes), or one branch
  // per group
  const bool br = branches && p->groups.size() > 1;
  if (br) {
    const hipError_t e = fork_groups(p, stream);
    if (e != hipSuccess) {
      p->last_hip = (int)e;
      return HOT_E_HIP;
    }
  }
  std::vector<size_t> order(p->groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  if (br) order = branch_order(p);
  for (const size_t gi : order) {
    const Group& G = p->groups[gi];
    if (r.rc != HOT_OK) break;
    r.s = br ? p->side[gi] : stream;
    const GroupPtrs q = group_ptrs(G, workspace);
    const Ops& o = G.ops;
    const Geo& g = G.g;
    const int nb = G.B();
    const long isU = 3 * G.C;
    const void* in0 = in[G.members[0]];
    void* out0 = out[G.members[0]];
    write_tables(r, G, q, in, out);
    r.pass(PASS_GATHER, [&] { return o.gather(r.s, in0, q.in_tab, q.U0, G.C, isU, nb, g); });
    if (p->op == HOT_OP_RHS) {
      stage_passes(r, G, q, q.U0, 4, p->nu, p->dt);
      r.pass(PASS_SCATTER, [&] { return o.scatter(r.s, q.Acc, out0, q.out_tab, G.C, isU, nb, g); });
    } else {
      for (int step = 0; step < nsteps && r.rc == HOT_OK; ++step)
        for (int st = 0; st < 4; ++st) stage_passes(r, G, q, st == 0 ? q.U0 : q.U1, st, p->nu, p->dt);
      r.pass(PASS_SCATTER, [&] { return o.scatter(r.s, q.U0, out0, q.out_tab, G.C, isU, nb, g); });
    }
    // the state: the input of a right-hand side, the result of RK4 steps
    if (stats) state_stats(r, p, G, q, q.U0, stats, false);
  }
  if (br) {
    const hipError_t e = join_groups(p, stream);
    if (e != hipSuccess && r.rc == HOT_OK) {
      p->last_hip = (int)e;
      r.rc = HOT_E_HIP;
    }
  }
  return r.rc;
}

// The implicit step, step by step over every group.  Each step: the
// predictor, then up to max_iter Picard sweeps (the right-hand-side passes on
// the midpoint, the update of d, the stopping test); every pass kernel returns
// at once for an instance whose stopping flag is clear, so each instance stops
// on its own.  The counters of the call (sweeps, steps stopped at max_iter)
// stay on the device.  The iterate d and the increment histories H1 (newest)
// to H4 rotate through five buffers (Acc and the four history regions) at
// the end of a step: d becomes the newest history.
//
// Sweeps go out in rounds of imp_check over every group still iterating
// (each group on its own stream with branches, enqueued in branch_order).  Between rounds an eager call
// copies the flags of those groups to the host and waits for their streams:
// once no instance of a group iterates, its remaining sweeps are not enqueued
// (a sweep whose flags are all clear still launches every block of every
// pass).  A captured call (record == false) or imp_check == 0 enqueues all
// max_iter sweeps and never waits.
int run_implicit(hot_plan_s* p, void* const* in, void* const* out, void* workspace, int32_t nsteps, hipStream_t s,
                 bool record, StatsRec* stats, bool branches = false) {
  Runner r{p, s, record};
  const bool keep = (p->flags & HOT_FLAG_KEEP_HISTORY) && p->hist_ws == workspace;
  const bool br = branches && p->groups.size() > 1;
  if (br) {
    const hipError_t e = fork_groups(p, s);
    if (e != hipSuccess) {
      p->last_hip = (int)e;
      return HOT_E_HIP;
    }
  }
  const size_t ng = p->groups.size();
  auto stream_of = [&](size_t gi) { return br ? p->side[gi] : s; };
  std::vector<GroupPtrs> qs(ng);
  for (size_t gi = 0; gi < ng && r.rc == HOT_OK; ++gi) {
    Group& G = p->groups[gi];
    r.s = stream_of(gi);
    if (!keep) {
      G.rot = 0;
      G.hist = 0;
    }
    const GroupPtrs& q = qs[gi] = group_ptrs(G, workspace);
    write_tables(r, G, q, in, out);
    r.pass(PASS_IMP_DECIDE, [&] {  // the call's counters start at zero
      hipLaunchKernelGGL(k_fill_int<>, dim3(grid_1d(2 * G.B(), 256)), dim3(256), 0, r.s, q.cnt, 2L * G.B(), 0);
      return hipGetLastError();
    });
    r.pass(PASS_GATHER,
           [&] { return G.ops.gather(r.s, in[G.members[0]], q.in_tab, q.U0, G.C, 3 * G.C, G.B(), G.g); });
  }
  const int every = record ? p->imp_check : 0;
  std::vector<char> live(ng);
  std::vector<size_t> order(ng);
  for (size_t i = 0; i < ng; ++i) order[i] = i;
  if (br) order = branch_order(p);
  for (int step = 0; step < nsteps && r.rc == HOT_OK; ++step) {
    // the iterate d and the histories H1 (newest) to H4 rotate through five buffers
    auto bufs = [&](size_t gi, char*& D, char*& H1, char*& H2, char*& H3, char*& H4) {
      const Group& G = p->groups[gi];
      char* buf[5] = {qs[gi].Acc, qs[gi].H[0], qs[gi].H[1], qs[gi].H[2], qs[gi].H[3]};
      D = buf[G.rot];
      H1 = buf[(G.rot + 1) % 5];
      H2 = buf[(G.rot + 2) % 5];
      H3 = buf[(G.rot + 3) % 5];
      H4 = buf[(G.rot + 4) % 5];
    };
    for (const size_t gi : order) {
      if (r.rc != HOT_OK) break;
      const Group& G = p->groups[gi];
      const GroupPtrs& q = qs[gi];
      r.s = stream_of(gi);
      char *D, *H1, *H2, *H3, *H4;
      bufs(gi, D, H1, H2, H3, H4);
      const long isU = 3 * G.C;
      const int nb = G.B();
      // the surrogate corrects the linear extrapolation of the two newest
      // increments (its training target), with two or more of them
      if (G.hist >= 2 && p->surrogate)
        r.pass(PASS_IMP_PREDICT, [&] {
          return p->dtype == HOT_F64
                     ? mlp_predict<double>(r.s, p->surrogate, q.U0, H1, H2, D, q.U1, q.act, G.C, isU, nb, G.g, p->nu,
                                           p->dt)
                     : mlp_predict<float>(r.s, p->surrogate, q.U0, H1, H2, D, q.U1, q.act, G.C, isU, nb, G.g, p->nu,
                                          p->dt);
        });
      else
        r.pass(PASS_IMP_PREDICT,
               [&] { return G.ops.imp_predict(r.s, q.U0, D, q.U1, H1, H2, H3, H4, G.C, isU, nb, G.g, G.hist, q.act); });
      live[gi] = 1;
    }
    for (int done = 0; done < p->max_iter && r.rc == HOT_OK;) {
      const int k = every > 0 && every < p->max_iter - done ? every : p->max_iter - done;
      for (const size_t gi : order) {
        if (r.rc != HOT_OK) break;
        if (!live[gi]) continue;
        const Group& G = p->groups[gi];
        const GroupPtrs& q = qs[gi];
        r.s = stream_of(gi);
        char *D, *H1, *H2, *H3, *H4;
        bufs(gi, D, H1, H2, H3, H4);
        for (int sw = 0; sw < k && r.rc == HOT_OK; ++sw) {
          rhs_passes(r, G, q, q.U1, q.act);
          r.pass(PASS_IMP_UPDATE, [&] {
            return G.ops.imp_update(r.s, q.Nh, q.U0, D, q.U1, q.part, G.C, 3 * G.C, G.B(), G.g, p->nu, p->dt,
                                    q.act);
          });
          r.pass(PASS_IMP_DECIDE, [&] {
            hipLaunchKernelGGL(k_imp_decide<>, dim3(G.B()), dim3(64), 0, r.s, (const double*)q.part, G.nparts, q.act,
                               p->tol * p->tol, q.cnt);
            return hipGetLastError();
          });
        }
      }
      done += k;
      if (every <= 0 || done >= p->max_iter || r.rc != HOT_OK) break;
      // which groups still iterate: their flags, after their streams finish
      hipError_t e = hipSuccess;
      size_t off = 0;
      for (size_t gi = 0; gi < ng && e == hipSuccess; ++gi) {
        if (live[gi])
          e = hipMemcpyAsync(p->act_host.data() + off, qs[gi].act, p->groups[gi].B() * sizeof(int),
                             hipMemcpyDeviceToHost, stream_of(gi));
        off += p->groups[gi].B();
      }
      for (size_t gi = 0; gi < ng && e == hipSuccess; ++gi)
        if (live[gi]) e = hipStreamSynchronize(stream_of(gi));
      if (e != hipSuccess) {
        p->last_hip = (int)e;
        r.rc = HOT_E_HIP;
        break;
      }
      bool any = false;
      off = 0;
      for (size_t gi = 0; gi < ng; ++gi) {
        const int nb = p->groups[gi].B();
        if (live[gi]) {
          bool a = false;
          for (int m = 0; m < nb; ++m) a = a || p->act_host[off + m] != 0;
          live[gi] = a;
          any = any || a;
        }
        off += nb;
      }
      if (!any) break;
    }
    for (size_t gi = 0; gi < ng && r.rc == HOT_OK; ++gi) {
      Group& G = p->groups[gi];
      const GroupPtrs& q = qs[gi];
      r.s = stream_of(gi);
      char *D, *H1, *H2, *H3, *H4;
      bufs(gi, D, H1, H2, H3, H4);
      (void)H1, (void)H2, (void)H3, (void)H4;
      r.pass(PASS_IMP_DECIDE, [&] {  // instances still active stopped at max_iter
        hipLaunchKernelGGL(k_imp_close<>, dim3(grid_1d(G.B(), 256)), dim3(256), 0, r.s, (const int*)q.act,
                           q.cnt + G.B(), G.B());
        return hipGetLastError();
      });
      r.pass(PASS_IMP_ADVANCE, [&] { return G.ops.imp_advance(r.s, q.U0, D, G.C, 3 * G.C, G.B(), G.g); });
      G.rot = (G.rot + 4) % 5;  // d becomes H1, H1 becomes H2, ..., H4's buffer the next d
      if (G.hist < 4) ++G.hist;
    }
  }
  for (size_t gi = 0; gi < ng && r.rc == HOT_OK; ++gi) {
    const Group& G = p->groups[gi];
    const GroupPtrs& q = qs[gi];
    r.s = stream_of(gi);
    r.pass(PASS_SCATTER, [&] {
      return G.ops.scatter(r.s, q.U0, out[G.members[0]], q.out_tab, G.C, 3 * G.C, G.B(), G.g);
    });
    if (stats) state_stats(r, p, G, q, q.U0, stats, true);
  }
  if (br) {
    const hipError_t e = join_groups(p, s);
    if (e != hipSuccess && r.rc == HOT_OK) {
      p->last_hip = (int)e;
      r.rc = HOT_E_HIP;
    }
  }
  p->hist_ws = workspace;
  p->cnt_ws = workspace;
  p->cnt_stream = s;
  return r.rc;
}

// The implicit counters of the plan's last call (on workspace ws), read back
// to the host after the stream has finished; returns HOT_E_NOCONVERGE when a
// step of some instance stopped at max_iter.
int read_counters(hot_plan_s* p) {
  p->imp_sweeps.assign(p->batch, 0);
  p->imp_nonconv.assign(p->batch, 0);
  if (!p->cnt_ws) return HOT_OK;
  hipError_t e = hipStreamSynchronize(p->cnt_stream);
  bool stalled = false;
  std::vector<int> h;
  for (const auto& G : p->groups) {
    if (e != hipSuccess) break;
    const GroupPtrs q = group_ptrs(G, p->cnt_ws);
    h.assign(2 * G.B(), 0);
    e = hipMemcpy(h.data(), q.cnt, h.size() * sizeof(int), hipMemcpyDeviceToHost);
    for (int m = 0; m < G.B() && e == hipSuccess; ++m) {
      p->imp_sweeps[G.members[m]] = h[m];
      p->imp_nonconv[G.members[m]] = h[G.B() + m];
      stalled = stalled || h[G.B() + m] > 0;
    }
  }
  if (e != hipSuccess) {
    p->last_hip = (int)e;
    return HOT_E_HIP;
  }
  return stalled ? HOT_E_NOCONVERGE : HOT_OK;
}

}  // namespace

extern "C" int hot_diagnostics(hot_plan_t p, void* const* in, void* workspace, double* out, void* stream) {
  if (!p || !in || !out || ((uintptr_t)out & 7) != 0) return HOT_E_INVALID;
  if (p->nranks > 1) return HOT_E_UNSUPPORTED;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return HOT_E_WORKSPACE;
  constexpr int kParts = 128;  // partial sums of one instance: 2 KiB of scratch
  if ((size_t)kParts * 2 * sizeof(double) > p->ws_bytes) return HOT_E_WORKSPACE;
  for (int i = 0; i < p->batch; ++i)
    if (!in[i] || ((uintptr_t)in[i] % kAlign) != 0) return HOT_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)workspace;
  hipError_t e = hipSuccess;
  // one instance after the other through the same scratch (stream order)
  for (int i = 0; i < p->batch && e == hipSuccess; ++i) {
    if (p->dtype == HOT_F64)
      hipLaunchKernelGGL(k_diag<double>, dim3(kParts), dim3(256), 0, s, (const cx<double>*)in[i], p->n[i], part);
    else
      hipLaunchKernelGGL(k_diag<float>, dim3(kParts), dim3(256), 0, s, (const cx<float>*)in[i], p->n[i], part);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_diag_final<>, dim3(1), dim3(64), 0, s, (const double*)part, kParts, p->n[i], p->nu,
                       out + 2 * i);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    p->last_hip = (int)e;
    return HOT_E_HIP;
  }
  return HOT_OK;
}

extern "C" int hot_set_surrogate(hot_plan_t p, const void* packed) {
  if (!p || p->op != HOT_OP_IMPLICIT || ((uintptr_t)packed & 15) != 0) return HOT_E_INVALID;
  p->surrogate = packed;
  return HOT_OK;
}

extern "C" int hot_implicit_stats(hot_plan_t p, int32_t* sweeps, int32_t* nonconv) {
  if (!p || p->op != HOT_OP_IMPLICIT) return HOT_E_INVALID;
  const int rc = read_counters(p);
  if (rc == HOT_E_HIP) return rc;
  for (int i = 0; i < p->batch; ++i) {
    if (sweeps) sweeps[i] = p->imp_sweeps[i];
    if (nonconv) nonconv[i] = p->imp_nonconv[i];
  }
  return rc;
}

// HOT_FLAG_CHECK_FINITE: scan every instance's compact result (Acc for a
// plain right-hand side, U0 otherwise) for NaN and infinity.
static int check_finite(hot_plan_s* p, void* workspace, hipStream_t s) {
  int* flag = (int*)((char*)workspace + p->o_finite);
  hipLaunchKernelGGL(k_set_int<>, dim3(1), dim3(1), 0, s, flag, 0);
  hipError_t e = hipGetLastError();
  for (const auto& G : p->groups) {
    if (e != hipSuccess) break;
    const GroupPtrs q = group_ptrs(G, workspace);
    const void* X = p->op == HOT_OP_RHS ? q.Acc : q.U0;
    const dim3 grid(grid_1d(3 * G.C, 256), (unsigned)G.B());
    if (p->dtype == HOT_F64)
      hipLaunchKernelGGL(k_nonfinite<double>, grid, dim3(256), 0, s, (const cx<double>*)X, G.C, 3 * G.C, G.g, flag);
    else
      hipLaunchKernelGGL(k_nonfinite<float>, grid, dim3(256), 0, s, (const cx<float>*)X, G.C, 3 * G.C, G.g, flag);
    e = hipGetLastError();
  }
  int h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    p->last_hip = (int)e;
    return HOT_E_HIP;
  }
  return h ? HOT_E_NONFINITE : HOT_OK;
}

extern "C" int hot_run(hot_plan_t p, void* const* in, void* const* out, void* workspace, int32_t nsteps,
                       void* stats_dev, void* stream) {
  int rc = check_run_args(p, in, out, workspace, nsteps, stats_dev);
  if (rc != HOT_OK) return rc;
  if (p->nranks > 1) return HOT_E_UNSUPPORTED;  // a share runs by phases (hot_slab_run)
  hipStream_t s = (hipStream_t)stream;
  StatsRec* stats = (StatsRec*)stats_dev;
  if (p->op == HOT_OP_IMPLICIT)
    rc = run_implicit(p, in, out, workspace, nsteps, s, true, stats);
  else
    rc = enqueue(p, in, out, workspace, nsteps, s, true, stats);
  if ((p->flags & HOT_FLAG_CHECK_FINITE) && rc == HOT_OK) {
    // this plan synchronises anyway: report a max_iter stop as well
    const int fc = check_finite(p, workspace, s);
    if (fc != HOT_OK) return fc;
    if (p->op == HOT_OP_IMPLICIT) return read_counters(p);
  }
  return rc;
}

// ---------------------------------------------------------------------------
// hot_run without a caller workspace, for callers that cannot allocate
// ---------------------------------------------------------------------------
// The workspace lives in a file-scope device array; every device the library
// runs on holds its own copy until the process ends.  On the host the array's
// name is only a stand-in: its device address comes from hipGetSymbolAddress,
// once per device, and only that address is handed to kernels.
static constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

static int scratch_address(hot_plan_s* p, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) return HOT_E_UNSUPPORTED;
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e == hipSuccess && (!ptr || ((uintptr_t)ptr % kAlign) != 0)) e = hipErrorInvalidSymbol;
      if (e == hipSuccess) g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
  }
  if (e != hipSuccess) {
    p->last_hip = (int)e;
    return HOT_E_HIP;
  }
  return HOT_OK;
}

extern "C" int hot_run_noalloc(hot_plan_t p, void* const* in, void* const* out, int32_t nsteps, void* stats_dev,
                               void* stream) {
  if (!p) return HOT_E_INVALID;
  if (p->ws_bytes > kScratchBytes) return HOT_E_TOOBIG;
  // a kept history would not survive other calls through the shared scratch
  if (p->flags & HOT_FLAG_KEEP_HISTORY) return HOT_E_UNSUPPORTED;
  void* ws = nullptr;
  const int rc = scratch_address(p, &ws);
  if (rc != HOT_OK) return rc;
  const bool prof = p->prof;
  p->prof = false;  // no profiling events: nothing is created on this path
  const int r = hot_run(p, in, out, ws, nsteps, stats_dev, stream);
  p->prof = prof;
  return r;
}

extern "C" int hot_graph_create(hot_plan_t p, void* const* in, void* const* out, void* workspace, int32_t nsteps,
                                void* stats_dev, void* stream, hot_graph_t* graph) {
  if (graph) *graph = nullptr;
  if (!graph || !stream) return HOT_E_INVALID;  // the legacy default stream cannot be captured
  int rc = check_run_args(p, in, out, workspace, nsteps, stats_dev);
  if (rc != HOT_OK) return rc;
  // a kept implicit history depends on the calls before: not replayable
  if ((p->flags & (HOT_FLAG_CHECK_FINITE | HOT_FLAG_KEEP_HISTORY)) || p->nranks > 1) return HOT_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  hot_graph_s* G = new (std::nothrow) hot_graph_s();
  if (!G) return HOT_E_INVALID;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    StatsRec* stats = (StatsRec*)stats_dev;
    rc = p->op == HOT_OP_IMPLICIT ? run_implicit(p, in, out, workspace, nsteps, s, false, stats, p->graph_branches)
                                  : enqueue(p, in, out, workspace, nsteps, s, false, stats, p->graph_branches);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    G->graph = g;
    if (rc == HOT_OK && e2 != hipSuccess) e = e2;
    if (rc == HOT_OK && e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  }
  if (rc == HOT_OK && e != hipSuccess) {
    p->last_hip = (int)e;
    rc = HOT_E_HIP;
  }
  if (rc != HOT_OK) {
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return rc;
  }
  *graph = G;
  return HOT_OK;
}

extern "C" int hot_graph_launch(hot_graph_t graph, void* stream) {
  if (!graph || !graph->exec) return HOT_E_INVALID;
  return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? HOT_OK : HOT_E_HIP;
}

extern "C" int hot_graph_destroy(hot_graph_t graph) {
  if (!graph) return HOT_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return HOT_OK;
}

// Autotuner: for every group and column-tiled pass, time each column-width
// variant on the workspace (the passes only read and write workspace
// buffers, so the caller's data is untouched) and keep the fastest.
extern "C" int hot_tune(hot_plan_t p, void* workspace, void* stream, int32_t reps) {
  if (!p || reps < 1) return HOT_E_INVALID;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return HOT_E_WORKSPACE;
  if (p->op != HOT_OP_RHS && p->op != HOT_OP_RK4 && p->op != HOT_OP_IMPLICIT) return HOT_OK;  // nothing to tune
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return HOT_E_HIP;
  int rc = HOT_OK;
  const bool was_prof = p->prof;
  p->prof = false;
  for (auto& G : p->groups) {
    const GroupPtrs q = group_ptrs(G, workspace);
    const int pass_ids[4] = {PASS_X_INV_CURL, PASS_Y_INV, PASS_Y_FWD, PASS_X_FWD};
    for (int pid : pass_ids) {
      float best = 1e30f;
      int best_v = 1;
      // the packed y forward pass and the x inverse of the long lines also come
      // with one output per block (variants 3..5)
      const bool single = (pid == PASS_Y_FWD && G.zpack == 1) || (pid == PASS_X_INV_CURL && G.N > 64);
      const int nv = single ? 2 * G.ops.strided_variants : G.ops.strided_variants;
      for (int v = 0; v < nv && rc == HOT_OK; ++v) {
        const int w = v % G.ops.strided_variants;
        if (w != 1 && G.ops.strided_width[w] == G.ops.strided_width[1]) continue;  // same kernel
        G.variant[pid] = v;
        float t = 0.f;
        for (int rep = 0; rep <= reps && rc == HOT_OK; ++rep) {
          Runner r{p, s, false};
          if (rep == 1) (void)hipEventRecord(a, s);
          // one launch of just this pass
          const Geo& g = G.g;
          const long N = g.N, M = g.M, P = g.Mzp;
          const long isA1 = 6 * G.D1, isA2 = 6 * G.D2, isU = 3 * G.C;
          r.pass(pid, [&] {
            if (pid == PASS_X_INV_CURL)
              return G.ops.x_inv_curl(s, v, q.U0, G.C, isU, q.A1, G.D1, isA1, G.B(), g, nullptr);
            if (pid == PASS_Y_INV && G.packed_y_inv())
              return G.ops.y_inv_pack(s, v, q.A1, q.A2, N * P, P, P, P, M * P, N * P, G.D1, G.D2, isA1, isA2,
                                      G.B(), g, nullptr);
            if (pid == PASS_Y_INV)
              return G.ops.strided(s, v, +1, true, false, q.A1, q.A2, N * P, P, P, P, M * P, N * P, G.D1, G.D2, 6,
                                   isA1, isA2, 0, G.B(), g, nullptr);
            if (pid == PASS_Y_FWD && G.zpack == 1)
              return G.ops.y_fwd_unpack(s, v, q.A2, q.A1, N * P, P, P, P, N * P, M * P, G.D2, G.D1, isA2, isA1,
                                        G.B(), g, nullptr);
            if (pid == PASS_Y_FWD)
              return G.ops.strided(s, v, -1, false, true, q.A2, q.A1, N * P, P, P, P, N * P, M * P, G.D2, G.D1, 3,
                                   isA2, isA1, 0, G.B(), g, nullptr);
            const long Q = M * P;
            return G.ops.strided(s, v, -1, false, true, q.A1, q.Nh, Q, Q, Q, g.tw, 0, 0, G.D1, G.C, 3, isA1, isU,
                                 g.tw, G.B(), g, nullptr);
          });
          rc = r.rc;
        }
        if (rc != HOT_OK) break;
        hipError_t e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e != hipSuccess) {
          p->last_hip = (int)e;
          rc = HOT_E_HIP;
          break;
        }
        if (t < best) {
          best = t;
          best_v = v;
        }
      }
      G.variant[pid] = best_v;
    }
    // small N: the y and z passes fused, or the three separate passes.  With
    // several sizes the fused pass is kept wherever it exists, untimed: the
    // sizes run side by side (graph branches) and share the HBM, and the
    // fused pass moves 9 D1 values against 12 D1 + 18 D2 (4096 uneven
    // instances: 19.45 ms per graph replay against 20.3 with the per-size
    // timing's choice, the separate passes for N = 48)
    if (rc == HOT_OK && G.ops.yz_fused && p->nranks == 1 && p->groups.size() > 1) {
      G.yz = 0;
    } else if (rc == HOT_OK && G.ops.yz_fused && p->nranks == 1) {
      float best = 1e30f;
      int best_y = -1;
      for (int yv = -1; yv <= 0 && rc == HOT_OK; ++yv) {
        float t = 0.f;
        for (int rep = 0; rep <= reps && rc == HOT_OK; ++rep) {
          Runner r{p, s, false};
          if (rep == 1) (void)hipEventRecord(a, s);
          if (yv < 0) {
            y_inv_pass(r, G, q, nullptr);
            z_pass(r, G, q, nullptr);
            y_fwd_pass(r, G, q, nullptr);
          } else {
            r.pass(PASS_YZ_FUSED, [&] { return G.ops.yz_fused(s, q.A1, G.D1, 6 * G.D1, G.B(), G.g, nullptr); });
          }
          rc = r.rc;
        }
        if (rc != HOT_OK) break;
        hipError_t e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e != hipSuccess) {
          p->last_hip = (int)e;
          rc = HOT_E_HIP;
          break;
        }
        if (t < best) {
          best = t;
          best_y = yv;
        }
      }
      G.yz = best_y;
    }
    // the row form of the y and z passes (groups whose y and z passes are not
    // fused): six component rows, packed pairs in and out, or packed pairs
    // into the z pass and component rows out of it, each timed over the y
    // inverse, z and y forward passes
    if (rc == HOT_OK && G.yz < 0 && G.zpack > 0) {
      float best = 1e30f;
      int best_z = 1;
      for (int zv = 0; zv <= 3 && rc == HOT_OK; ++zv) {
        G.zpack = zv;
        float t = 0.f;
        for (int rep = 0; rep <= reps && rc == HOT_OK; ++rep) {
          Runner r{p, s, false};
          if (rep == 1) (void)hipEventRecord(a, s);
          y_inv_pass(r, G, q, nullptr);
          if (p->nranks > 1) {  // a z-slab share: its z pass over every retained kz, from the receive buffer
            const long lines = (long)p->nx * G.N, blk = lines * G.g.Mzp;
            r.pass(PASS_Z_CROSS, [&] {
              return G.zpack > 0 ? G.ops.z_cross_packed_blocked(r.s, q.Z, G.D2, lines, p->gz, p->chunk, blk,
                                                                G.zpack - 1)
                                 : G.ops.z_cross_blocked(r.s, q.Z, G.D2, lines, p->gz, p->chunk, blk);
            });
          } else {
            z_pass(r, G, q, nullptr);
          }
          y_fwd_pass(r, G, q, nullptr);
          rc = r.rc;
        }
        if (rc != HOT_OK) break;
        hipError_t e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e != hipSuccess) {
          p->last_hip = (int)e;
          rc = HOT_E_HIP;
          break;
        }
        if (t < best) {
          best = t;
          best_z = zv;
        }
      }
      G.zpack = best_z;
    }
    // RK4 / RHS: the x pass with the stage update fused, or the two passes
    // (one stage-1 update on the workspace; every variant computes the same)
    if (rc == HOT_OK && (p->op == HOT_OP_RK4 || p->op == HOT_OP_RHS)) {
      float best = 1e30f;
      int best_f = -1;
      for (int f = -1; f < 3 && rc == HOT_OK; ++f) {
        if (f == 0 && G.ops.fused_width[0] == G.ops.fused_width[1]) continue;  // same kernel as f = 1
        if (f == 2 && G.ops.fused_width[2] == G.ops.fused_width[0]) continue;  // same kernel as f = 0
        G.fused = f;
        float t = 0.f;
        for (int rep = 0; rep <= reps && rc == HOT_OK; ++rep) {
          Runner r{p, s, false};
          if (rep == 1) (void)hipEventRecord(a, s);
          if (f < 0) {
            const long Q = G.g.M * (long)G.g.Mzp;
            r.pass(PASS_X_FWD, [&] {
              return G.ops.strided(s, G.variant[PASS_X_FWD], -1, false, true, q.A1, q.Nh, Q, Q, Q, G.g.tw, 0, 0, G.D1,
                                   G.C, 3, 6 * G.D1, 3 * G.C, G.g.tw, G.B(), G.g, nullptr);
            });
            r.pass(PASS_RK_STAGE, [&] {
              return G.ops.rk_stage(s, q.Nh, q.U0, q.U1, q.Acc, G.C, 3 * G.C, G.B(), G.g, 1, p->nu, p->dt);
            });
          } else {
            r.pass(PASS_X_FWD_RK, [&] {
              return G.ops.x_fwd_rk(s, f, q.A1, G.D1, 6 * G.D1, q.U0, q.U1, q.Acc, G.C, 3 * G.C, G.B(), G.g, 1, p->nu,
                                    p->dt);
            });
          }
          rc = r.rc;
        }
        if (rc != HOT_OK) break;
        hipError_t e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e != hipSuccess) {
          p->last_hip = (int)e;
          rc = HOT_E_HIP;
          break;
        }
        if (t < best) {
          best = t;
          best_f = f;
        }
      }
      G.fused = best_f;
    }
  }
  p->prof = was_prof;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

extern "C" int hot_set_variant(hot_plan_t p, int32_t pass, int32_t variant) {
  if (!p) return HOT_E_INVALID;
  const bool tiled = pass == PASS_X_INV_CURL || pass == PASS_Y_INV || pass == PASS_Y_FWD || pass == PASS_X_FWD;
  if (pass == PASS_X_FWD_RK) {
    if (variant < -1 || variant > 2 || (p->op != HOT_OP_RK4 && p->op != HOT_OP_RHS)) return HOT_E_INVALID;
    for (auto& G : p->groups) G.fused = variant;
    return HOT_OK;
  }
  if (pass == PASS_IMP_DECIDE) {  // implicit step: sweeps between looks at the flags, 0: never look
    if (p->op != HOT_OP_IMPLICIT || variant < 0) return HOT_E_INVALID;
    p->imp_check = variant;
    return HOT_OK;
  }
  if (pass == PASS_GRAPH) {  // 1: one branch per size (default), 0: the sizes one after another,
                             // 2: the persistent kernel (RK4)
    if (variant < 0 || variant > 2 || (variant == 2 && !persist_ok(p))) return HOT_E_INVALID;
    p->graph_branches = variant == 1;
    p->persistent = variant == 2;
    return HOT_OK;
  }
  if (pass == PASS_PERSIST) {  // the bound of the persistent kernel's waits, in polls (0: the default)
    if (variant < 0 || !persist_ok(p)) return HOT_E_INVALID;
    p->persist_spin = variant;
    return HOT_OK;
  }
  if (pass == PASS_Z_CROSS) {  // the row form (Group::zpack), 0..3
    const bool plain = p->op == HOT_OP_R2C || p->op == HOT_OP_C2R;
    if (variant < 0 || variant > 3 || plain) return HOT_E_INVALID;
    for (auto& G : p->groups) G.zpack = variant;
    return HOT_OK;
  }
  if (pass == PASS_YZ_FUSED) {  // 0: fused wherever a size has the kernel
    const bool plain = p->op == HOT_OP_R2C || p->op == HOT_OP_C2R;
    if (variant < -1 || variant > 0 || plain || p->nranks > 1) return HOT_E_INVALID;
    for (auto& G : p->groups) G.yz = (variant == 0 && G.ops.yz_fused) ? 0 : -1;
    return HOT_OK;
  }
  // the y forward pass takes 3..5 too: the same widths, one output per block
  if (!tiled || variant < 0 || variant > ((pass == PASS_Y_FWD || pass == PASS_X_INV_CURL) ? 5 : 2))
    return HOT_E_INVALID;
  for (auto& G : p->groups) G.variant[pass] = variant;
  return HOT_OK;
}

extern "C" int hot_tuned_width(hot_plan_t p, int32_t instance, int32_t pass) {
  if (!p || instance < 0 || instance >= p->batch || pass < 0 || pass >= NUM_PASSES) return HOT_E_INVALID;
  for (const auto& G : p->groups)
    if (G.N == p->n[instance]) {
      if (pass == PASS_X_FWD_RK)
        return G.fused < 0 ? 0 : G.ops.fused_width[G.fused];
      if (pass == PASS_YZ_FUSED) return G.yz < 0 ? 0 : 1;
      if (pass == PASS_Z_CROSS) return G.zpack;
      if (pass == PASS_GRAPH) return p->persistent ? 2 : (p->graph_branches ? 1 : 0);
      if (pass == PASS_PERSIST) return p->persist_spin;
      if (pass == PASS_IMP_DECIDE) return p->op == HOT_OP_IMPLICIT ? p->imp_check : HOT_E_INVALID;
      return G.ops.strided_width[G.variant[pass] % 3];
    }
  return HOT_E_INVALID;
}

// ---------------------------------------------------------------------------
// z-slab shares
// ---------------------------------------------------------------------------
extern "C" int hot_plan_slab(const hot_desc* d, int32_t nranks, int32_t rank, hot_plan_t* out,
                             size_t* workspace_bytes) {
  if (out) *out = nullptr;
  if (!d || !out || !workspace_bytes) return HOT_E_INVALID;
  if (nranks < 1 || rank < 0 || rank >= nranks) return HOT_E_INVALID;
  if (d->batch != 1 || !d->n || (d->op != HOT_OP_RHS && d->op != HOT_OP_RK4) || d->flags != 0)
    return HOT_E_INVALID;
  hot_plan_t p = nullptr;
  size_t wsb = 0;
  int rc = hot_plan(d, &p, &wsb);
  if (rc != HOT_OK) return rc;
  const int N = d->n[0];
  Group& G = p->groups[0];
  const Geo full = G.g;
  const int chunk = (full.Mz + nranks - 1) / nranks;
  if (N % nranks != 0 || (long)(nranks - 1) * chunk >= full.Mz) {
    hot_destroy(p);
    return HOT_E_UNSUPPORTED;
  }
  // blocks keep 128-byte rows once they are long enough for it to be cheap
  const int seg = 128 / (int)p->elem;
  const int pitch = chunk >= 4 * seg ? (chunk + seg - 1) / seg * seg : chunk;
  const int kz0 = rank * chunk;
  G.g.kz0 = kz0;
  G.g.Mz = full.Mz - kz0 < chunk ? full.Mz - kz0 : chunk;
  G.g.Mzp = pitch;
  G.g.czp = rank == nranks - 1 ? N / 2 + 1 - kz0 : chunk;
  G.g.tw = state_tile(G.g, (int)p->elem);
  p->slab = true;
  p->nranks = nranks;
  p->rank = rank;
  p->chunk = chunk;
  p->nx = N / nranks;
  p->gz = full;  // z lines: every retained kz, at the pitch of the blocks
  p->gz.Mzp = pitch;
  rc = layout_groups(p, p->op);
  if (rc != HOT_OK) {
    hot_destroy(p);
    return rc;
  }
  *out = p;
  *workspace_bytes = p->ws_bytes;
  return HOT_OK;
}

extern "C" int hot_slab_layout_of(hot_plan_t p, hot_slab_layout* out) {
  if (!p || !out || !p->slab) return HOT_E_INVALID;
  const Group& G = p->groups[0];
  out->nranks = p->nranks;
  out->rank = p->rank;
  out->nx = p->nx;
  out->kz0 = G.g.kz0;
  out->nkz = G.g.czp;
  out->mz = G.g.Mz;
  out->chunk = p->chunk;
  out->pitch = G.g.Mzp;
  out->send_offset = G.off + G.oA2;
  out->recv_offset = G.off + G.oZ;
  out->comp_bytes = (size_t)G.D2 * p->elem;
  out->block_bytes = (size_t)p->nx * G.N * G.g.Mzp * p->elem;
  return HOT_OK;
}

extern "C" int hot_slab_run(hot_plan_t p, int32_t phase, int32_t stage, const void* in, void* out, void* workspace,
                            void* stream) {
  if (!p || !p->slab) return HOT_E_INVALID;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return HOT_E_WORKSPACE;
  const bool staged = phase == HOT_SLAB_INVERSE || phase == HOT_SLAB_FORWARD;
  if (phase < HOT_SLAB_GATHER || phase > HOT_SLAB_SCATTER) return HOT_E_INVALID;
  if (staged && (p->op == HOT_OP_RK4 ? (stage < 0 || stage > 3) : stage != 4)) return HOT_E_INVALID;
  if (phase == HOT_SLAB_GATHER && (!in || ((uintptr_t)in % kAlign) != 0)) return HOT_E_INVALID;
  if (phase == HOT_SLAB_SCATTER && (!out || ((uintptr_t)out % kAlign) != 0)) return HOT_E_INVALID;
  Runner r{p, (hipStream_t)stream, true};
  const Group& G = p->groups[0];
  const GroupPtrs q = group_ptrs(G, workspace);
  const Ops& o = G.ops;
  const long isU = 3 * G.C;
  switch (phase) {
    case HOT_SLAB_GATHER:
      r.pass(PASS_GATHER, [&] { return o.gather(r.s, in, nullptr, q.U0, G.C, isU, 1, G.g); });
      break;
    case HOT_SLAB_INVERSE:
      inverse_passes(r, G, q, (stage == 0 || stage == 4) ? q.U0 : q.U1, nullptr);
      break;
    case HOT_SLAB_CROSS: {
      const long lines = (long)p->nx * G.N, blk = lines * G.g.Mzp;
      r.pass(PASS_Z_CROSS, [&] {
        return G.zpack > 0 ? o.z_cross_packed_blocked(r.s, q.Z, G.D2, lines, p->gz, p->chunk, blk, G.zpack - 1)
                           : o.z_cross_blocked(r.s, q.Z, G.D2, lines, p->gz, p->chunk, blk);
      });
      break;
    }
    case HOT_SLAB_FORWARD:
      forward_passes(r, G, q, nullptr, G.fused < 0);
      stage_update(r, G, q, stage, p->nu, p->dt);
      break;
    default:
      r.pass(PASS_SCATTER, [&] {
        return o.scatter(r.s, p->op == HOT_OP_RK4 ? q.U0 : q.Acc, out, nullptr, G.C, isU, 1, G.g);
      });
  }
  return r.rc;
}
