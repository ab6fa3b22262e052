// libhot host side: plan validation, workspace layout, pass schedule and the
// C ABI of include/hot.h.  All arithmetic runs in the kernels of kernels.hpp.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/hot.h"
#include "impl.hpp"

namespace hot {

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
// geometry and workspace of one instance
// ---------------------------------------------------------------------------
struct Inst {
  Geo g;      // retained geometry for the op
  Ops ops;
  long C;     // compact slots per component, M*M*Mzp
  long D1;    // per component after the x pass: N*M*Mzp
  long D2;    // per component after the y pass: N*N*Mzp
  double lC, lD1, lD2;  // the same counts of live values (Mz instead of Mzp)
  size_t ws;  // workspace bytes
};

// mode: 0 = 2/3 rule, 1 = all but Nyquist, 2 = every mode (plain transforms).
// elem: bytes per complex value; the z pitch is padded to whole 128-byte rows
// once rows are long enough for the padding to be cheap.
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
  return g;
}

}  // namespace hot

using namespace hot;

struct hot_plan_s {
  int op, dtype, dealias;
  double nu, dt;
  size_t elem;  // bytes per complex element
  std::vector<Inst> inst;
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
};

static const size_t kAlign = 256;
static inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

extern "C" {

const char* hot_error_string(int code) {
  switch (code) {
    case HOT_OK: return "ok";
    case HOT_E_INVALID: return "invalid argument";
    case HOT_E_UNSUPPORTED: return "unsupported request";
    case HOT_E_WORKSPACE: return "workspace missing or misaligned";
    case HOT_E_HIP: return "HIP error";
    default: return "unknown error";
  }
}

int hot_plan(const hot_desc* d, hot_plan_t* out, size_t* workspace_bytes) {
  if (out) *out = nullptr;
  if (!d || !out || !workspace_bytes) return HOT_E_INVALID;
  if (d->abi_version != HOT_ABI_VERSION) return HOT_E_INVALID;
  if (d->batch < 1 || !d->n) return HOT_E_INVALID;
  if (d->dtype != HOT_F64 && d->dtype != HOT_F32) return HOT_E_INVALID;
  if (d->op < HOT_OP_R2C || d->op > HOT_OP_RK4) return HOT_E_INVALID;
  if (d->dealias != HOT_DEALIAS_TWO_THIRDS && d->dealias != HOT_DEALIAS_NONE) return HOT_E_INVALID;
  if (d->flags != 0) return HOT_E_INVALID;
  if (!(d->nu >= 0.0)) return HOT_E_INVALID;  // also rejects NaN
  if (d->op == HOT_OP_RK4 && !(d->dt > 0.0)) return HOT_E_INVALID;
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
  p->elem = d->dtype == HOT_F64 ? 16 : 8;
  p->last_hip = 0;
  p->prof = false;
  p->ws_bytes = 0;
  const bool plain = d->op == HOT_OP_R2C || d->op == HOT_OP_C2R;
  for (int i = 0; i < d->batch; ++i) {
    Inst I{};
    const int N = d->n[i];
    const bool ok = d->dtype == HOT_F64 ? ops_for<double>(N, &I.ops) : ops_for<float>(N, &I.ops);
    if (!ok) {
      delete p;
      return HOT_E_UNSUPPORTED;
    }
    I.g = make_geo(N, plain ? 2 : d->dealias, (int)p->elem);
    I.C = (long)I.g.M * I.g.M * I.g.Mzp;
    I.D1 = (long)N * I.g.M * I.g.Mzp;
    I.D2 = (long)N * N * I.g.Mzp;
    I.lC = (double)I.g.M * I.g.M * I.g.Mz;
    I.lD1 = (double)N * I.g.M * I.g.Mz;
    I.lD2 = (double)N * N * I.g.Mz;
    if (plain) {
      I.ws = 2 * align_up(3 * (size_t)I.D2 * p->elem);
    } else {
      I.ws = 4 * align_up(3 * (size_t)I.C * p->elem) + align_up(6 * (size_t)I.D1 * p->elem) +
             align_up(6 * (size_t)I.D2 * p->elem);
    }
    if (I.ws > p->ws_bytes) p->ws_bytes = I.ws;
    p->inst.push_back(I);
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
  if (!p || !bytes || instance < 0 || instance >= (int)p->inst.size()) return HOT_E_INVALID;
  const Inst& I = p->inst[instance];
  const double e = (double)p->elem, C = I.lC, D1 = I.lD1, D2 = I.lD2;
  const double N = I.g.N, canon = 3.0 * N * N * (N / 2 + 1);
  double b = 0;
  const bool plain = p->op == HOT_OP_R2C || p->op == HOT_OP_C2R;
  switch (pass) {
    case PASS_GATHER: b = plain ? 0 : 6 * C; break;  // read the 3C retained values, write 3C
    case PASS_X_INV_CURL: b = plain ? 0 : 3 * C + 6 * D1; break;
    case PASS_Y_INV: b = plain ? (p->op == HOT_OP_C2R ? 6 * D2 : 0) : 6 * D1 + 6 * D2; break;
    case PASS_Z_CROSS: b = plain ? 0 : 6 * D2 + 3 * D2; break;
    case PASS_Y_FWD: b = plain ? (p->op == HOT_OP_R2C ? 6 * D2 : 0) : 3 * D2 + 3 * D1; break;
    case PASS_X_FWD: b = plain ? (p->op == HOT_OP_R2C ? 6 * D2 : 0) : 3 * D1 + 3 * C; break;
    // RK4 stages move 12C, 18C, 18C, 12C (mean 15C); the plain RHS 9C
    case PASS_RK_STAGE: b = plain ? 0 : (p->op == HOT_OP_RHS ? 9 * C : 15 * C); break;
    case PASS_SCATTER: b = plain ? 0 : 3 * C + canon; break;
    case PASS_Z_R2C: b = p->op == HOT_OP_R2C ? 3 * D2 + 3 * N * N * N / 2 : 0; break;  // reals count half
    case PASS_Z_C2R: b = p->op == HOT_OP_C2R ? 3 * D2 + 3 * N * N * N / 2 : 0; break;
    case PASS_X_INV: b = p->op == HOT_OP_C2R ? 6 * D2 : 0; break;
    default: return HOT_E_INVALID;
  }
  *bytes = b * e;
  return HOT_OK;
}

}  // extern "C"

namespace {

struct Runner {
  hot_plan_s* p;
  hipStream_t s;
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
    if (p->prof) {
      a = ev();
      b = ev();
      if (a && b) (void)hipEventRecord(a, s);
    }
    hipError_t e = launch();
    if (p->prof && a && b) {
      (void)hipEventRecord(b, s);
      p->recs.push_back({id, a, b});
    }
    if (e != hipSuccess) {
      p->last_hip = (int)e;
      rc = HOT_E_HIP;
    }
  }
};

// One evaluation of the right-hand side from compact state `src` into Nh.
void rhs_passes(Runner& r, const Inst& I, const char* src, char* A1, char* A2, char* Nh) {
  const Geo& g = I.g;
  const long N = g.N, M = g.M, P = g.Mzp;
  const Ops& o = I.ops;
  r.pass(PASS_X_INV_CURL, [&] { return o.x_inv_curl(r.s, src, I.C, A1, I.D1, g); });
  // y inverse: 6 components, batch over x, rows ky (compact) -> y (all N)
  r.pass(PASS_Y_INV, [&] {
    return o.strided(r.s, +1, true, false, A1, A2, N * P, P, P, P, M * P, N * P, I.D1, I.D2, 6, g);
  });
  r.pass(PASS_Z_CROSS, [&] { return o.z_cross(r.s, A2, I.D2, N * N, g); });
  // y forward: 3 components, y (all N) -> ky (compact)
  r.pass(PASS_Y_FWD, [&] {
    return o.strided(r.s, -1, false, true, A2, A1, N * P, P, P, P, N * P, M * P, I.D2, I.D1, 3, g);
  });
  // x forward: rows x (all N) -> kx (compact), columns (ky, kz)
  r.pass(PASS_X_FWD, [&] {
    const long Q = M * P;
    return o.strided(r.s, -1, false, true, A1, Nh, Q, Q, Q, Q, 0, 0, I.D1, I.C, 3, g);
  });
}

}  // namespace

extern "C" int hot_run(hot_plan_t p, void* const* in, void* const* out, void* workspace, int32_t nsteps,
                       void* stream) {
  if (!p || !in || !out || nsteps < 0) return HOT_E_INVALID;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return HOT_E_WORKSPACE;
  for (size_t i = 0; i < p->inst.size(); ++i) {
    if (!in[i] || !out[i]) return HOT_E_INVALID;
    if (((uintptr_t)in[i] % kAlign) != 0 || ((uintptr_t)out[i] % kAlign) != 0) return HOT_E_INVALID;
  }
  Runner r{p, (hipStream_t)stream};
  char* ws = (char*)workspace;
  const size_t e = p->elem;
  for (size_t i = 0; i < p->inst.size() && r.rc == HOT_OK; ++i) {
    const Inst& I = p->inst[i];
    const Geo& g = I.g;
    const Ops& o = I.ops;
    const long N = g.N;
    if (p->op == HOT_OP_R2C || p->op == HOT_OP_C2R) {
      char* Z1 = ws;
      char* Z2 = ws + align_up(3 * (size_t)I.D2 * e);
      const long Nh = g.Mz, D2 = I.D2;
      if (p->op == HOT_OP_R2C) {
        r.pass(PASS_Z_R2C, [&] { return o.z_r2c(r.s, in[i], Z1, 3 * N * N, g); });
        r.pass(PASS_Y_FWD, [&] {
          return o.strided(r.s, -1, false, false, Z1, Z2, N * Nh, Nh, Nh, Nh, N * Nh, N * Nh, D2, D2, 3, g);
        });
        r.pass(PASS_X_FWD, [&] {
          const long Q = N * Nh;
          return o.strided(r.s, -1, false, false, Z2, out[i], Q, Q, Q, Q, 0, 0, D2, D2, 3, g);
        });
      } else {
        r.pass(PASS_X_INV, [&] {
          const long Q = N * Nh;
          return o.strided(r.s, +1, false, false, in[i], Z1, Q, Q, Q, Q, 0, 0, D2, D2, 3, g);
        });
        r.pass(PASS_Y_INV, [&] {
          return o.strided(r.s, +1, false, false, Z1, Z2, N * Nh, Nh, Nh, Nh, N * Nh, N * Nh, D2, D2, 3, g);
        });
        r.pass(PASS_Z_C2R, [&] { return o.z_c2r(r.s, Z2, out[i], 3 * N * N, g); });
      }
      continue;
    }
    const size_t sC = align_up(3 * (size_t)I.C * e);
    char* U0 = ws;
    char* U1 = U0 + sC;
    char* Acc = U1 + sC;
    char* Nh = Acc + sC;
    char* A1 = Nh + sC;
    char* A2 = A1 + align_up(6 * (size_t)I.D1 * e);
    r.pass(PASS_GATHER, [&] { return o.gather(r.s, in[i], U0, I.C, g); });
    if (p->op == HOT_OP_RHS) {
      rhs_passes(r, I, U0, A1, A2, Nh);
      r.pass(PASS_RK_STAGE, [&] { return o.rk_stage(r.s, Nh, U0, U1, Acc, I.C, g, 4, p->nu, p->dt); });
      r.pass(PASS_SCATTER, [&] { return o.scatter(r.s, Acc, out[i], I.C, g); });
    } else {
      for (int step = 0; step < nsteps && r.rc == HOT_OK; ++step) {
        for (int st = 0; st < 4; ++st) {
          rhs_passes(r, I, st == 0 ? U0 : U1, A1, A2, Nh);
          r.pass(PASS_RK_STAGE, [&] { return o.rk_stage(r.s, Nh, U0, U1, Acc, I.C, g, st, p->nu, p->dt); });
        }
      }
      r.pass(PASS_SCATTER, [&] { return o.scatter(r.s, U0, out[i], I.C, g); });
    }
  }
  return r.rc;
}
