// Device FFT core for gfx950: complex type, compile-time roots of unity,
// in-register small DFTs and a Stockham line engine that exchanges through LDS.
//
// A line of length N is held by Tl = N/R threads, R complex values each.
// Thread j always holds positions j + s*Tl (s = 0..R-1) on entry and on exit,
// in natural order, so a pass loads and stores lines with the same pattern.
// Stage k of radix r (span Ns = product of earlier radices) runs N/r virtual
// butterflies; real thread j runs jj = j + m*Tl for m < R/r.  Butterfly jj
// reads positions jj + q*N/r, scales by w^((jj mod Ns) q / (Ns r)), does an
// r-point DFT and writes positions (jj/Ns)*Ns*r + (jj mod Ns) + q*Ns
// (the self-sorting Stockham order), so no bit reversal is needed.
//
// Transform sign: DIR = -1 is the forward transform exp(-i k.x) of Eq. ffteq,
// DIR = +1 the inverse (unnormalised; callers apply 1/N^3 once).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace hot {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
// multiply by i
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }

// ---------------------------------------------------------------------------
// compile-time roots of unity
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series on |x| <= pi/4 (terms decay below 1e-20 after n = 12).
constexpr double ct_sin(double x) {
  double x2 = x * x, t = x, s = x;
  for (int n = 1; n <= 12; ++n) {
    t = -t * x2 / double((2 * n) * (2 * n + 1));
    s += t;
  }
  return s;
}
constexpr double ct_cos(double x) {
  double x2 = x * x, t = 1.0, s = 1.0;
  for (int n = 1; n <= 12; ++n) {
    t = -t * x2 / double((2 * n - 1) * (2 * n));
    s += t;
  }
  return s;
}

struct cs_pair {
  double c, s;
};

// cos and sin of 2*pi*m/n; the quadrant and the half-quadrant fold are done in
// integers so the series only ever sees an angle in [0, pi/4].
constexpr cs_pair unit_root(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n;   // quadrant
  const long r = 4 * m - q * n; // remainder, angle within quadrant = (pi/2) r/n
  double c0 = 0, s0 = 0;
  if (2 * r <= n) {
    const double a = (kPi / 2) * double(r) / double(n);
    c0 = ct_cos(a);
    s0 = ct_sin(a);
  } else {
    const double a = (kPi / 2) * double(n - r) / double(n);
    c0 = ct_sin(a);
    s0 = ct_cos(a);
  }
  switch (q) {
    case 0: return {c0, s0};
    case 1: return {-s0, c0};
    case 2: return {-c0, -s0};
    default: return {s0, -c0};
  }
}

// ---------------------------------------------------------------------------
// compile-time loops
// ---------------------------------------------------------------------------
template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}

// v * exp(DIR * 2 pi i E / R) with E, R compile-time; trivial angles are
// special-cased so no multiply by an exact 0 or 1 is emitted.
template <int E, int R, int DIR, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> v) {
  constexpr int e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (2 * e == R) {
    return {-v.x, -v.y};
  } else if constexpr (4 * e == R) {  // exp(DIR i pi/2) = DIR i
    return DIR > 0 ? cx<T>{-v.y, v.x} : cx<T>{v.y, -v.x};
  } else if constexpr (4 * e == 3 * R) {  // exp(DIR i 3pi/2) = -DIR i
    return DIR > 0 ? cx<T>{v.y, -v.x} : cx<T>{-v.y, v.x};
  } else {
    constexpr cs_pair w = unit_root(e, R);
    constexpr T c = T(w.c);
    constexpr T s = T(DIR * w.s);
    return {v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// ---------------------------------------------------------------------------
// in-register DFT of compile-time size R (natural order in and out)
// ---------------------------------------------------------------------------
template <int R, int DIR, typename T>
struct Dft;

template <int DIR, typename T>
struct Dft<1, DIR, T> {
  __device__ __forceinline__ static void run(cx<T>*) {}
};

template <int DIR, typename T>
struct Dft<2, DIR, T> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const cx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  }
};

template <int DIR, typename T>
struct Dft<3, DIR, T> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    // X0 = a0+a1+a2; X1,2 = a0 - (a1+a2)/2 +- DIR i (sqrt3/2)(a1-a2)
    constexpr T h = T(0.86602540378443864676372317075293618);
    const cx<T> s = a[1] + a[2];
    const cx<T> d = a[1] - a[2];
    const cx<T> m = {a[0].x - T(0.5) * s.x, a[0].y - T(0.5) * s.y};
    const cx<T> id = DIR > 0 ? cx<T>{-d.y * h, d.x * h} : cx<T>{d.y * h, -d.x * h};
    a[0] = a[0] + s;
    a[1] = m + id;
    a[2] = m - id;
  }
};

template <int DIR, typename T>
struct Dft<4, DIR, T> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const cx<T> s0 = a[0] + a[2], d0 = a[0] - a[2];
    const cx<T> s1 = a[1] + a[3], d1 = a[1] - a[3];
    const cx<T> jd1 = rot<1, 4, DIR>(d1);
    a[0] = s0 + s1;
    a[2] = s0 - s1;
    a[1] = d0 + jd1;
    a[3] = d0 - jd1;
  }
};

template <int R>
constexpr int first_factor() {
  if constexpr (R % 4 == 0 && R != 4) return 4;
  else if constexpr (R % 2 == 0) return 2;
  else if constexpr (R % 3 == 0) return 3;
  else return R;
}

// Composite R = P*Q: n = Q n1 + n2, k = k1 + P k2,
// X[k1 + P k2] = sum_n2 W_R^(n2 k1) W_Q^(n2 k2) sum_n1 x[Q n1 + n2] W_P^(n1 k1).
template <int R, int DIR, typename T>
struct Dft {
  static constexpr int P = first_factor<R>();
  static constexpr int Q = R / P;
  static_assert(P > 1 && Q > 1, "unsupported DFT size");
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> y[R];
    static_for<0, Q>([&](auto n2) {
      cx<T> b[P];
      static_for<0, P>([&](auto n1) { b[n1] = a[Q * n1 + n2]; });
      Dft<P, DIR, T>::run(b);
      static_for<0, P>([&](auto k1) { y[n2 * P + k1] = rot<n2 * k1, R, DIR>(b[k1]); });
    });
    static_for<0, P>([&](auto k1) {
      cx<T> c[Q];
      static_for<0, Q>([&](auto n2) { c[n2] = y[n2 * P + k1]; });
      Dft<Q, DIR, T>::run(c);
      static_for<0, Q>([&](auto k2) { a[k1 + P * k2] = c[k2]; });
    });
  }
};

// Stage twiddle for DIR: forward multiplies by w, inverse by conj(w).
template <int DIR, typename T>
__device__ __forceinline__ cx<T> twmul(cx<T> v, cx<T> w) {
  return DIR < 0 ? cmul(v, w) : cmulc(v, w);
}

// Stage twiddles in stage-major order.  For stage k >= 1 (0-based) with span
// Ns and radix r, entry off_k + (q-1)*Ns + b holds exp(-2 pi i b q / (Ns r))
// for q in [1, r) and butterfly residue b in [0, Ns); off_k = sum over the
// earlier stages k' >= 1 of (r_k' - 1) Ns_k'.  Neighbouring butterflies read
// neighbouring entries, so the loads coalesce and LDS reads do not conflict.
// The table has N - r_0 entries (padded to N).
template <typename T, int N>
struct StageTw {
  cx<T> w[N];
};

template <typename T, int N, int... Rs>
constexpr StageTw<T, N> make_stage_tw() {
  StageTw<T, N> t{};
  constexpr int rr[] = {Rs...};
  long Ns = rr[0];
  int off = 0;
  for (int k = 1; k < (int)sizeof...(Rs); ++k) {
    const int r = rr[k];
    for (int q = 1; q < r; ++q)
      for (long b = 0; b < Ns; ++b) {
        const cs_pair p = unit_root(b * q, Ns * r);
        t.w[off + (q - 1) * Ns + b].x = T(p.c);
        t.w[off + (q - 1) * Ns + b].y = T(-p.s);
      }
    off += (r - 1) * (int)Ns;
    Ns *= r;
  }
  return t;
}

// Twiddle source: operator()(i) returns entry i of the stage-major table.
template <typename T>
struct TwTab {
  const cx<T>* tab;
  __device__ __forceinline__ cx<T> operator()(int i) const { return tab[i]; }
};

// ---------------------------------------------------------------------------
// Stockham engine
// ---------------------------------------------------------------------------
// Lds must provide put(pos, v), get(pos) for this thread's line and sync().
template <typename T, int DIR, int N, int R, int Ns, int OFF, int... Rs>
struct Stages;

template <typename T, int DIR, int N, int R, int Ns, int OFF>
struct Stages<T, DIR, N, R, Ns, OFF> {
  template <class L, class TW>
  __device__ __forceinline__ static void run(cx<T>*, int, L&, const TW&) {
    static_assert(Ns == N, "radices must multiply to N");
  }
};

template <typename T, int DIR, int N, int R, int Ns, int OFF, int r, int... Rs>
struct Stages<T, DIR, N, R, Ns, OFF, r, Rs...> {
  static constexpr int Tl = N / R;
  static constexpr int nb = R / r;
  static constexpr bool last = (Ns * r == N);
  static constexpr int NEXT_OFF = Ns > 1 ? OFF + (r - 1) * Ns : OFF;
  static_assert(R % r == 0, "each radix must divide the per-thread count");

  // Butterfly jj = j + m Tl (0 <= j < Tl) splits as jj = blk Ns + res.  With
  // Tl and Ns compile-time, most splits need no division: when the m-th
  // range [m Tl, (m+1) Tl) lies inside one Ns-block, blk is a constant and
  // res = j + constant; when Ns divides Tl, res = j mod Ns for every m and
  // blk = j / Ns + m Tl / Ns, split once per stage.  (Divisions by the
  // constant non-powers of two of the radix-6 and radix-3 lengths cost about
  // as much as their butterflies.)
  template <int m>
  static constexpr bool in_one_block() {
    return (m * Tl) / Ns == (m * Tl + Tl - 1) / Ns;
  }
  template <class L, class TW>
  __device__ __forceinline__ static void run(cx<T>* v, int j, L& lds, const TW& tw) {
    constexpr bool hoist = Ns > 1 && Tl % Ns == 0;
    const int j_blk = hoist ? j / Ns : 0;
    const int j_res = hoist ? j - j_blk * Ns : 0;
    static_for<0, nb>([&](auto m) {
      const int jj = j + m * Tl;
      int blk, res;
      if constexpr (Ns == 1) {
        blk = jj;
        res = 0;
      } else if constexpr (in_one_block<decltype(m)::value>()) {
        constexpr int b0 = (decltype(m)::value * Tl) / Ns;
        blk = b0;
        res = jj - b0 * Ns;
      } else if constexpr (hoist) {
        blk = j_blk + m * (Tl / Ns);
        res = j_res;
      } else {
        blk = jj / Ns;
        res = jj - blk * Ns;
      }
      cx<T> b[r];
      static_for<0, r>([&](auto q) { b[q] = v[m + q * nb]; });
      if constexpr (Ns > 1) {
        static_for<1, r>([&](auto q) { b[q] = twmul<DIR>(b[q], tw(OFF + (q - 1) * Ns + res)); });
      }
      Dft<r, DIR, T>::run(b);
      if constexpr (!last) {
        const int ob = blk * (Ns * r) + res;
        static_for<0, r>([&](auto q) { lds.put(ob + q * Ns, b[q]); });
      } else {
        static_for<0, r>([&](auto q) { v[m + q * nb] = b[q]; });
      }
    });
    if constexpr (!last) {
      lds.sync();
      static_for<0, R>([&](auto s) { v[s] = lds.get(j + s * Tl); });
      lds.sync();
      Stages<T, DIR, N, R, Ns * r, NEXT_OFF, Rs...>::run(v, j, lds, tw);
    }
  }
};

template <int V>
constexpr int ilog2() {
  int k = 0;
  while ((1 << (k + 1)) <= V) ++k;
  return k;
}

template <int First, int... Rest>
struct FirstOf {
  static constexpr int value = First;
};

// A line-length plan: N points, R per thread, radix sequence.
template <int N_, int R_, int... Rs>
struct LinePlan {
  static constexpr int N = N_;
  static constexpr int R = R_;
  static constexpr int Tl = N_ / R_;
  // First-stage writes go to positions r1 apart (r1 = first radix); the LDS
  // line view spreads them over the banks (an XOR swizzle for r1 >= 16, one
  // padding slot every 2^SH positions below).
  static constexpr int SH = ilog2<FirstOf<Rs...>::value>();
  static constexpr int line_slots = SH >= 4 ? N_ : N_ + (N_ >> SH) + 1;
  // distance between the LDS regions of two lines held by one wave
  static constexpr int line_stride = line_slots;
  template <typename T>
  static constexpr StageTw<T, N_> twiddles() {
    return make_stage_tw<T, N_, Rs...>();
  }
  template <typename T, int DIR, class L, class TW>
  __device__ __forceinline__ static void fft(cx<T>* v, int j, L& lds, const TW& tw) {
    Stages<T, DIR, N_, R_, 1, 0, Rs...>::run(v, j, lds, tw);
  }
};

// A plan whose lines sit S slots apart in LDS instead of line_slots, so that
// the lines of one wave fall on different LDS banks.
template <class Plan, int S>
struct StridedLines : Plan {
  static_assert(S >= Plan::line_slots, "lines would overlap");
  static constexpr int line_stride = S;
};

// Stage-major twiddles of a plan, in device memory.
template <typename T, class Plan>
__device__ const StageTw<T, Plan::N> g_stage_tw = Plan::template twiddles<T>();

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace hot
