// The y and z passes of a right-hand side fused into one kernel, for sizes
// whose six (y, kz) planes of one x-plane fit in LDS.  One block owns one
// x-plane of one instance:
//   load   A[6][x][M rows (ky)][Mzp] (compact rows) -> P[6][N][Mz] in LDS
//          (row pitch Mz | 1: an odd pitch spreads a column over the banks);
//          the rows outside the retained set are read as zeros
//   y      inverse transform of every (component, kz) column, in place
//   z      per y line: the z pass (u and omega packed in three complex
//          lines read straight from P, inverse transforms, u x omega, forward
//          transforms; u and omega carry the 1/N^3 already), components 0..2
//          of the row written back
//   y      forward transform of every (component 0..2, kz) column, in place
//   store  the retained rows of components 0..2 -> A[3][x][M][Mzp]
// So the (x, y, kz) intermediate never goes to HBM: per x-plane the block
// reads 6 M Mz and writes 3 M Mz values.  The transforms use the plans,
// twiddles and arithmetic of the separate passes; the compiler may still
// contract multiplies and adds differently in the two kernels, so the results
// agree to rounding.  In place on A: a block reads and writes only its own
// x-plane.
#pragma once

#include "kernels.hpp"

namespace hot {

// Stockham exchange view over one column of P (positions `stride` apart);
// the column's lanes sit in one wave.
template <typename T>
struct LdsColumn {
  cx<T>* base;
  int stride;
  __device__ __forceinline__ void put(int pos, cx<T> v) { base[pos * stride] = v; }
  __device__ __forceinline__ cx<T> get(int pos) const { return base[pos * stride]; }
  __device__ __forceinline__ void sync() { wave_sync(); }
};

// Block shape: enough waves for all N z lines of the plane in one round
// (at most 8), so that the lanes stay busy at every size; NWF > 0 sets the
// number of waves instead (the persistent batch kernel's block).
template <typename T, class Plan, int NWF = 0>
struct YzShape {
  static constexpr int N = Plan::N, Tl = Plan::Tl;
  static constexpr int LPW = Tl <= 64 ? 64 / Tl : 1;  // lines per wave (leftover lanes idle)
  static constexpr int NW = NWF > 0 ? NWF : ((N + LPW - 1) / LPW < 8 ? (N + LPW - 1) / LPW : 8);
  static constexpr int NT = 64 * NW;
  static constexpr int LPR = NW * LPW;  // lines per round
  static constexpr int ZL = LPR < N ? LPR : N;  // z lines in flight (exchange slots)
  static constexpr int MZ = (N - 1) / 3 + 1 > N / 2 ? (N - 1) / 3 + 1 : N / 2;  // widest Mz (no dealiasing)
  static constexpr int pitch(int Mz) { return Mz | 1; }
  static constexpr long lds_bytes(int Mz) {
    return (long)sizeof(cx<T>) * (6L * N * pitch(Mz) + (long)ZL * Plan::line_stride + N);
  }
  // the fused pass exists when a line sits in one wave and the widest
  // retained z extent fits
  static constexpr bool kFits = Tl <= 64 && lds_bytes(MZ) <= 163840;
};

// x-plane x of instance `inst`, run by the S::NT threads of a block (tid)
// with S::lds_bytes(g.Mz) of LDS at sm.  G23: the caller has checked that g
// is the 2/3-rule geometry of N.  k_yz_fused runs one plane per block; the
// persistent batch kernel calls it for its work items.
template <typename T, class Plan, int KL, bool G23, int NWF = 0>
__device__ __forceinline__ void yz_fused_plane(cx<T>* __restrict__ A, long csA, long isA, const Geo& g_in, long x,
                                               int inst, int tid, cx<T>* sm) {
  const Geo g = G23 ? geo_two_thirds<Plan::N>(g_in) : g_in;
  using S = YzShape<T, Plan, NWF>;
  constexpr int N = Plan::N, R = Plan::R, Tl = Plan::Tl, LS = Plan::line_stride;
  constexpr int NT = S::NT;
  const int Mz = g.Mz, M = g.M;
  const int Ps = S::pitch(Mz);         // row pitch of P
  const long cs = (long)N * Ps;        // component stride of P
  cx<T>* P = sm;                       // [6][N][Ps]
  cx<T>* X = P + 6 * cs;               // z-line exchange slots [ZL][LS]
  cx<T>* tws = X + (long)S::ZL * LS;   // stage twiddles [N]
  const int w = tid >> 6, lane = tid & 63;
  const bool lane_live = lane / Tl < S::LPW;
  const int lslot = w * S::LPW + lane / Tl;  // line of this lane within a round
  const int j = lane % Tl;
  A += inst * isA;
  const long plane = (long)M * g.Mzp;  // one x-plane of one component
  TwStage<T, Plan, NT> twst;
  twst.fetch(tid);
  // load: the retained rows of the six components into their rows of P.  A
  // thread keeps one kz and walks the (component, compact row) pairs a
  // block-size step apart, twelve loads in flight at a time; the rows of P
  // outside the retained set are never written here, and the y inverse
  // takes them as zeros.
  {
    constexpr int B = 12;
    const int q = NT / Mz;  // rows one pass of the block covers
    const int kz = tid - (tid / Mz) * Mz;
    const int rho = tid / Mz;
    const int qc = q / M, qm = q - (q / M) * M;
    int c = rho / M, ky = rho - (rho / M) * M;
    for (int r0 = rho; rho < q && r0 < 6 * M; r0 += B * q) {
      cx<T> ld[B];
      int at[B];
      static_for<0, B>([&](auto i) {
        const bool in = c < 6;
        ld[i] = A[in ? c * csA + x * plane + (long)ky * g.Mzp + kz : 0];
        at[i] = in ? c * (int)cs + cpos(ky, g) * Ps + kz : -1;
        ky += qm;
        c += qc;
        if (ky >= M) {
          ky -= M;
          ++c;
        }
      });
      static_for<0, B>([&](auto i) {
        if (at[i] >= 0) P[at[i]] = ld[i];
      });
    }
  }
  twst.put(tws, tid);
  __syncthreads();
  const TwTab<T> tw{tws};
  // y inverse: every (component, kz) column
  for (int base = 0; base < 6 * Mz; base += S::LPR) {
    const int id = base + lslot;
    if (lane_live && id < 6 * Mz) {
      const int c = id / Mz, kz = id - c * Mz;
      LdsColumn<T> col{P + c * cs + kz, Ps};
      cx<T> v[R];
      static_for<0, R>([&](auto s) {
        const int p = j + s * Tl;
        const cx<T> t = col.get(p);  // rows outside the retained set hold no data
        v[s] = kept(p, g) ? t : cx<T>{T(0), T(0)};
      });
      col.sync();
      Plan::template fft<T, +1>(v, j, col, tw);
      static_for<0, R>([&](auto s) { col.put(j + s * Tl, v[s]); });
    }
  }
  __syncthreads();
  // z lines: the computation of k_z_cross with the coefficients in P
  for (int base = 0; base < N; base += S::ZL) {
    const int y = base + lslot;
    if (lane_live && lslot < S::ZL && y < N) {
      LdsLine<T, Plan::SH, false> lds{X + (long)lslot * LS};
      const cx<T>* row = P + (long)y * Ps;
      // each complex line packs two real ones, a + i b, straight from their
      // rows of P: Z_p = a_p + i b_p for p < Mz, Z_p = conj a_{N-p} + i conj
      // b_{N-p} for N - p < Mz (the Hermitian halves of the real lines), the
      // imaginary parts of a_0, b_0 (and of the Nyquist terms) dropped as a
      // real inverse transform does; registers that no coefficient reaches
      // (col_live) stay zero without a read
      cx<T> ph[3][R];
      static_for<0, 3>([&](auto pr) {
        const cx<T>* ra = row + (2 * pr) * cs;
        const cx<T>* rb = ra + cs;
        static_for<0, R>([&](auto s) {
          constexpr bool dead = s * Tl >= KL * Tl && (s + 1) * Tl - 1 <= N - KL * Tl;
          if constexpr (dead) {
            ph[pr][s] = cx<T>{T(0), T(0)};
          } else {
            const int p = j + s * Tl;
            const bool lo = p < Mz, hi = !lo && N - p < Mz;
            const int k = lo ? p : (hi ? N - p : 0);
            cx<T> a = ra[k], b = rb[k];
            if (k == 0 || 2 * k == N) {
              a.y = T(0);
              b.y = T(0);
            }
            ph[pr][s] = lo ? cx<T>{a.x - b.y, a.y + b.x}
                           : (hi ? cx<T>{a.x + b.y, b.x - a.y} : cx<T>{T(0), T(0)});
          }
        });
        Plan::template fft<T, +1>(ph[pr], j, lds, tw);
      });
      cx<T> z01[R], z2[R];
      static_for<0, R>([&](auto s) {
        const T u0 = ph[0][s].x, u1 = ph[0][s].y, u2 = ph[1][s].x;
        const T w0 = ph[1][s].y, w1 = ph[2][s].x, w2 = ph[2][s].y;
        z01[s] = {u1 * w2 - u2 * w1, u2 * w0 - u0 * w2};
        z2[s] = {u0 * w1 - u1 * w0, T(0)};
      });
      Plan::template fft<T, -1>(z2, j, lds, tw);
      Plan::template fft<T, -1>(z01, j, lds, tw);
      static_for<0, R>([&](auto s) { lds.put(j + s * Tl, z01[s]); });
      lds.sync();
      cx<T>* o = P + (long)y * Ps;
      static_for<0, R>([&](auto s) {
        const int k = j + s * Tl;
        if (k < Mz) {
          const cx<T> zk = lds.get(k);
          const cx<T> zm = lds.get((N - k) % N);
          o[k] = cx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
          o[cs + k] = cx<T>{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
          o[2 * cs + k] = z2[s];
        }
      });
      lds.sync();  // the slot's next line overwrites the exchange region
    }
  }
  __syncthreads();
  // y forward: components 0..2
  for (int base = 0; base < 3 * Mz; base += S::LPR) {
    const int id = base + lslot;
    if (lane_live && id < 3 * Mz) {
      const int c = id / Mz, kz = id - c * Mz;
      LdsColumn<T> col{P + c * cs + kz, Ps};
      cx<T> v[R];
      static_for<0, R>([&](auto s) { v[s] = col.get(j + s * Tl); });
      col.sync();
      Plan::template fft<T, -1>(v, j, col, tw);
      static_for<0, R>([&](auto s) { col.put(j + s * Tl, v[s]); });
    }
  }
  __syncthreads();
  // store the retained rows of components 0..2 ([3][M][Mz], stepped as the
  // load)
  {
    const int sq = NT / Mz, sr = NT - (NT / Mz) * Mz;
    int kz = tid - (tid / Mz) * Mz, ky = tid / Mz, c = ky / M;
    ky -= c * M;
    while (c < 3) {
      A[c * csA + x * plane + (long)ky * g.Mzp + kz] = P[c * cs + (long)cpos(ky, g) * Ps + kz];
      kz += sr;
      ky += sq;
      if (kz >= Mz) {
        kz -= Mz;
        ++ky;
      }
      while (ky >= M) {
        ky -= M;
        ++c;
      }
    }
  }
}

template <typename T, class Plan, int KL, bool G23>
__global__ __launch_bounds__((YzShape<T, Plan>::NT)) void k_yz_fused(cx<T>* __restrict__ A, long csA, long isA,
                                                  Geo g_in, const int* __restrict__ act) {
  if (act && !act[blockIdx.y]) return;  // instance no longer iterating
  extern __shared__ unsigned char smem_raw[];
  yz_fused_plane<T, Plan, KL, G23>(A, csA, isA, g_in, blockIdx.x, blockIdx.y, threadIdx.x,
                                   reinterpret_cast<cx<T>*>(smem_raw));
}

}  // namespace hot
