// FP64 matrix-core building blocks (gfx950, v_mfma_f64_16x16x4f64).
#pragma once

#include "kernels_common.hpp"

namespace hyb {

typedef double dx4 __attribute__((ext_vector_type(4)));

// D = A B + C for a 16 x 4 block A and a 4 x 16 block B on one wave: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; element r of lane l's
// result is D[l / 16 + 4 r][l % 16] (layout measured on the device).
__device__ __forceinline__ dx4 mfma16x16x4(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef float fx4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core step D = A B + C on one wave for FP32 and FP64:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; element r of
// lane l's result is D[row(l, r)][l % 16] (both layouts measured on the
// device: FP32 rows 4 (l / 16) + r, FP64 rows l / 16 + 4 r).
template <class T>
struct MfmaT;
template <>
struct MfmaT<float> {
  using v4 = fx4;
  __device__ static v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct MfmaT<double> {
  using v4 = dx4;
  __device__ static v4 op(double a, double b, v4 c) { return mfma16x16x4(a, b, c); }
  __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// Makes the wave's earlier LDS and global stores visible to its later loads
// (other lanes of the same wave) without a block barrier: work that one wave
// owns.  Workgroup-scope fences wait for the stores to complete.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// index of the symmetric 3x3 pair (d, e) in (00, 01, 02, 11, 12, 22)
__device__ __forceinline__ int gidx(int d, int e) {
  int lo = d < e ? d : e, hi = d < e ? e : d;
  return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
}

// Quadrature points per staging chunk of assemble_mfma (where LDS allows):
// the team copies the basis values and divergences of QC points (2 n QC
// doubles) into LDS at once.
constexpr int kAsmQC = 16;

// Element matrix M_T by Gauss quadrature on the FP64 matrix cores.  With the
// per-point terms of element_qd (qd: 6 metric weights w alpha (J^T J)_de /
// det J, the div-div weight w beta / det J), tile (I, J) of M_T is the sum
// over the points q of A_q B_q with
//   A_q[i][c] = phi_i(q) if comp(i) = c (c < 3),  div phi_i(q) (c = 3),
//   B_q[c][j] = G_{c, comp(j)}(q) phi_j(q)        (c < 3),
//               w_div(q) div phi_j(q)            (c = 3),
// one MFMA per tile and point (rows and columns past n are zero).  The team's
// waves share out the lower tiles, G at a time (every wave runs the same
// number of groups, so the staging barriers match); the tables of QC points
// at a time come through LDS (stage: 2 n QC doubles).
// store(i, j, v) receives every entry with j <= i < n.
template <int K, int TEAM, int QC, class Store>
__device__ __forceinline__ void assemble_mfma(const DeviceMaps& mp, const double* qd, double* stage, int lane,
                                              Store store) {
  using R = RT<K>;
  constexpr int n = R::n, Q = R::Q, QD = 10, NT = (n + 15) / 16, NTILE = NT * (NT + 1) / 2;
  constexpr int NW = TEAM / 64, G = 4, NGROUP = (NTILE + NW * G - 1) / (NW * G);
  static_assert(QC >= 1, "at least one point per chunk");
  static_assert(TEAM % 64 == 0, "whole waves per team");
  const int w = lane / 64, l = lane % 64, li = l % 16, lc = l / 16;
  for (int grp = 0; grp < NGROUP; ++grp) {
    const int t0 = w + grp * NW * G;
    int ti[G], tj[G];
    bool on[G];
    dx4 acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int t = t0 + g * NW;
      on[g] = t < NTILE;
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      ti[g] = I;
      tj[g] = t - I * (I + 1) / 2;
      acc[g] = dx4{0.0, 0.0, 0.0, 0.0};
    }
    for (int q0 = 0; q0 < Q; q0 += QC) {
      const int nq = Q - q0 < QC ? Q - q0 : QC;
      __syncthreads();  // the previous chunk is consumed
      for (int t = lane; t < nq * n; t += TEAM) {
        stage[t] = mp.tab_s[q0 * n + t];
        stage[QC * n + t] = mp.tab_d[q0 * n + t];
      }
      __syncthreads();
      for (int qq = 0; qq < nq; ++qq) {
        const double* ts = stage + qq * n;
        const double* td = stage + QC * n + qq * n;
        const double* wq = qd + (q0 + qq) * QD;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (!on[g]) continue;  // uniform across the wave
          const int i = 16 * ti[g] + li, j = 16 * tj[g] + li;
          // one table load per operand (the LDS bandwidth bounds this loop;
          // loading both tables at clamped indices measured 1.5x slower)
          double a = 0.0, b = 0.0;
          if (i < n) a = lc < 3 ? (R::comp(i) == lc ? ts[i] : 0.0) : td[i];
          if (j < n) b = lc < 3 ? wq[gidx(lc, R::comp(j))] * ts[j] : wq[6] * td[j];
          acc[g] = mfma16x16x4(a, b, acc[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (!on[g]) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * ti[g] + lc + 4 * r, j = 16 * tj[g] + li;
        if (i < n && j <= i) store(i, j, acc[g][r]);
      }
    }
  }
}

// Local index (interior dofs first, then faces) of the component-d basis
// function whose 1D factors along axes 0, 1, 2 have indices a0, a1, a2 (the
// closed index along axis d, the open ones along the two other axes in
// increasing order).
template <int K>
__device__ __forceinline__ int dof_index(int d, int a0, int a1, int a2) {
  using R = RT<K>;
  const int ic = d == 0 ? a0 : (d == 1 ? a1 : a2);
  const int j0 = d == 0 ? a1 : a0, j1 = d == 2 ? a1 : a2;
  if (ic >= 1 && ic <= K) return d * K * R::K2 + (j1 * R::K1 + j0) * K + (ic - 1);
  return R::ni + (2 * d + (ic == 0 ? 0 : 1)) * R::K2 + j0 + R::K1 * j1;
}

// Whether the element assembly of order k uses sum factorization.  It needs
// about 1.1 Mflop per RT3 element against 14.4 for the dense Gram sum on the
// matrix cores and is then much faster (measured 50 against about 370 us per
// element in a workgroup); for k <= 2 the saving is small in absolute terms
// (0.17 against 1.49 Mflop for RT2) and the dense sum's independent tiles hide
// latency better than the sum factorization's 18 barrier-separated passes
// (RT2 48^3 setup 37.5 ms dense against 49.9 ms factored).
template <int K>
constexpr bool use_sumfact() { return K >= 3; }

// LDS doubles used by assemble_sumfact: the 1D tables, then the axis-0 and
// axis-1 partial sums of both terms.
template <int K>
constexpr int sumfact_tables() {
  return (2 * (K + 2) + (K + 1)) * (K + 2);
}
template <int K>
constexpr int sumfact_stage() {
  constexpr int KC = K + 2, K1 = K + 1, q1 = K + 2;
  return sumfact_tables<K>() + 2 * (KC * KC * q1 * q1 + KC * KC * K1 * K1 * q1);
}

// Element matrix M_T by sum factorization (k >= 1, any trilinear element).
// The basis is a tensor product (per component d: the closed Lagrange factor
// along axis d, open ones along the other two) and the Gauss rule is a
// tensor rule, so block (d, e) of M_T,
//   sum_q G_de(q) prod_x A_x[a_x][q_x] B_x[b_x][q_x]
//     + w_div(q) prod_x A'_x[a_x][q_x] B'_x[b_x][q_x],
// (A, B: the 1D factors of components d and e, A', B' those of the
// divergences: derivatives of the closed factor on the own axis) is summed
// one axis at a time: over the points along axis 0 into S1[a0][b0][q1][q2],
// along axis 1 into S2[a0][b0][a1][b1][q2], along axis 2 into the entries.
// The per-point weights come from element_qd (qd: 6 metric weights
// w alpha (J^T J)_de / det J, the div-div weight w beta / det J).  Team-wide,
// three barriers per block of components; store(i, j, v) receives every
// entry with j <= i < n once.  stage: sumfact_stage<K>() doubles of LDS.
template <int K, int TEAM, class Store>
__device__ __forceinline__ void assemble_sumfact(const DeviceMaps& mp, const double* qd, double* stage, int lane,
                                                 Store store) {
  constexpr int KC = K + 2, K1 = K + 1, q1 = K + 2, QD = 10;
  static_assert(K >= 1, "sum factorization for k >= 1");
  // the 1D tables into LDS (read in every inner loop below)
  constexpr int TB = sumfact_tables<K>();
  __syncthreads();   // the team is done with the staging area
  for (int t = lane; t < TB; t += TEAM) stage[t] = mp.tab1d[t];
  const double* Lc = stage;             // [KC][q1]
  const double* Dc = Lc + KC * q1;      // [KC][q1]
  const double* Lo = Dc + KC * q1;      // [K1][q1]
  double* S1 = stage + TB;                             // [2][a0][b0][q1][q2]
  double* S2 = S1 + 2 * KC * KC * q1 * q1;             // [2][a0][b0][a1][b1][q2]
  constexpr int S1P = KC * KC * q1 * q1, S2P = KC * KC * K1 * K1 * q1;
  __syncthreads();
  for (int d = 0; d < 3; ++d) {
    for (int e = d; e < 3; ++e) {
      const int gi = gidx(d, e);
      // 1D factor of the own (x == c) or another axis; part 1: divergence
      auto fac = [&](int c, int part, int x, int a, int q) {
        return x == c ? (part ? Dc[a * q1 + q] : Lc[a * q1 + q]) : Lo[a * q1 + q];
      };
      const int pa0 = d == 0 ? KC : K1, pb0 = e == 0 ? KC : K1;
      const int pa1 = d == 1 ? KC : K1, pb1 = e == 1 ? KC : K1;
      const int pa2 = d == 2 ? KC : K1, pb2 = e == 2 ? KC : K1;
      // axis 0: task (part, q1 q2, a0)
      const int n1 = 2 * q1 * q1 * pa0;
      for (int t = lane; t < n1; t += TEAM) {
        const int part = t / (q1 * q1 * pa0), r = t % (q1 * q1 * pa0), a0 = r % pa0, qq = r / pa0;
        double aw[q1];
#pragma unroll
        for (int q0 = 0; q0 < q1; ++q0)
          aw[q0] = fac(d, part, 0, a0, q0) * qd[(q0 + q1 * qq) * QD + (part ? 6 : gi)];
        for (int b0 = 0; b0 < pb0; ++b0) {
          double s = 0.0;
#pragma unroll
          for (int q0 = 0; q0 < q1; ++q0) s += aw[q0] * fac(e, part, 0, b0, q0);
          S1[part * S1P + (a0 * pb0 + b0) * q1 * q1 + qq] = s;
        }
      }
      __syncthreads();
      // axis 1: task (part, a0 b0, q2, a1)
      const int n2 = 2 * pa0 * pb0 * q1 * pa1;
      for (int t = lane; t < n2; t += TEAM) {
        const int part = t / (pa0 * pb0 * q1 * pa1), r = t % (pa0 * pb0 * q1 * pa1);
        const int a1 = r % pa1, q2 = (r / pa1) % q1, ab0 = r / (pa1 * q1);
        double aw[q1];
#pragma unroll
        for (int qy = 0; qy < q1; ++qy)
          aw[qy] = fac(d, part, 1, a1, qy) * S1[part * S1P + ab0 * q1 * q1 + qy + q1 * q2];
        for (int b1 = 0; b1 < pb1; ++b1) {
          double s = 0.0;
#pragma unroll
          for (int qy = 0; qy < q1; ++qy) s += aw[qy] * fac(e, part, 1, b1, qy);
          S2[part * S2P + ((ab0 * pa1 + a1) * pb1 + b1) * q1 + q2] = s;
        }
      }
      __syncthreads();
      // axis 2: task (a0 b0 a1 b1, a2), both terms into the entries
      const int n3 = pa0 * pb0 * pa1 * pb1 * pa2;
      for (int t = lane; t < n3; t += TEAM) {
        const int a2 = t % pa2, r = t / pa2;
        const int b1 = r % pb1, a1 = (r / pb1) % pa1, b0 = (r / (pb1 * pa1)) % pb0, a0 = r / (pb1 * pa1 * pb0);
        double am[q1], ad[q1];
#pragma unroll
        for (int qz = 0; qz < q1; ++qz) {
          am[qz] = fac(d, 0, 2, a2, qz) * S2[r * q1 + qz];
          ad[qz] = fac(d, 1, 2, a2, qz) * S2[S2P + r * q1 + qz];
        }
        const int ia = dof_index<K>(d, a0, a1, a2);
        for (int b2 = 0; b2 < pb2; ++b2) {
          const int ib = dof_index<K>(e, b0, b1, b2);
          if (d == e && ib > ia) continue;
          double s = 0.0;
#pragma unroll
          for (int qz = 0; qz < q1; ++qz) s += am[qz] * fac(e, 0, 2, b2, qz) + ad[qz] * fac(e, 1, 2, b2, qz);
          if (ia >= ib) store(ia, ib, s); else store(ib, ia, s);
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace hyb
