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

}  // namespace hyb
