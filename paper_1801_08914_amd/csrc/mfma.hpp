// FP64 matrix-core building blocks (gfx950, v_mfma_f64_16x16x4f64).
#pragma once

#include "kernels_common.hpp"

namespace hyb {

typedef double dx4 __attribute__((ext_vector_type(4)));
// a double in LDS (address space 3), for stores the compiler must not turn
// into flat ones
typedef __attribute__((address_space(3))) double lds_double;

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

// Whether the element assembly of order k uses sum factorization: about
// 1.1 Mflop per RT3 element and 0.17 per RT2 element against 14.4 and 1.49
// for the dense Gram sum on the matrix cores.  Measured per element and CU:
// RT2 45 against 59 us (at the single-plan register budget of 128, two
// workgroups per CU, which its kernels carry as a launch bound; with the
// compiler's 202 registers, one workgroup per CU, it lost: 65), RT1 9.6
// against 10.9.  RT0 keeps the per-entry sum.
template <int K>
constexpr bool use_sumfact() { return K >= 1; }

// The six component blocks (d, e), d <= e, of the sum-factorized assembly:
// (0,0) (0,1) (0,2) (1,1) (1,2) (2,2).  Component d has np(d, x) 1D factors
// along axis x (K + 2 closed ones on its own axis, K + 1 open ones on the
// others).  Pass 1 (axis 0) has, per block, a task per (part, point pair
// (q1, q2), a0) and writes S1[part][a0][b0][q1][q2]; pass 2 (axes 1 and 2)
// has a task per (a0, b0, a1, b1).  Offsets into the LDS partial sums and the
// task ranges are prefix sums over the blocks.
template <int K>
struct SfBlocks {
  static constexpr int KC = K + 2, K1 = K + 1, q1 = K + 2;
  static constexpr int d_of(int b) { return b < 3 ? 0 : (b < 5 ? 1 : 2); }
  static constexpr int e_of(int b) { return b < 3 ? b : (b < 5 ? b - 2 : 2); }
  static constexpr int np(int d, int x) { return d == x ? KC : K1; }
  static constexpr int s1_size(int b) { return 2 * np(d_of(b), 0) * np(e_of(b), 0) * q1 * q1; }
  static constexpr int t1_count(int b) { return 2 * q1 * q1 * np(d_of(b), 0); }
  static constexpr int t2_count(int b) {
    return np(d_of(b), 0) * np(e_of(b), 0) * np(d_of(b), 1) * np(e_of(b), 1);
  }
  static constexpr int s1_off(int b) { return b == 0 ? 0 : s1_off(b - 1) + s1_size(b - 1); }
  static constexpr int t1_off(int b) { return b == 0 ? 0 : t1_off(b - 1) + t1_count(b - 1); }
  static constexpr int t2_off(int b) { return b == 0 ? 0 : t2_off(b - 1) + t2_count(b - 1); }
};

// LDS doubles used by assemble_sumfact: the 1D tables, then the axis-0
// partial sums of both terms for all six blocks.
template <int K>
constexpr int sumfact_tables() {
  return (2 * (K + 2) + (K + 1)) * (K + 2);
}
template <int K>
constexpr int sumfact_stage() {
  return sumfact_tables<K>() + SfBlocks<K>::s1_off(6);
}

// 1D factor a at point q of component d along axis x: closed (x == d; the
// derivative for the divergence term, part 1) or open.  Tables in LDS:
// Lc[KC][q1], Dc[KC][q1], Lo[K1][q1].
template <int K>
struct SfTables {
  const double* Lc;
  const double* Dc;
  const double* Lo;
  __device__ double operator()(int d, int part, int x, int a, int q) const {
    constexpr int q1 = K + 2;
    return x == d ? (part ? Dc[a * q1 + q] : Lc[a * q1 + q]) : Lo[a * q1 + q];
  }
};

// Pass 1 task t of block B: S1[part][a0][b0][qq] = sum over the points q0
// along axis 0 of (A_0[a0][q0] w(q)) B_0[b0][q0], w the metric weight of
// (d, e) (part 0) or the div-div weight (part 1).
template <int K, int B>
__device__ __forceinline__ void sf_pass1(int t, const double* qd, SfTables<K> fac, double* S1) {
  using SB = SfBlocks<K>;
  constexpr int d = SB::d_of(B), e = SB::e_of(B), q1 = SB::q1, QD = 10;
  constexpr int pa0 = SB::np(d, 0), pb0 = SB::np(e, 0), S1P = pa0 * pb0 * q1 * q1;
  const int gi = gidx(d, e);
  const int part = t / (q1 * q1 * pa0), r = t % (q1 * q1 * pa0), a0 = r % pa0, qq = r / pa0;
  double aw[q1];
#pragma unroll
  for (int q0 = 0; q0 < q1; ++q0) aw[q0] = fac(d, part, 0, a0, q0) * qd[(q0 + q1 * qq) * QD + (part ? 6 : gi)];
  // every load before the first store (the tables and S1 share LDS)
  double res[pb0];
#pragma unroll
  for (int b0 = 0; b0 < pb0; ++b0) {
    double s = 0.0;
#pragma unroll
    for (int q0 = 0; q0 < q1; ++q0) s += aw[q0] * fac(e, part, 0, b0, q0);
    res[b0] = s;
  }
  double* out = S1 + SB::s1_off(B) + part * S1P + a0 * pb0 * q1 * q1 + qq;
#pragma unroll
  for (int b0 = 0; b0 < pb0; ++b0) out[b0 * q1 * q1] = res[b0];
}

// Pass 2 task t of block B, (a0, b0, a1, b1): both terms summed over the
// points along axis 1 into registers (S2[part][q2]), then over axis 2 into
// every entry (a2, b2) of the task (the lower triangle of a diagonal block).
template <int K, int B, class Store>
__device__ __forceinline__ void sf_pass2(int t, SfTables<K> fac, const double* S1, Store store) {
  using SB = SfBlocks<K>;
  constexpr int d = SB::d_of(B), e = SB::e_of(B), q1 = SB::q1;
  constexpr int pa0 = SB::np(d, 0), pb0 = SB::np(e, 0), pa1 = SB::np(d, 1), pb1 = SB::np(e, 1);
  constexpr int pa2 = SB::np(d, 2), pb2 = SB::np(e, 2), S1P = pa0 * pb0 * q1 * q1;
  const int b1 = t % pb1, a1 = (t / pb1) % pa1, b0 = (t / (pb1 * pa1)) % pb0, a0 = t / (pb1 * pa1 * pb0);
  const double* s1 = S1 + SB::s1_off(B) + (a0 * pb0 + b0) * q1 * q1;
  double s2[2][q1];
#pragma unroll
  for (int part = 0; part < 2; ++part)
#pragma unroll
    for (int qz = 0; qz < q1; ++qz) {
      double s = 0.0;
#pragma unroll
      for (int qy = 0; qy < q1; ++qy)
        s += fac(d, part, 1, a1, qy) * s1[part * S1P + qy + q1 * qz] * fac(e, part, 1, b1, qy);
      s2[part][qz] = s;
    }
  // every entry of the task in registers before the first store (the
  // tables and the stored entries may share LDS)
  double ent[pa2][pb2];
#pragma unroll
  for (int a2 = 0; a2 < pa2; ++a2) {
    double am[q1], ad[q1];
#pragma unroll
    for (int qz = 0; qz < q1; ++qz) {
      am[qz] = fac(d, 0, 2, a2, qz) * s2[0][qz];
      ad[qz] = fac(d, 1, 2, a2, qz) * s2[1][qz];
    }
#pragma unroll
    for (int b2 = 0; b2 < pb2; ++b2) {
      double s = 0.0;
#pragma unroll
      for (int qz = 0; qz < q1; ++qz) s += am[qz] * fac(e, 0, 2, b2, qz) + ad[qz] * fac(e, 1, 2, b2, qz);
      ent[a2][b2] = s;
    }
  }
#pragma unroll
  for (int a2 = 0; a2 < pa2; ++a2) {
    const int ia = dof_index<K>(d, a0, a1, a2);
#pragma unroll
    for (int b2 = 0; b2 < pb2; ++b2) {
      const int ib = dof_index<K>(e, b0, b1, b2);
      if (d == e && ib > ia) continue;
      if (ia >= ib) store(ia, ib, ent[a2][b2]); else store(ib, ia, ent[a2][b2]);
    }
  }
}

// The load vector by sum factorization: entry i (component d, 1D indices
// a0, a1, a2) is sum_q prod_x A_x[a_x][q_x] w_d(q), w_d(q) the per-point load
// weight of component d from element_qd (qd[q * 10 + 7 + d]), summed over the
// points along axis 0 into T1[d][a0][q1][q2] (one team-wide pass), then per
// (d, a0, a1) along axes 1 and 2 into the entries.  out(i, v) receives every
// entry once; stage: load_sumfact_stage<K>() doubles of LDS.  Ends with a
// barrier.
template <int K>
constexpr int load_sumfact_stage() {
  return sumfact_tables<K>() + (3 * (K + 1) + 2) * (K + 2) * (K + 2);
}
template <int K, int TEAM, class Out>
__device__ __forceinline__ void load_sumfact(const DeviceMaps& mp, const double* qd, double* stage, int lane, Out out) {
  using SB = SfBlocks<K>;
  constexpr int KC = K + 2, q1 = K + 2, QD = 10, TB = sumfact_tables<K>();
  __syncthreads();   // the team is done with the staging area
  for (int t = lane; t < TB; t += TEAM) stage[t] = mp.tab1d[t];
  const SfTables<K> fac{stage, stage + KC * q1, stage + 2 * KC * q1};
  double* T1 = stage + TB;
  // T1 of component d at (KC + (d - 1) K1) q1^2 for d >= 1: d = 0 has KC factors along axis 0
  auto t1_off = [](int d) { return d == 0 ? 0 : (SB::KC + (d - 1) * SB::K1) * q1 * q1; };
  constexpr int n1 = (SB::KC + 2 * SB::K1) * q1 * q1;
  __syncthreads();
  for (int t = lane; t < n1; t += TEAM) {
    const int d = t < SB::KC * q1 * q1 ? 0 : (t < (SB::KC + SB::K1) * q1 * q1 ? 1 : 2);
    const int r = t - t1_off(d), a0 = r / (q1 * q1), qq = r % (q1 * q1);
    double s = 0.0;
#pragma unroll
    for (int q0 = 0; q0 < q1; ++q0) s += fac(d, 0, 0, a0, q0) * qd[(q0 + q1 * qq) * QD + 7 + d];
    T1[t] = s;
  }
  __syncthreads();
  // tasks (d, a0, a1): KC K1 for d = 0 and d = 1, K1 K1 for d = 2
  constexpr int n2 = 2 * SB::KC * SB::K1 + SB::K1 * SB::K1;
  for (int t = lane; t < n2; t += TEAM) {
    const int d = t < SB::KC * SB::K1 ? 0 : (t < 2 * SB::KC * SB::K1 ? 1 : 2);
    const int r = t - (d == 0 ? 0 : (d == 1 ? SB::KC * SB::K1 : 2 * SB::KC * SB::K1));
    const int pa1 = SB::np(d, 1), pa2 = SB::np(d, 2);
    const int a0 = r / pa1, a1 = r % pa1;
    const double* t1 = T1 + t1_off(d) + a0 * q1 * q1;
    double t2[q1];
#pragma unroll
    for (int qz = 0; qz < q1; ++qz) {
      double s = 0.0;
#pragma unroll
      for (int qy = 0; qy < q1; ++qy) s += fac(d, 0, 1, a1, qy) * t1[qy + q1 * qz];
      t2[qz] = s;
    }
    for (int a2 = 0; a2 < pa2; ++a2) {
      double s = 0.0;
#pragma unroll
      for (int qz = 0; qz < q1; ++qz) s += fac(d, 0, 2, a2, qz) * t2[qz];
      out(dof_index<K>(d, a0, a1, a2), s);
    }
  }
  __syncthreads();
}

// Element matrix M_T by sum factorization (k >= 1, any trilinear element).
// The basis is a tensor product (per component d: the closed Lagrange factor
// along axis d, open ones along the other two) and the Gauss rule is a
// tensor rule, so block (d, e) of M_T,
//   sum_q G_de(q) prod_x A_x[a_x][q_x] B_x[b_x][q_x]
//     + w_div(q) prod_x A'_x[a_x][q_x] B'_x[b_x][q_x],
// (A, B: the 1D factors of components d and e, A', B' those of the
// divergences: derivatives of the closed factor on the own axis) is summed
// one axis at a time: over the points along axis 0 into S1[a0][b0][q1][q2]
// (all six blocks in one team-wide pass), then per (a0, b0, a1, b1) along
// axes 1 and 2 into the entries (a second pass), two barriers in all.  The
// per-point weights come from element_qd (qd: 6 metric weights
// w alpha (J^T J)_de / det J, the div-div weight w beta / det J).
// store(i, j, v) receives every entry with j <= i < n once.  stage:
// sumfact_stage<K>() doubles of LDS.
template <int K, int TEAM, class Store>
__device__ __forceinline__ void assemble_sumfact(const DeviceMaps& mp, const double* qd, double* stage, int lane,
                                                 Store store) {
  using SB = SfBlocks<K>;
  static_assert(K >= 1, "sum factorization for k >= 1");
  constexpr int KC = K + 2, q1 = K + 2;
  constexpr int TB = sumfact_tables<K>();
  __syncthreads();   // the team is done with the staging area
  for (int t = lane; t < TB; t += TEAM) stage[t] = mp.tab1d[t];
  const SfTables<K> fac{stage, stage + KC * q1, stage + 2 * KC * q1};
  double* S1 = stage + TB;
  __syncthreads();
  for (int t = lane; t < SB::t1_off(6); t += TEAM) {
    if (t < SB::t1_off(1)) sf_pass1<K, 0>(t, qd, fac, S1);
    else if (t < SB::t1_off(2)) sf_pass1<K, 1>(t - SB::t1_off(1), qd, fac, S1);
    else if (t < SB::t1_off(3)) sf_pass1<K, 2>(t - SB::t1_off(2), qd, fac, S1);
    else if (t < SB::t1_off(4)) sf_pass1<K, 3>(t - SB::t1_off(3), qd, fac, S1);
    else if (t < SB::t1_off(5)) sf_pass1<K, 4>(t - SB::t1_off(4), qd, fac, S1);
    else sf_pass1<K, 5>(t - SB::t1_off(5), qd, fac, S1);
  }
  __syncthreads();
  for (int t = lane; t < SB::t2_off(6); t += TEAM) {
    if (t < SB::t2_off(1)) sf_pass2<K, 0>(t, fac, S1, store);
    else if (t < SB::t2_off(2)) sf_pass2<K, 1>(t - SB::t2_off(1), fac, S1, store);
    else if (t < SB::t2_off(3)) sf_pass2<K, 2>(t - SB::t2_off(2), fac, S1, store);
    else if (t < SB::t2_off(4)) sf_pass2<K, 3>(t - SB::t2_off(3), fac, S1, store);
    else if (t < SB::t2_off(5)) sf_pass2<K, 4>(t - SB::t2_off(4), fac, S1, store);
    else sf_pass2<K, 5>(t - SB::t2_off(5), fac, S1, store);
  }
  __syncthreads();
}

}  // namespace hyb
