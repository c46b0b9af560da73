// Generic per-element setup / rhs / recovery kernels: one team of threads per
// element, the element matrix packed in LDS.  Used for every order whose
// packed FP64 matrix fits in LDS; faster order-specific kernels may replace
// it for particular k.
#pragma once

#include <type_traits>

#include "kernels_common.hpp"
#include "mfma.hpp"

namespace hyb {

enum : int { MODE_MATRIX = 1, MODE_RHS = 2 };

struct SetupArgs {
  DeviceMaps mp;
  int64_t ne;
  const double* alpha;
  const double* beta;
  const double* f;       // ne x 3 or null
  const double* g;       // ne x nb or null
  double* factor;        // ne x npk
  double* y;             // ne x n
  double* Hval;
  double* r;
  int32_t* status;
  int mode;
  int stat;              // 1: static condensation (S, its load) instead of H, r
};

struct RecoverArgs {
  DeviceMaps mp;
  int64_t ne;
  const double* factor;
  const double* y;
  const double* lambda;  // multipliers, or (static condensation) the face dofs
  double* u;
  int stat;
};

// Per-element LDS layout.  From k = 3 on the packed element matrix (231 KB)
// does not fit in LDS: it is then assembled and factored in place in its
// factor record in HBM (L2-resident while the element is processed), and the
// face block is inverted in place.
template <int K, int TEAM, int EPB>
struct GenericLayout {
  using R = RT<K>;
  static constexpr bool kGlobal = K >= 3;
  static constexpr int QD = 10;  // per-qp: 6 weighted metric terms, div weight, 3 load weights
  // assembly tables (and, HBM-resident matrices, the Cholesky's 32-column panel)
  static constexpr int stage_asm = TEAM % 64 == 0 ? 2 * R::n * kAsmQC : 0;
  static constexpr int stage = kGlobal && stage_asm < 32 * (R::n | 1) ? 32 * (R::n | 1) : stage_asm;
  // the last area holds the assembly tables and, once the element matrix is
  // assembled, the inverse face block (LDS-resident matrices)
  static constexpr int area = kGlobal ? stage : (stage > R::nbpk ? stage : R::nbpk);
  static constexpr int per = (kGlobal ? 0 : R::npk) + R::Q * QD + R::n + 24 + R::nb + area;
};

// Geometry at the Gauss points of one element (team of TEAM lanes): the
// trilinear map's Jacobian J from the 8 vertices and, per point q, the
// weighted terms w alpha (J^T J)_de / det J (6, when need_matrix), the
// div-div weight w beta / det J, and (need_rhs) w (J^T f)_d for the element
// load f.  det J <= 0 is reported.  Ends with a barrier.
template <int K, int TEAM>
__device__ __forceinline__ void element_qd(const DeviceMaps& mp, int64_t es, double al, double be, const double* fv,
                                           bool need_matrix, bool need_rhs, double* xe, double* qd, int lane,
                                           bool live, int32_t* status, int64_t e) {
  using R = RT<K>;
  constexpr int Q = R::Q, q1 = R::q1, QD = 10;
  for (int t = lane; t < 24; t += TEAM) xe[t] = mp.xyz[3 * int64_t(mp.e2v[es * 8 + t / 3]) + t % 3];
  __syncthreads();
  for (int q = lane; q < Q; q += TEAM) {
    double xi[3] = {mp.gauss_x[q % q1], mp.gauss_x[(q / q1) % q1], mp.gauss_x[q / (q1 * q1)]};
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      double fa[3], ga[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int bit = (v >> c) & 1;
        fa[c] = bit ? xi[c] : 1.0 - xi[c];
        ga[c] = bit ? 1.0 : -1.0;
      }
      const double dN[3] = {ga[0] * fa[1] * fa[2], fa[0] * ga[1] * fa[2], fa[0] * fa[1] * ga[2]};
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) J[r][c] += xe[3 * v + r] * dN[c];
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (live && !(det > 0.0)) report_error(status, HYB_E_JACOBIAN, e);
    const double w = mp.tab_w[q];
    if (need_matrix) {
      const double s = w * al / det;
      double G[6];
      int t = 0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = d; c < 3; ++c) G[t++] = J[0][d] * J[0][c] + J[1][d] * J[1][c] + J[2][d] * J[2][c];
#pragma unroll
      for (int t2 = 0; t2 < 6; ++t2) qd[q * QD + t2] = s * G[t2];
      qd[q * QD + 6] = w * be / det;
    }
    if (need_rhs) {
#pragma unroll
      for (int d = 0; d < 3; ++d) qd[q * QD + 7 + d] = w * (fv[0] * J[0][d] + fv[1] * J[1][d] + fv[2] * J[2][d]);
    }
  }
  __syncthreads();
}

// Entry (i, j) of M_T by Gauss quadrature from element_qd's per-point terms.
template <int K>
__device__ __forceinline__ double m_entry(const DeviceMaps& mp, const double* qd, int i, int j) {
  using R = RT<K>;
  constexpr int n = R::n, Q = R::Q, QD = 10;
  const int gi = gidx(R::comp(i), R::comp(j));
  double s = 0.0;
  for (int q = 0; q < Q; ++q)
    s += qd[q * QD + gi] * mp.tab_s[q * n + i] * mp.tab_s[q * n + j] +
         qd[q * QD + 6] * mp.tab_d[q * n + i] * mp.tab_d[q * n + j];
  return s;
}

// Lane src's value of v in every lane of the wave, for a wave-uniform src and
// all lanes active (the value __shfl(v, src) would give): two v_readlane
// through scalar registers instead of an LDS-routed permute.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ float wave_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// 1/sqrt(x) for a positive normal x: the hardware estimate refined by Newton
// steps on y^-2 = x (y <- y + y (1 - x y^2) / 2, each step roughly squaring
// the relative error; two steps reach the FP64 rounding level from the
// estimate's, one the FP32 level).
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ float rsqrt_refined(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  const float e = fmaf(-x * y, y, 1.0f);
  return fmaf(0.5f * y, e, y);
}

// Lane J's value of v in every lane of its row of 16 lanes (DPP
// row_newbcast: one instruction for 32- and 64-bit values, the result in a
// vector register).  row_bcast takes j as an argument for unrolled loops, where
// it is a constant.
template <int J, class T>
__device__ __forceinline__ T row_bcast_t(T v) {
  return __builtin_amdgcn_update_dpp(T(0), v, 0x150 + J, 0xf, 0xf, true);
}
template <class T>
__device__ __forceinline__ T row_bcast(T v, int j) {
  switch (j) {
    case 0: return row_bcast_t<0>(v);
    case 1: return row_bcast_t<1>(v);
    case 2: return row_bcast_t<2>(v);
    case 3: return row_bcast_t<3>(v);
    case 4: return row_bcast_t<4>(v);
    case 5: return row_bcast_t<5>(v);
    case 6: return row_bcast_t<6>(v);
    case 7: return row_bcast_t<7>(v);
    case 8: return row_bcast_t<8>(v);
    case 9: return row_bcast_t<9>(v);
    case 10: return row_bcast_t<10>(v);
    case 11: return row_bcast_t<11>(v);
    case 12: return row_bcast_t<12>(v);
    case 13: return row_bcast_t<13>(v);
    case 14: return row_bcast_t<14>(v);
    default: return row_bcast_t<15>(v);
  }
}

// The w x w (w <= 16) diagonal block at (c0, c0) of a packed lower triangle,
// factored on one wave: lane l holds row c0 + l % 16 in registers (the four
// rows of 16 lanes compute the same), pivots and column entries come by row
// broadcast (no barrier, no scalar registers).  Each pivot costs one refined
// reciprocal square root: L_cc = p / sqrt(p), the column below it scaled by
// 1 / sqrt(p), which also goes to rd[c] (LDS, for the rows below the block).
// The updates run unmasked: a lane's entries right of its diagonal take
// values that are never read or stored.  A non-positive pivot is replaced by
// 1 and reported (in every lane of the wave).
template <class T>
__device__ __forceinline__ bool chol_diag16(T* A, T* rd, int c0, int w, int l) {
  T d[16];
  const int r = l & 15, i = c0 + r;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    // every lane loads (a valid address), then keeps its own entries: no
    // lane-dependent branch around the loads
    const bool in = r < w && j <= r;
    const T v = A[in ? pk(i, c0 + j) : pk(c0, c0)];
    d[j] = in ? v : T(0);
  }
  bool bad = false;
  T rs = T(0);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c < w) {
      T piv = row_bcast(d[c], c);
      if (!(piv > T(0))) {
        bad = true;
        piv = T(1);
      }
      const T y = rsqrt_refined(piv);
      if (r == c) rs = y;
      d[c] = r == c ? piv * y : d[c] * y;
#pragma unroll
      for (int j = c + 1; j < 16; ++j) d[j] = fma(-d[c], row_bcast(d[c], j), d[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (l < w && j <= l) A[pk(i, c0 + j)] = d[j];
  if (l < w) rd[l] = rs;
  return bad;
}

// Rows c0 + 16 .. N - 1 of a full-width panel: L_21 = A_21 L_11^{-T} with
// the factored diagonal block L_11 and the reciprocals of its diagonal rd
// (LDS), one row per lane (its 16 entries in registers).  Column by column:
// entry c is finished, then taken off the entries after it, so the dependent
// chain is one multiply-add per column (the operations per entry, and their
// order, those of the dot-product form).
template <class T, int N, int TEAM>
__device__ __forceinline__ void chol_panel_rows(T* A, const T* rd, int c0, int lane) {
  for (int i = c0 + 16 + lane; i < N; i += TEAM) {
    T* Ai = A + i * (i + 1) / 2 + c0;
    T x[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = Ai[c];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      x[c] *= rd[c];
#pragma unroll
      for (int j = c + 1; j < 16; ++j) x[j] -= x[c] * A[pk(c0 + j, c0 + c)];
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) Ai[c] = x[c];
  }
}

// Packed lower Cholesky factorization in place in LDS, teams of whole waves,
// right-looking by panels of 16 columns aligned with 16 x 16 tiles: the
// panel's diagonal block on one wave (chol_diag16), the rows below it one
// per lane, and the trailing update of every lower tile (I, J) as
// C -= L_I L_J^T over the panel on the matrix cores of T (four 16 x 16 x 4
// steps per tile; each trailing entry belongs to one tile).  Look-ahead: of
// the trailing tiles, wave 0 takes the next diagonal tile and then factors it
// while the other waves update the rest, so each panel costs two barriers and
// the diagonal blocks (a serial chain of 16 pivots) overlap the updates.  A
// panel with rows below it is full width (only the last may be narrower).
// With active false the team only takes part in the barriers.  rd: 16 T of
// team LDS.  Returns true in the lanes of wave 0 when a pivot was not
// positive (replaced by 1).
template <class T, int N, int TEAM>
__device__ __forceinline__ bool chol_tiles16(T* A, T* rd, int lane, bool active) {
  using M = MfmaT<T>;
  constexpr int NB = 16, NT = (N + 15) / 16, NW = TEAM / 64;
  static_assert(TEAM % 64 == 0, "whole waves per team");
  const int w_id = lane / 64, l = lane % 64, li = l % 16, lc = l / 16;
  bool bad = false;
  __syncthreads();
  if (active && w_id == 0) bad |= chol_diag16(A, rd, 0, N < NB ? N : NB, l);
  __syncthreads();
  for (int K = 0; K + 1 < NT; ++K) {
    const int c0 = NB * K;
    if (active) chol_panel_rows<T, N, TEAM>(A, rd, c0, lane);
    __syncthreads();
    // trailing tiles (I, J), K < J <= I < NT, numbered row by row from (K + 1, K + 1)
    const int T0 = K + 1, m = NT - T0;
    auto tile = [&](int t) {
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      const int J = T0 + (t - I * (I + 1) / 2);
      I += T0;
      typename M::v4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + M::row(l, r), j = 16 * J + li;
        const bool in = i < N && j <= i;
        const T v = A[in ? pk(i, j) : 0];
        acc[r] = in ? v : T(0);
      }
      // operand loads at clamped (valid) addresses, masked values: no
      // lane-dependent branches around the loads
      const int ia = 16 * I + li, jb = 16 * J + li;
      const int iac = ia < N ? ia : N - 1, jbc = jb < N ? jb : N - 1;
#pragma unroll
      for (int kk = 0; kk < NB / 4; ++kk) {
        const int q = c0 + 4 * kk + lc;
        const T av = A[pk(iac, q)], bv = A[pk(jbc, q)];
        acc = M::op(ia < N ? -av : T(0), jb < N ? bv : T(0), acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + M::row(l, r), j = 16 * J + li;
        if (i < N && j <= i) A[pk(i, j)] = acc[r];
      }
    };
    const int c1 = c0 + NB, w1 = N - c1 < NB ? N - c1 : NB;
    if (active) {
      if (NW == 1) {
        for (int t = 0; t < m * (m + 1) / 2; ++t) tile(t);
        wave_sync();
        bad |= chol_diag16(A, rd, c1, w1, l);
      } else if (w_id == 0) {
        tile(0);
        wave_sync();
        bad |= chol_diag16(A, rd, c1, w1, l);
      } else {
        for (int t = w_id; t < m * (m + 1) / 2; t += NW - 1) tile(t);
      }
    }
    __syncthreads();
  }
  return bad;
}

// Inverses of the 16 x 16 diagonal blocks of a lower factor L (lower
// triangular, the identity past N), one block per wave in turn and a lane
// per column (forward substitution, x_i = (delta_ij - sum_k L_ik x_k) / L_ii):
// Linv[256 I + 16 i + j].  L(i, j) reads the factor for j <= i < N.
template <class T, int N, int TEAM, class LAcc>
__device__ __forceinline__ void diag_inverses(LAcc L, T* Linv, int lane, bool active) {
  constexpr int NT = (N + 15) / 16, NW = TEAM / 64;
  const int w_id = lane / 64, j = lane % 64;
  if (!active || j >= 16) return;
  for (int I = w_id; I < NT; I += NW) {
    const int c0 = 16 * I;
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      // x_k = 0 for k < j, so the sum needs no lane-dependent bounds (no
      // branch around the loads)
      T s = i == j ? T(1) : T(0);
      if (c0 + i < N) {   // uniform
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L(c0 + i, c0 + k) * x[k];
        const T xi = s / L(c0 + i, c0 + i);
        x[i] = i >= j ? xi : T(0);
      } else {
        x[i] = s;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Linv[256 * I + 16 * i + j] = x[i];
  }
}

// FP64 forward substitution W := L^{-1} W on one column tile (columns c0 ..
// c0 + ncol - 1, ncol <= 16) by one wave with the whole tile in registers:
// the FP64 matrix-core result layout (rows l/16 + 4r of column l % 16) is the
// layout of the B operand at k-step r (rows 4r + l/16), so a solved 16-row
// block feeds the next blocks' products straight from its accumulator, and
// the tile touches memory only when it is loaded.  load(i, c) reads the tile
// (i < N, c < c0 + ncol); L(i, j) is the factor (j <= i < N, LDS) and Linv
// its diagonal blocks' inverses.  The tile's row blocks before I0 are zero
// (and stay so), and are skipped.  On return X[I][r] holds row 16 I + l/16 +
// 4 r of column c0 + l % 16 (zero past N and for columns past ncol).
template <int N, class LAcc, class Load>
__device__ __forceinline__ void tile_forward_regs(LAcc L, const double* Linv, Load load, dx4 (&X)[(N + 15) / 16], int c0,
                                                  int ncol, int l, int I0 = 0) {
  using M = MfmaT<double>;
  constexpr int NT = (N + 15) / 16;
  const int li = l & 15, lk = l >> 4;
  const bool cok = li < ncol;
  const int cc = cok ? c0 + li : c0;
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + M::row(l, r);
      const double v = load(i < N ? i : N - 1, cc);
      X[I][r] = (cok && i < N) ? v : 0.0;
    }
#pragma unroll
  for (int I = 0; I < NT; ++I) {
    if (I < I0) continue;   // uniform
    const int i = 16 * I + li, ic = i < N ? i : N - 1;
    dx4 acc = X[I];
#pragma unroll
    for (int J = 0; J < I; ++J)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (J < I0) continue;
        const double lv = L(ic, 16 * J + 4 * s + lk);
        acc = M::op(i < N ? -lv : 0.0, X[J][s], acc);
      }
    dx4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) x = M::op(Linv[256 * I + 16 * li + 4 * s + lk], acc[s], x);
    X[I] = x;
  }
}

// tile_forward_regs with the result stored through store(i, c, v) (i < N,
// c < c0 + ncol).
template <int N, class LAcc, class Load, class Store>
__device__ __forceinline__ void tile_forward_reg(LAcc L, const double* Linv, Load load, Store store, int c0, int ncol,
                                                 int l, int I0 = 0) {
  using M = MfmaT<double>;
  constexpr int NT = (N + 15) / 16;
  dx4 X[NT];
  tile_forward_regs<N>(L, Linv, load, X, c0, ncol, l, I0);
  const int li = l & 15;
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + M::row(l, r);
      if (li < ncol && i < N) store(i, c0 + li, X[I][r]);
    }
}

// The FP64 form for LDS-resident matrices and teams of whole waves
// (chol_tiles16).  rd: 16 doubles of team LDS.
template <int N, int TEAM>
__device__ __forceinline__ bool chol_packed_mfma(double* A, int lane, double* rd) {
  return chol_tiles16<double, N, TEAM>(A, rd, lane, true);
}

// Packed lower Cholesky factorization in place (LDS or global), right-
// looking by panels of NB columns: each panel column is factored and applied
// to the panel's later columns (one barrier per column; the column is scaled
// after the barrier, it is not read again within the panel), then one
// rank-NB update of the trailing triangle reads and writes every trailing
// entry once per panel.  In the trailing update S = TEAM / N lanes share a
// row and each keeps the row's NB panel entries in registers.  Returns true
// (in every lane) when a pivot was not positive (replaced by 1).  FP64 on
// LDS with teams of whole waves takes chol_packed_mfma (rd: 16 T of team LDS
// for it).
template <class T, int N, int TEAM>
__device__ __forceinline__ bool chol_packed(T* A, int lane, T* rd) {
  if constexpr (std::is_same<T, double>::value && TEAM % 64 == 0 && N >= 32) return chol_packed_mfma<N, TEAM>(A, lane, rd);
  constexpr int NB = N >= 64 ? 8 : 4;
  constexpr int S = TEAM / N > 0 ? TEAM / N : 1;
  bool bad = false;
  for (int c0 = 0; c0 < N; c0 += NB) {
    const int w = N - c0 < NB ? N - c0 : NB;
    for (int c = c0; c < c0 + w; ++c) {
      T d = A[pk(c, c)];
      if (!(d > T(0))) {
        bad = true;
        d = T(1);
      }
      const T inv = T(1) / d;
      for (int i = c + 1 + lane; i < N; i += TEAM) {
        T* Ai = A + i * (i + 1) / 2;
        const T aic = Ai[c] * inv;
        const int jend = i < c0 + w - 1 ? i : c0 + w - 1;
        for (int j = c + 1; j <= jend; ++j) Ai[j] -= aic * A[pk(j, c)];
      }
      __syncthreads();
      const T sq = sqrt(d), is = T(1) / sq;
      for (int i = c + 1 + lane; i < N; i += TEAM) A[pk(i, c)] *= is;
      if (lane == 0) A[pk(c, c)] = sq;
    }
    __syncthreads();
    for (int i = c0 + w + lane / S; i < N && lane / S < TEAM / S; i += TEAM / S) {
      T* Ai = A + i * (i + 1) / 2;
      T li[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) li[t] = t < w ? Ai[c0 + t] : T(0);
      for (int j = c0 + w + lane % S; j <= i; j += S) {
        const T* Aj = A + j * (j + 1) / 2 + c0;
        T acc = Ai[j];
#pragma unroll
        for (int t = 0; t < NB; ++t)
          if (t < w) acc -= li[t] * Aj[t];
        Ai[j] = acc;
      }
    }
    __syncthreads();
  }
  return bad;
}

// chol_packed for an FP64 matrix in HBM (the element's record), teams of
// whole waves, by panels of 32 columns staged column-major in LDS
// (P[q * LD + r] = A[c0 + r][c0 + q], LD odd for conflict-free lanes).  The
// panel is factored in LDS as two sub-panels of 16: each one's diagonal block
// on one wave (registers and wave broadcasts), the rows below it one per lane, the
// second sub-panel first updated by the first.  The finished panel is written
// back, then the trailing update A_ij -= sum_q L_iq L_jq runs over chunks of
// 64 columns: a lane keeps its column's panel entries in registers and the
// team's waves take the chunk's rows in turn, each row read and written as 64
// consecutive entries (one HBM read-modify-write per trailing entry and
// panel).  With own false (a padding team) nothing is written to A.
template <int N, int TEAM>
__device__ __forceinline__ bool chol_hbm32(double* A, double* P, int lane, bool own) {
  constexpr int NB = 32, NW = TEAM / 64, LD = N | 1;
  static_assert(TEAM % 64 == 0, "whole waves per team");
  const int wv = lane / 64, l = lane % 64;
  bool bad = false;
  for (int c0 = 0; c0 < N; c0 += NB) {
    const int w = N - c0 < NB ? N - c0 : NB, R = N - c0;
    for (int t = lane; t < R * NB; t += TEAM) {
      const int r = t / NB, q = t % NB;
      P[q * LD + r] = (q < w && q <= r) ? A[pk(c0 + r, c0 + q)] : 0.0;
    }
    __syncthreads();
    for (int s0 = 0; s0 < w; s0 += 16) {
      const int ws = w - s0 < 16 ? w - s0 : 16;
      if (s0 > 0) {
        // the second sub-panel's columns minus the first's contribution
        for (int r = s0 + lane; r < R; r += TEAM) {
          double x[16];
#pragma unroll
          for (int t = 0; t < 16; ++t) x[t] = P[t * LD + r];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            if (q < ws && s0 + q <= r) {
              double acc = P[(s0 + q) * LD + r];
#pragma unroll
              for (int t = 0; t < 16; ++t) acc -= x[t] * P[t * LD + s0 + q];
              P[(s0 + q) * LD + r] = acc;
            }
          }
        }
        __syncthreads();
      }
      if (wv == 0) {
        double d[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) d[j] = (l < ws && j <= l) ? P[(s0 + j) * LD + s0 + l] : 0.0;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c < ws) {
            double piv = wave_bcast(d[c], c);
            if (!(piv > 0.0)) {
              bad = true;
              piv = 1.0;
            }
            const double sq = sqrt(piv), is = 1.0 / sq;
            d[c] = l == c ? sq : (l > c ? d[c] * is : d[c]);
#pragma unroll
            for (int j = c + 1; j < 16; ++j) {
              const double ljc = wave_bcast(d[c], j);
              if (l >= j) d[j] -= d[c] * ljc;
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (l < ws && j <= l) P[(s0 + j) * LD + s0 + l] = d[j];
      }
      __syncthreads();
      for (int r = s0 + ws + lane; r < R; r += TEAM) {
        double x[16], rc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          x[c] = c < ws ? P[(s0 + c) * LD + r] : 0.0;
          rc[c] = c < ws ? 1.0 / P[(s0 + c) * LD + s0 + c] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c < ws) {
            double sum = x[c];
#pragma unroll
            for (int q = 0; q < c; ++q) sum -= x[q] * P[(s0 + q) * LD + s0 + c];
            x[c] = sum * rc[c];
          }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c < ws) P[(s0 + c) * LD + r] = x[c];
      }
      __syncthreads();
    }
    for (int t = lane; t < R * NB; t += TEAM) {
      const int r = t / NB, q = t % NB;
      if (own && q < w && q <= r) A[pk(c0 + r, c0 + q)] = P[q * LD + r];
    }
    for (int j0 = w; j0 < R; j0 += 64) {
      const int jr = j0 + l;   // the lane's column, relative to c0
      double pj[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) pj[q] = (q < w && jr < R) ? P[q * LD + jr] : 0.0;
      for (int ir = j0 + wv; ir < R; ir += NW) {
        if (own && jr <= ir) {
          double* a = A + pk(c0 + ir, c0 + jr);
          double acc = *a;
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < w) acc -= P[q * LD + ir] * pj[q];
          *a = acc;
        }
      }
    }
    __syncthreads();
  }
  return bad;
}

// Triangular solves with the leading NI x NI block of a packed lower factor
// L in LDS, by the team's first wave: its lanes keep the vector in registers
// (rows lane + 64 r) and every solved entry reaches them by a wave broadcast, so
// there is no block barrier per column.  Per entry the operations and their
// order are those of the column-oriented loops (y_c = y_c / L_cc, then
// y_i -= L_ic y_c).  Both end with a barrier.
template <int NI>
__device__ __forceinline__ void wave_forward(const double* L, double* y, int lane) {
  constexpr int RPL = (NI + 63) / 64;
  if (RPL > 0 && lane < 64) {
    // the reciprocals of the lane's diagonal entries first, off the chain of
    // updates: a step multiplies by one in the lane of its row and
    // broadcasts the product
    double yr[RPL > 0 ? RPL : 1], rinv[RPL > 0 ? RPL : 1];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      yr[r] = i < NI ? y[i] : 0.0;
      rinv[r] = i < NI ? 1.0 / L[pk(i, i)] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int cend = NI < 64 * (s + 1) ? NI : 64 * (s + 1);
      for (int c = 64 * s; c < cend; ++c) {
        const double yc = wave_bcast(yr[s] * rinv[s], c - 64 * s);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          // unconditional load (clamped address), masked product: no branch
          const int i = lane + 64 * r;
          const bool in = i > c && i < NI;
          const double lic = L[in ? pk(i, c) : pk(c, c)];
          yr[r] -= (in ? lic : 0.0) * yc;
        }
        if (lane == c - 64 * s) yr[s] = yc;
      }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      if (i < NI) y[i] = yr[r];
    }
  }
  __syncthreads();
}

// z := L^{-T} z with the same leading block (back substitution); UNROLL
// steps of the column loop at a time, so that a factor in HBM has its loads
// (which do not depend on z) in flight ahead of the chain of updates.
template <int NI, int UNROLL = 1>
__device__ __forceinline__ void wave_backward(const double* L, double* z, int lane) {
  constexpr int RPL = (NI + 63) / 64;
  if (RPL > 0 && lane < 64) {
    double zr[RPL > 0 ? RPL : 1];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int j = lane + 64 * r;
      zr[r] = j < NI ? z[j] : 0.0;
    }
#pragma unroll
    for (int s = RPL - 1; s >= 0; --s) {
      const int cend = NI < 64 * (s + 1) ? NI : 64 * (s + 1);
#pragma unroll UNROLL
      for (int c = cend - 1; c >= 64 * s; --c) {
        const double uc = wave_bcast(zr[s], c - 64 * s) / L[pk(c, c)];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int j = lane + 64 * r;
          const bool in = j < c;
          const double lcj = L[in ? pk(c, j) : pk(c, c)];
          zr[r] -= (in ? lcj : 0.0) * uc;
        }
        if (lane == c - 64 * s) zr[s] = uc;
      }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int j = lane + 64 * r;
      if (j < NI) z[j] = zr[r];
    }
  }
  __syncthreads();
}

// Local assembly (Gauss quadrature), essential-face masking, packed
// Cholesky in i-first order, inversion of the face block, H_T scatter, and
// the right-hand side y = L^{-1} f_hat, r_T = D L_bb^{-T} y_b.
// Static condensation (a.stat): the element Schur complement
// S_hat_T = A_bb - A_bi A_ii^{-1} A_ib = L_bb L_bb^T is scattered instead,
// each face-dof copy signed by sigma = eps_f (owner) or -eps_f (neighbour),
// the global face dof being the owner's outward flux, with the load
// sigma (f_b - L_bi L_ii^{-1} f_i); the face block is not inverted.
template <int K, int TEAM, int EPB>
__device__ __forceinline__ void setup_generic_body(const SetupArgs& a, double* smem, int64_t blk) {
  using R = RT<K>;
  using Lay = GenericLayout<K, TEAM, EPB>;
  constexpr int n = R::n, ni = R::ni, nb = R::nb, K1 = R::K1, K2 = R::K2, Q = R::Q, q1 = R::q1;
  constexpr int QD = Lay::QD;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t e = blk * EPB + team;
  const bool live = e < a.ne;
  const int64_t es = live ? e : 0;  // safe index for loads of padding teams
  double* base = smem + team * Lay::per;
  double* A = Lay::kGlobal ? a.factor + es * R::npk : base;
  // a padding team (past the last element) of an HBM-resident matrix reads
  // element 0's record, which another team factors: it writes nothing there
  const bool own = !Lay::kGlobal || live;
  double* qd = Lay::kGlobal ? base : base + R::npk;
  double* fh = qd + Q * QD;
  double* xe = fh + n;
  double* tb = xe + 24;
  double* stg = tb + nb;
  double* Li = Lay::kGlobal ? nullptr : stg;   // written after the assembly
  // packed inverse of the face block: its own LDS array, or (global matrix)
  // the face block of A, inverted in place
  // (an HBM-resident matrix has its face block copied to the staging area
  // of LDS for the inversion and what reads the inverse in the same call)
  bool fb_lds = false;
  auto LI = [&](int i, int j) -> double& {
    return Lay::kGlobal ? (fb_lds ? stg[pk(i, j)] : A[pk(ni + i, ni + j)]) : Li[pk(i, j)];
  };
  const DeviceMaps& mp = a.mp;

  int fid[6], pic[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    fid[f] = mp.elem_face[es * 6 + f];
    pic[f] = mp.elem_pi[es * 8 + f];
  }
  // essential dofs: those of boundary faces not marked natural
  const int nat = mp.elem_pi[es * 8 + 6];
  auto is_ess = [&](int i) {
    const int f = (i - ni) / K2;
    return i >= ni && fid[f] < 0 && !((nat >> f) & 1);
  };
  // static condensation: sign of face dof b's copy of the owner's outward flux
  auto sigma = [&](int b) {
    const int f = b / K2;
    const double eps = (f & 1) ? 1.0 : -1.0;
    return mp.face_owner[fid[f]] == e ? eps : -eps;
  };

  const double al = a.alpha ? a.alpha[es] : 0.0, be = a.beta ? a.beta[es] : 0.0;
  double fv[3] = {0.0, 0.0, 0.0};
  if (a.mode & MODE_RHS) {
    fv[0] = a.f[es * 3 + 0]; fv[1] = a.f[es * 3 + 1]; fv[2] = a.f[es * 3 + 2];
  }
  const bool need_matrix = (a.mode & MODE_MATRIX) || ((a.mode & MODE_RHS) && a.g);
  element_qd<K, TEAM>(mp, es, al, be, fv, need_matrix, (a.mode & MODE_RHS) != 0, xe, qd, lane, live, a.status, e);

  // entry (i, j) of M_T by Gauss quadrature
  auto mij = [&](int i, int j) {
    const int gi = gidx(R::comp(i), R::comp(j));
    double s = 0.0;
    for (int q = 0; q < Q; ++q)
      s += qd[q * QD + gi] * mp.tab_s[q * n + i] * mp.tab_s[q * n + j] +
           qd[q * QD + 6] * mp.tab_d[q * n + i] * mp.tab_d[q * n + j];
    return s;
  };
  // (an HBM-resident matrix is the stored factor: a right-hand side alone
  // must not overwrite it, and computes the entries it needs directly)
  const bool store_matrix = need_matrix && (!Lay::kGlobal || (a.mode & MODE_MATRIX));
  if (store_matrix) {
    if constexpr (use_sumfact<K>()) {
      static_assert(Lay::stage >= sumfact_stage<K>(), "the sum factorization's partial sums fit in the staging area");
      assemble_sumfact<K, TEAM>(mp, qd, stg, lane, [=](int i, int j, double v) {
        if (own) A[pk(i, j)] = v;
      });
    } else if constexpr (TEAM % 64 == 0) {
      assemble_mfma<K, TEAM, kAsmQC>(mp, qd, stg, lane, [=](int i, int j, double v) {
        if (own) A[pk(i, j)] = v;
      });
    } else {
      for (int p = lane; p < R::npk; p += TEAM) {
        int i, j;
        unpk(p, i, j);
        if (own) A[p] = mij(i, j);
      }
    }
    __syncthreads();
  }
  if (a.mode & MODE_RHS) {
    for (int i = lane; i < n; i += TEAM) {
      const int d = R::comp(i);
      double s = 0.0;
#pragma unroll 8
      for (int q = 0; q < Q; ++q) s += mp.tab_s[q * n + i] * qd[q * QD + 7 + d];
      if (is_ess(i)) {
        s = a.g ? a.g[es * nb + (i - ni)] : 0.0;
      } else if (a.g) {
        // f_r -= M_re g_e (unmasked matrix)
        for (int j = ni; j < n; ++j)
          if (is_ess(j))
            s -= (store_matrix ? A[i > j ? pk(i, j) : pk(j, i)] : (i > j ? mij(i, j) : mij(j, i))) *
                 a.g[es * nb + (j - ni)];
      }
      fh[i] = s;
    }
    __syncthreads();
  }

  if (a.mode & MODE_MATRIX) {
    // boundary faces are essential: identity rows/columns (a pass over the
    // matrix only for an element with an essential face)
    bool any_ess = false;
#pragma unroll
    for (int f = 0; f < 6; ++f) any_ess |= is_ess(ni + f * K2);
    if (any_ess) {   // uniform across the team
      for (int p = lane; p < R::npk; p += TEAM) {
        int i, j;
        unpk(p, i, j);
        if (own && (is_ess(i) || is_ess(j))) A[p] = (i == j) ? 1.0 : 0.0;
      }
    }
    __syncthreads();
    // Cholesky (interior block first, so L_bb L_bb^T is the element's Schur
    // complement onto its face dofs)
    bool notspd;
    if constexpr (Lay::kGlobal) {
      static_assert(Lay::stage >= 32 * (n | 1), "the panel fits in the staging area");
      notspd = chol_hbm32<n, TEAM>(A, stg, lane, own);
    } else {
      static_assert(TEAM % 64 != 0 || n < 32 || Lay::stage >= 16, "the pivots' reciprocals fit in the staging area");
      notspd = chol_packed<double, n, TEAM>(A, lane, stg);
    }
    if (notspd && live && lane == 0) report_error(a.status, HYB_E_NOT_SPD, e);
    __syncthreads();
    if (a.stat) {
      // S_hat_T = L_bb L_bb^T (lower triangle), sigma-signed, into S
      if (live) {
        for (int t = lane; t < R::nbpk; t += TEAM) {
          int aa, bb;
          unpk(t, aa, bb);
          const int fa = aa / K2, fb = bb / K2;
          if (fid[fa] < 0 || fid[fb] < 0) continue;
          double h = 0.0;
          for (int c = 0; c <= bb; ++c) h += A[pk(ni + aa, ni + c)] * A[pk(ni + bb, ni + c)];
          const double v = sigma(aa) * sigma(bb) * h;
          int a0 = (aa % K2) % K1, a1 = (aa % K2) / K1, b0 = (bb % K2) % K1, b1 = (bb % K2) / K1;
          frame_map(pic[fa], K, a0, a1);
          frame_map(pic[fb], K, b0, b1);
          const int ja = a0 + K1 * a1, jb = b0 + K1 * b1;
          const int Fa = fid[fa], Fb = fid[fb];
          const int64_t pab = mp.face_rowbase[Fa] + int64_t(ja) * mp.face_nslots[Fa] * K2 +
                              mp.elem_slot[e * 36 + fa * 6 + fb] * K2 + jb;
          const int64_t pba = mp.face_rowbase[Fb] + int64_t(jb) * mp.face_nslots[Fb] * K2 +
                              mp.elem_slot[e * 36 + fb * 6 + fa] * K2 + ja;
          if (fa == fb) {
            atomicAdd(&a.Hval[pab], v);
            if (aa != bb) atomicAdd(&a.Hval[pba], v);
          } else {
            a.Hval[pab] = v;
            a.Hval[pba] = v;
          }
        }
      }
    } else if constexpr (!Lay::kGlobal && TEAM % 64 == 0 && TEAM / 64 >= (nb + 15) / 16) {
      // Inverse of the face block L_bb by forward tile solves held in
      // registers, a wave per 16-column tile, the 16-row blocks on the FP64
      // matrix cores (the inverses of L_bb's diagonal blocks staged after Li)
      double* LiB = stg + R::nbpk;
      static_assert(Lay::area >= R::nbpk + ((nb + 15) / 16) * 256, "Li and the diagonal blocks' inverses fit");
      auto Lbb = [=](int i, int j) -> double { return A[pk(ni + i, ni + j)]; };
      diag_inverses<double, nb, TEAM>(Lbb, LiB, lane, true);
      __syncthreads();
      const int wv = lane / 64;
      if (wv < (nb + 15) / 16)
        tile_forward_reg<nb>(Lbb, LiB, [](int i, int c) { return i == c ? 1.0 : 0.0; },
                             [=](int i, int c, double v) {
                               if (i >= c) Li[pk(i, c)] = v;
                             },
                             16 * wv, nb - 16 * wv < 16 ? nb - 16 * wv : 16, lane % 64, wv);
    } else if constexpr (!Lay::kGlobal && TEAM % 64 == 0 && nb <= 64) {
      // Inverse of the face block L_bb, its columns dealt to the waves: lane
      // l holds row l of RC columns in registers, forward substitution row by
      // row, each solved entry broadcast to the wave (no block barrier); per
      // entry the sum runs over c = col..i-1 in order, as in the loop below.
      constexpr int NW = TEAM / 64, RC = (nb + NW - 1) / NW;
      const int wv = lane / 64, l = lane % 64;
      double x[RC];
#pragma unroll
      for (int r = 0; r < RC; ++r) x[r] = (l == wv + NW * r) ? 1.0 : 0.0;
      for (int c = 0; c < nb; ++c) {
        const double lcc = A[pk(ni + c, ni + c)];
        const double lic = (l > c && l < nb) ? A[pk(ni + l, ni + c)] : 0.0;
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          if (wv + NW * r <= c) {   // uniform across the wave
            if (l == c) x[r] = x[r] / lcc;
            const double xc = wave_bcast(x[r], c);
            if (l > c) x[r] -= lic * xc;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const int col = wv + NW * r;
        if (col < nb && l >= col && l < nb) Li[pk(l, col)] = x[r];
      }
    } else if constexpr (!Lay::kGlobal) {
      // Inverse of the face block L_bb, one column per thread.
      for (int col = lane; col < nb; col += TEAM) {
        Li[pk(col, col)] = 1.0 / A[pk(ni + col, ni + col)];
        for (int i = col + 1; i < nb; ++i) {
          double s = 0.0;
          for (int c = col; c < i; ++c) s += A[pk(ni + i, ni + c)] * Li[pk(c, col)];
          Li[pk(i, col)] = -s / A[pk(ni + i, ni + i)];
        }
      }
    } else {
      // the face block into LDS, inverted in place there, written back
      static_assert(Lay::stage >= R::nbpk, "the face block fits in the staging area");
      double* Fb = stg;
      for (int t = lane; t < R::nbpk; t += TEAM) {
        int i, j;
        unpk(t, i, j);
        Fb[t] = A[pk(ni + i, ni + j)];
      }
      __syncthreads();
      // In place, by blocks of 16 columns right to left, from
      // X_jj = 1 / L_jj and X_ij = -(sum_{c=j+1..i} X_ic L_cj) / L_jj: a lane per
      // row i sums the terms of the finished columns c beyond the block into
      // registers (reading the block's original columns), then, after a
      // barrier, finishes its row of the block from right to left with the
      // block's diagonal part of L kept in Dg (the block's columns are being
      // overwritten).  Two barriers per block instead of two per column.
      static_assert(Lay::stage >= R::nbpk + 136, "the face block and a diagonal block fit in the staging area");
      static_assert(TEAM >= nb, "a lane per row of the face block");
      double* Dg = Fb + R::nbpk;
      for (int j0 = ((nb - 1) / 16) * 16; j0 >= 0; j0 -= 16) {
        const int w = nb - j0 < 16 ? nb - j0 : 16;
        for (int t = lane; t < w * (w + 1) / 2; t += TEAM) {
          int aa, bb;
          unpk(t, aa, bb);
          Dg[t] = Fb[pk(j0 + aa, j0 + bb)];
        }
        const int i = j0 + lane;
        double pr[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) pr[jj] = 0.0;
        if (i >= j0 + w && i < nb) {
          for (int c = j0 + w; c <= i; ++c) {
            const double xic = Fb[pk(i, c)];
            const double* Lc = Fb + pk(c, j0);
#pragma unroll
            for (int jj = 0; jj < 16; ++jj)
              if (jj < w) pr[jj] += xic * Lc[jj];
          }
        }
        __syncthreads();   // the block's columns of L are read, Dg is complete
        if (i < nb) {
          double x[16];
#pragma unroll
          for (int jj = 15; jj >= 0; --jj) {
            x[jj] = 0.0;
            const int j = j0 + jj;
            if (jj < w && j <= i) {
              if (j == i) {
                x[jj] = 1.0 / Dg[pk(jj, jj)];
              } else {
                double sacc = pr[jj];
#pragma unroll
                for (int cc = jj + 1; cc < 16; ++cc)
                  if (cc < w && j0 + cc <= i) sacc += x[cc] * Dg[pk(cc, jj)];
                x[jj] = -sacc / Dg[pk(jj, jj)];
              }
            }
          }
#pragma unroll
          for (int jj = 0; jj < 16; ++jj)
            if (jj < w && j0 + jj <= i) Fb[pk(i, j0 + jj)] = x[jj];
        }
        __syncthreads();
      }
      for (int t = lane; t < R::nbpk; t += TEAM) {
        int i, j;
        unpk(t, i, j);
        if (own) A[pk(ni + i, ni + j)] = Fb[t];
      }
      fb_lds = true;
    }
    __syncthreads();
    // H_T = D L_bb^{-T} L_bb^{-1} D, scattered into H (lower triangle computed,
    // mirrored; same-face blocks receive two element terms by atomic add).
    // Where the face block's inverse is in LDS and the team has whole waves,
    // the lower 16 x 16 tiles of X^T X (X = L_bb^{-1}, lower triangular: the
    // sum starts at row block I) on the FP64 matrix cores; else per entry.
    auto scatter = [&](int aa, int bb, double h) {
      const int fa = aa / K2, fb = bb / K2;
      if (fid[fa] < 0 || fid[fb] < 0) return;
      const double v = ((fa ^ fb) & 1) ? -h : h;
      int a0 = (aa % K2) % K1, a1 = (aa % K2) / K1, b0 = (bb % K2) % K1, b1 = (bb % K2) / K1;
      frame_map(pic[fa], K, a0, a1);
      frame_map(pic[fb], K, b0, b1);
      const int ja = a0 + K1 * a1, jb = b0 + K1 * b1;
      const int Fa = fid[fa], Fb = fid[fb];
      const int64_t pab = mp.face_rowbase[Fa] + int64_t(ja) * mp.face_nslots[Fa] * K2 +
                          mp.elem_slot[e * 36 + fa * 6 + fb] * K2 + jb;
      const int64_t pba = mp.face_rowbase[Fb] + int64_t(jb) * mp.face_nslots[Fb] * K2 +
                          mp.elem_slot[e * 36 + fb * 6 + fa] * K2 + ja;
      const double vw = v * (mp.face_w[ja] * mp.face_w[jb]);   // M_s H_T M_s (weighted C)
      if (fa == fb) {
        atomicAdd(&a.Hval[pab], vw);
        if (aa != bb) atomicAdd(&a.Hval[pba], vw);
      } else {
        a.Hval[pab] = vw;
        a.Hval[pba] = vw;
      }
    };
    if constexpr (!Lay::kGlobal && TEAM % 64 == 0 && nb >= 16) {
      using M = MfmaT<double>;
      constexpr int NTb = (nb + 15) / 16, NW = TEAM / 64;
      const int wv = lane / 64, l = lane % 64, li = l & 15, lk = l >> 4;
      for (int t = a.stat ? (1 << 30) : wv; t < NTb * (NTb + 1) / 2; t += NW) {
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        const int J = t - I * (I + 1) / 2;
        // column 16 I + li (A operand) and 16 J + li (B operand) of X, rows
        // c >= the column (zero above the diagonal), clamped loads
        const int ca = 16 * I + li, cb = 16 * J + li;
        const int cac = ca < nb ? ca : nb - 1, cbc = cb < nb ? cb : nb - 1;
        dx4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int c0 = 16 * I; c0 < nb; c0 += 4) {
          const int c = c0 + lk, cc = c < nb ? c : nb - 1;
          const double xa = Li[pk(cc, cc >= cac ? cac : cc)], xb = Li[pk(cc, cc >= cbc ? cbc : cc)];
          acc = M::op((c < nb && ca < nb && c >= ca) ? xa : 0.0, (c < nb && cb < nb && c >= cb) ? xb : 0.0, acc);
        }
        if (!live) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int aa = 16 * I + M::row(l, r), bb = cb;
          if (aa < nb && bb < nb && bb <= aa) scatter(aa, bb, acc[r]);
        }
      }
    } else if (live && !a.stat) {
      for (int t = lane; t < R::nbpk; t += TEAM) {
        int aa, bb;
        unpk(t, aa, bb);
        const int fa = aa / K2, fb = bb / K2;
        if (fid[fa] < 0 || fid[fb] < 0) continue;
        double h = 0.0;
        for (int c = aa; c < nb; ++c) h += LI(c, aa) * LI(c, bb);
        const double v = ((fa ^ fb) & 1) ? -h : h;
        int a0 = (aa % K2) % K1, a1 = (aa % K2) / K1, b0 = (bb % K2) % K1, b1 = (bb % K2) / K1;
        frame_map(pic[fa], K, a0, a1);
        frame_map(pic[fb], K, b0, b1);
        const int ja = a0 + K1 * a1, jb = b0 + K1 * b1;
        const int Fa = fid[fa], Fb = fid[fb];
        const int64_t pab = mp.face_rowbase[Fa] + int64_t(ja) * mp.face_nslots[Fa] * K2 +
                            mp.elem_slot[e * 36 + fa * 6 + fb] * K2 + jb;
        const int64_t pba = mp.face_rowbase[Fb] + int64_t(jb) * mp.face_nslots[Fb] * K2 +
                            mp.elem_slot[e * 36 + fb * 6 + fa] * K2 + ja;
        const double vw = v * (mp.face_w[ja] * mp.face_w[jb]);   // M_s H_T M_s (weighted C)
        if (fa == fb) {
          atomicAdd(&a.Hval[pab], vw);
          if (aa != bb) atomicAdd(&a.Hval[pba], vw);
        } else {
          a.Hval[pab] = vw;
          a.Hval[pba] = vw;
        }
      }
    }
  } else if (a.mode & MODE_RHS) {
    if constexpr (!Lay::kGlobal) {
      // rhs only: bring the stored factor back (face block holds L_bb^{-1})
      for (int p = lane; p < R::npk; p += TEAM) {
        int i, j;
        unpk(p, i, j);
        const double v = a.factor[es * R::npk + p];
        if (i >= ni && j >= ni) Li[pk(i - ni, j - ni)] = v; else A[p] = v;
      }
      __syncthreads();
    }
  }

  if (a.mode & MODE_RHS) {
    // y_i = L_ii^{-1} f_i
    if constexpr (TEAM >= 64 && !Lay::kGlobal) {
      wave_forward<ni>(A, fh, lane);
    } else {
      // (column-oriented, one barrier per column)
      for (int c = 0; c < ni; ++c) {
        const double yc = fh[c] / A[pk(c, c)];
        for (int i = c + 1 + lane; i < ni; i += TEAM) fh[i] -= A[pk(i, c)] * yc;
        __syncthreads();
        if (lane == 0) fh[c] = yc;
      }
      __syncthreads();
    }
    // y_b = L_bb^{-1} (f_b - L_bi y_i) (loops unrolled so that the loads run
    // ahead of the chain of sums)
    for (int b = lane; b < nb; b += TEAM) {
      double s = fh[ni + b];
      const double* rb = A + pk(ni + b, 0);
#pragma unroll 8
      for (int j = 0; j < ni; ++j) s -= rb[j] * fh[j];
      tb[b] = s;
    }
    __syncthreads();
    // static condensation keeps f_b - L_bi y_i (on boundary faces: their data g)
    for (int b = lane; b < nb; b += TEAM) {
      double s = tb[b];
      if (!a.stat) {
        s = 0.0;
        if constexpr (!Lay::kGlobal) {
          const double* lr = Li + pk(b, 0);
#pragma unroll 8
          for (int c = 0; c <= b; ++c) s += lr[c] * tb[c];
        } else {
          for (int c = 0; c <= b; ++c) s += LI(b, c) * tb[c];
        }
      }
      fh[ni + b] = s;
    }
    __syncthreads();
    if (live) {
      for (int i = lane; i < n; i += TEAM) a.y[e * n + i] = fh[i];
      // r_T = D L_bb^{-T} y_b, or (static condensation) sigma (f_b - L_bi y_i)
      for (int b = lane; b < nb; b += TEAM) {
        const int fb = b / K2;
        if (fid[fb] < 0) continue;
        double s;
        if (a.stat) {
          s = sigma(b) * fh[ni + b];
        } else {
          s = 0.0;
          if constexpr (!Lay::kGlobal) {
            int p = pk(b, b);
#pragma unroll 8
            for (int c = b; c < nb; ++c) {
              s += Li[p] * fh[ni + c];
              p += c + 1;
            }
          } else {
            for (int c = b; c < nb; ++c) s += LI(c, b) * fh[ni + c];
          }
          if (!(fb & 1)) s = -s;
        }
        int b0 = (b % K2) % K1, b1 = (b % K2) / K1;
        frame_map(pic[fb], K, b0, b1);
        if (!a.stat) s *= mp.face_w[b0 + K1 * b1];   // M_s r_T (weighted C)
        atomicAdd(&a.r[int64_t(fid[fb]) * K2 + b0 + K1 * b1], s);
      }
    }
  }

  if constexpr (!Lay::kGlobal) {
    if ((a.mode & MODE_MATRIX) && live) {
      for (int p = lane; p < R::npk; p += TEAM) {
        int i, j;
        unpk(p, i, j);
        a.factor[e * R::npk + p] = (i >= ni && j >= ni && !a.stat) ? Li[pk(i - ni, j - ni)] : A[p];
      }
    }
  }
}

// (RT2: at most 128 registers, two workgroups per CU; measured faster than
// the compiler's own choice, which takes one)
template <int K, int TEAM, int EPB>
__global__ __launch_bounds__(TEAM* EPB, K == 2 ? 4 : 2) void k_setup_generic(SetupArgs a) {
  __shared__ double smem[EPB * GenericLayout<K, TEAM, EPB>::per];
  setup_generic_body<K, TEAM, EPB>(a, smem, blockIdx.x);
}

// u_T = L^{-T} (y - [0; L_bb^{-1} D lambda_b]) from the stored factor; with
// static condensation u_b = sigma x_b and u_i = L_ii^{-T} (y_i - L_bi^T u_b).
// (k <= 2 also stage the factor's interior block, for a wave-level back
// substitution, and its face block, read by rows and by columns, with
// coalesced copies; for k = 3 the two would take 125 KB of LDS per element,
// one element per CU: measured 57 against 33 us per element for reading the
// record directly with many elements in flight per CU; RT2 the other way
// round: 5.0 us staged against 7.2 on the RT3 path with a wave per element)
template <int K>
constexpr bool recover_stages() { return K <= 2; }
// Recovery team (lanes per element) and elements per workgroup of order k.
// RT3 runs one wave per element: every step waits on record loads (the back
// substitution on one wave in any case), so the elements in flight per CU
// set the rate (16 with 64-lane teams, 4 with 256-lane ones).  RT2 stages
// 26 KB of the factor per element in LDS: 256-lane teams keep six elements
// per CU.
__host__ __device__ constexpr int recover_team(int k) { return k == 0 ? 16 : (k == 1 ? 64 : (k == 2 ? 256 : 64)); }
__host__ __device__ constexpr int recover_teams(int k) { return k == 0 ? 16 : (k == 1 ? 4 : (k == 2 ? 2 : 8)); }
template <int K>
constexpr int recover_per() {
  return 2 * RT<K>::n + RT<K>::nb + (recover_stages<K>() ? RT<K>::ni * (RT<K>::ni + 1) / 2 + RT<K>::nbpk : 0);
}

template <int K, int TEAM, int EPB>
__device__ __forceinline__ void recover_generic_body(const RecoverArgs& a, double* smem, int64_t blk,
                                                     int64_t e_end = INT64_MAX) {
  using R = RT<K>;
  constexpr int n = R::n, ni = R::ni, nb = R::nb, K1 = R::K1, K2 = R::K2;
  constexpr int per = recover_per<K>();
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  // element blk * EPB + team; blk counts elements instead when EPB is 1 and
  // several teams share the workgroup (elements blk, blk + 1, .., below e_end)
  const int64_t e = EPB == 1 ? blk + team : blk * EPB + team;
  const bool live = e < a.ne && e < e_end;
  const int64_t es = live ? e : 0;
  double* yv = smem + team * per;   // y, then v / u
  double* zb = yv + n;              // z_b, then u_b
  double* tl = zb + n;              // D lambda_b
  double* Lii = tl + nb;             // the factor's interior block (packed, leading)
  double* Lfb = Lii + ni * (ni + 1) / 2;   // its face block (packed)
  const double* F = a.factor + es * R::npk;
  const DeviceMaps& mp = a.mp;
  for (int i = lane; i < n; i += TEAM) yv[i] = a.y[es * n + i];
  if constexpr (recover_stages<K>()) {
    for (int t = lane; t < ni * (ni + 1) / 2; t += TEAM) Lii[t] = F[t];
    // face rows b: their entries c = 0..b of the face block are contiguous
    for (int t = lane; t < R::nbpk; t += TEAM) {
      int b, c;
      unpk(t, b, c);
      Lfb[t] = F[pk(ni + b, ni + c)];
    }
  }
  for (int b = lane; b < nb; b += TEAM) {
    const int fb = b / K2;
    const int F_ = mp.elem_face[es * 6 + fb];
    double v = 0.0;
    if (F_ >= 0) {
      int b0 = (b % K2) % K1, b1 = (b % K2) / K1;
      frame_map(mp.elem_pi[es * 8 + fb], K, b0, b1);
      v = a.lambda[int64_t(F_) * K2 + b0 + K1 * b1];
      if (a.stat) {
        // u_b = sigma x: the face dof is the owner's outward flux
        const double eps = (fb & 1) ? 1.0 : -1.0;
        v = mp.face_owner[F_] == es ? eps * v : -eps * v;
      } else {
        v *= mp.face_w[b0 + K1 * b1];   // C^T M_s lambda (weighted C)
        if (!(fb & 1)) v = -v;
      }
    } else if (a.stat) {
      v = yv[ni + b];  // boundary data
    }
    tl[b] = v;
  }
  __syncthreads();
  if constexpr (!recover_stages<K>() && TEAM == 64) {
    if (!a.stat) {
      // One wave per element, the face block read once, by rows (coalesced):
      // row c gives z_c = y_c - sum_{c' <= c} L_bb[c][c'] tl[c'] (a wave sum,
      // every lane the same value), then its terms L_bb[c][b] z_c of
      // u_b = sum_{c >= b} L_bb[c][b] z_c for the lanes' b = lane, lane + 64.
      static_assert(nb <= 128, "at most two face dofs per lane");
      const int b1 = lane + 64;
      const double t0 = lane < nb ? tl[lane] : 0.0, t1 = b1 < nb ? tl[b1] : 0.0;
      double u0 = 0.0, u1 = 0.0;
#pragma unroll 4
      for (int c = 0; c < nb; ++c) {
        const double* row = F + pk(ni + c, ni);   // entries 0..c of face row c
        const double l0 = row[lane <= c ? lane : c];
        const double l1 = row[b1 <= c ? b1 : c];
        const double m0 = lane <= c ? l0 : 0.0, m1 = b1 <= c ? l1 : 0.0;
        double p = m0 * t0 + m1 * t1;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, 64);
        const double zc = yv[ni + c] - p;
        u0 += m0 * zc;
        u1 += m1 * zc;
      }
      if (lane < nb) tl[lane] = u0;   // u_b
      if (b1 < nb) tl[b1] = u1;
    }
    __syncthreads();
  } else if (!a.stat) {
    // (loops unrolled so that the loads run ahead of the chain of sums)
    // (face row b: Lfb + pk(b, 0) in LDS, or F + pk(ni + b, ni) in the
    // record; column b steps by the row lengths in both)
    for (int b = lane; b < nb; b += TEAM) {
      double s = yv[ni + b];
      const double* fr = recover_stages<K>() ? Lfb + pk(b, 0) : F + pk(ni + b, ni);
#pragma unroll 8
      for (int c = 0; c <= b; ++c) s -= fr[c] * tl[c];
      zb[b] = s;
    }
    __syncthreads();
    for (int b = lane; b < nb; b += TEAM) {
      double s = 0.0;
      const double* fc = recover_stages<K>() ? Lfb + pk(b, b) : F + pk(ni + b, ni + b);
      int p = 0;
#pragma unroll 8
      for (int c = b; c < nb; ++c) {
        s += fc[p] * zb[c];
        p += (recover_stages<K>() ? c : ni + c) + 1;
      }
      tl[b] = s;  // u_b
    }
    __syncthreads();
  }
  {
    // z_j = y_j - sum_b L[ni + b][j] u_b for the lane's rows j = lane + TEAM r,
    // all of them in one pass over b (their loads issued together)
    constexpr int RPJ = (ni + TEAM - 1) / TEAM;
    double s[RPJ > 0 ? RPJ : 1];
#pragma unroll
    for (int r = 0; r < RPJ; ++r) {
      const int j = lane + TEAM * r;
      s[r] = j < ni ? yv[j] : 0.0;
    }
#pragma unroll 8
    for (int b = 0; b < (lane < ni ? nb : 0); ++b) {
      const double* row = F + pk(ni + b, 0);   // face row b: its L_bi part, columns j
      const double ub = tl[b];
#pragma unroll
      for (int r = 0; r < RPJ; ++r) {
        const int j = lane + TEAM * r;
        s[r] -= row[j < ni ? j : 0] * ub;
      }
    }
#pragma unroll
    for (int r = 0; r < RPJ; ++r) {
      const int j = lane + TEAM * r;
      if (j < ni) zb[j] = s[r];
    }
  }
  __syncthreads();
  if constexpr (TEAM >= 64 && recover_stages<K>()) {
    wave_backward<ni>(Lii, zb, lane);
  } else if constexpr (TEAM >= 64) {
    // one wave, the factor read from the record, 16 columns' loads in flight
    wave_backward<ni, 16>(F, zb, lane);
  } else {
    const double* Lb = recover_stages<K>() ? Lii : F;
    for (int c = ni - 1; c >= 0; --c) {
      const double uc = zb[c] / Lb[pk(c, c)];
      for (int j = lane; j < c; j += TEAM) zb[j] -= Lb[pk(c, j)] * uc;
      __syncthreads();
      if (lane == 0) zb[c] = uc;
    }
    __syncthreads();
  }
  if (live)
    for (int i = lane; i < n; i += TEAM) a.u[e * n + i] = i < ni ? zb[i] : tl[i - ni];
}

template <int K, int TEAM, int EPB>
__global__ __launch_bounds__(TEAM* EPB) void k_recover_generic(RecoverArgs a) {
  __shared__ double smem[EPB * recover_per<K>()];
  recover_generic_body<K, TEAM, EPB>(a, smem, blockIdx.x);
}

}  // namespace hyb
