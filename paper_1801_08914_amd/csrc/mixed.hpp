// Mixed-precision form of the element kernels (precision = HYB_MIXED).
//
// The element matrix M_T is assembled in FP64 (as in the plain form) and
// kept for the refinement residuals.  Its Cholesky factor is computed in FP32
// on the matrix cores after an exact power-of-two diagonal scaling S (S M_T S
// has its diagonal in [0.5, 2)): panels of 16 columns, the trailing lower
// tiles by v_mfma_f32_16x16x4f32.  X = M_T^{-1} C_T^T (the columns that give
// H_T, Sec. 3.1) and y = M_T^{-1} f_hat are then solved with the FP32 factor
// and refined: every sweep forms the residual B - M_T X on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64), solves for the correction in FP32 and adds
// it in FP64.  The triangular solves run by column tiles of 16, one wave per
// tile and no block barrier: each block of 16 rows is updated by the solved
// blocks on the matrix cores and multiplied by the inverse of its diagonal
// block (inverted once per factorization).  An element whose FP32 factor
// breaks down, or whose refinement fails the backward-error test, is solved
// in FP64 instead (its FP64 Cholesky and the same tile solves on the FP64
// matrix cores) and counted.  H_T = C_T X (symmetrized), its scatter into H,
// r_T = C_T y and the recovery u_T = y - X lambda_T are FP64.
//
// Element record: X only (n x nb, column-major, FP64): a right-hand side
// alone re-assembles M_T from the coefficients and re-derives the FP32
// factor, so the record is no larger than the FP64 form's (smaller for
// k = 3).  For k = 3 the FP64 element matrix (231 KB) and the FP32 work
// columns stay in a per-workgroup scratch slot in HBM (L2-resident while the
// element is processed); the FP32 factor is in LDS for every order.
#pragma once

#include "setup_generic.hpp"

namespace hyb {

// chol_tiles16 with the result in every lane of the team: true when a pivot
// was not positive (replaced by 1).  With active false the team only takes
// part in the barriers.  flag: one int of team LDS, rd: 16 T of team LDS.
template <class T, int N, int TEAM>
__device__ __forceinline__ bool chol_mfma_t(T* A, int lane, bool active, int* flag, T* rd) {
  __syncthreads();
  if (lane == 0) *flag = 0;
  const bool bad = chol_tiles16<T, N, TEAM>(A, rd, lane, active);
  if (active && lane == 0 && bad) *flag = 1;
  __syncthreads();
  const bool out = *flag != 0;
  __syncthreads();
  return out;
}

// W := (L L^T)^{-1} W (BACK) or L^{-1} W on one column tile (columns c0 ..
// c0 + ncol - 1 of W, ncol <= 16) by one wave: forward, then backward
// substitution by blocks of 16 rows; every block is first updated by the
// blocks already solved (on the matrix cores of T) and then multiplied by
// the inverse of its diagonal block.  Only this wave touches these columns of
// W (LDS or global), so wave-level ordering suffices.  L(i, j): the factor,
// j <= i < N.
template <class T, int N, bool BACK = true, class LAcc, class WAcc>
__device__ __forceinline__ void tile_solve(LAcc L, const T* Linv, WAcc W, int c0, int ncol, int l) {
  using M = MfmaT<T>;
  using v4 = typename M::v4;
  constexpr int NT = (N + 15) / 16;
  const int li = l & 15, lk = l >> 4;
  const int c = c0 + li;
  const bool cok = li < ncol;
  // loads at clamped (valid) positions, masked values: no lane-dependent
  // branch around the loads
  const int cc = cok ? c : c0;
  auto ld = [&](int i) -> T {
    const T v = static_cast<T>(W(i < N ? i : N - 1, cc));
    return (cok && i < N) ? v : T(0);
  };
  auto st = [&](int I, v4 v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + M::row(l, r);
      if (cok && i < N) W(i, c) = v[r];
    }
  };
  for (int I = 0; I < NT; ++I) {
    v4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = ld(16 * I + M::row(l, r));
    const int i = 16 * I + li, ic = i < N ? i : N - 1;
    // (unrolled: the operand loads of several blocks are in flight together)
#pragma unroll 4
    for (int J = 0; J < I; ++J) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int q = 16 * J + 4 * s + lk;
        const T lv = L(ic, q);
        acc = M::op(i < N ? -lv : T(0), ld(q), acc);
      }
    }
    st(I, acc);
    wave_sync();
    v4 x = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s) x = M::op(Linv[256 * I + 16 * li + 4 * s + lk], ld(16 * I + 4 * s + lk), x);
    wave_sync();
    st(I, x);
    wave_sync();
  }
  if constexpr (!BACK) return;
  for (int I = NT - 1; I >= 0; --I) {
    v4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = ld(16 * I + M::row(l, r));
    const int j = 16 * I + li;
#pragma unroll 4
    for (int K = I + 1; K < NT; ++K) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int q = 16 * K + 4 * s + lk;
        const T lv = L(q < N ? q : N - 1, j);
        acc = M::op(q < N ? -lv : T(0), ld(q), acc);
      }
    }
    st(I, acc);
    wave_sync();
    v4 x = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s) x = M::op(Linv[256 * I + 16 * (4 * s + lk) + li], ld(16 * I + 4 * s + lk), x);
    wave_sync();
    st(I, x);
    wave_sync();
  }
}

// R = B - M X (FP64) on the output tiles (16 rows x 16 columns) dealt to the
// team's waves; out(i, c, R) receives every entry i < N, c < ncol.  Returns
// the lane's largest |R|.  Mf(i, j): the symmetric FP64 matrix, any i, j < N.
template <int N, int TEAM, class MAcc, class XAcc, class BFn, class Out>
__device__ __forceinline__ double residual_tiles(MAcc Mf, XAcc X, BFn B, Out out, int ncol, int lane) {
  using M = MfmaT<double>;
  constexpr int NT = (N + 15) / 16, NW = TEAM / 64;
  const int w_id = lane / 64, l = lane % 64, li = l & 15, lk = l >> 4;
  const int CT = (ncol + 15) / 16;
  double rm = 0.0;
  for (int t = w_id; t < NT * CT; t += NW) {
    const int I = t / CT, c = 16 * (t % CT) + li;
    const bool cok = c < ncol;
    const int ia = 16 * I + li;
    dx4 acc = {0.0, 0.0, 0.0, 0.0};
    const int iac = ia < N ? ia : N - 1, cc = cok ? c : 0;
#pragma unroll 4
    for (int J = 0; J < NT; ++J) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        // loads at clamped (valid) positions, masked values
        const int q = 16 * J + 4 * s + lk, qc = q < N ? q : N - 1;
        const double av = Mf(iac, qc), bv = static_cast<double>(X(qc, cc));
        acc = M::op((ia < N && q < N) ? av : 0.0, (cok && q < N) ? bv : 0.0, acc);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + M::row(l, r);
      if (cok && i < N) {
        const double R = B(i, c) - acc[r];
        rm = fmax(rm, fabs(R));
        out(i, c, R);
      }
    }
  }
  return rm;
}

// Sweep control of the refinement.  sweeps >= 0: exactly that many sweeps
// after the FP32 solve.  sweeps < 0 (adaptive): sweep while the correction
// keeps shrinking (the classical forward-error rule: stop once
// ||dx||_inf <= 2^-53 ||x||_inf, or once a correction is more than half the
// previous one, the FP64 floor kappa 2^-53 reached), at most kRefineMax
// sweeps; the result is accepted if the FP64 residual then passes the
// backward-error test ||b - M x||_inf <= sqrt(n) 2^-53 ||M||_inf ||x||_inf
// (the test of LAPACK's mixed-precision Cholesky solver), otherwise the
// element is solved in FP64.
constexpr int kRefineMax = 30;

// Team-wide maximum of non-negative doubles through their bit patterns
// (monotonic for non-negative values) in LDS.
__device__ __forceinline__ void team_max(double* slot, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(slot), static_cast<unsigned long long>(__double_as_longlong(v)));
}

// ||M||_inf of the N x N matrix given by mrow, by the team (red: 1 double of
// team scratch).  Starts and ends with a barrier.
template <int N, int TEAM, class MRow>
__device__ __forceinline__ double norm_inf(MRow mrow, double* red, int lane) {
  __syncthreads();
  if (lane == 0) red[0] = 0.0;
  __syncthreads();
  double m = 0.0;
  for (int i = lane; i < N; i += TEAM) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += fabs(mrow(i, j));
    m = fmax(m, s);
  }
  team_max(red, m);
  __syncthreads();
  const double out = red[0];
  __syncthreads();
  return out;
}

// M X = B for ncol columns with the FP32 factor (L, diagonal-block inverses
// Li) and FP64 refinement: the first solve for S B, every later sweep for
// the residual B - M X (FP64 matrix cores), its correction added in FP64.
// W: FP32 work columns (same shape as X).  red: 8 doubles of team scratch.
// Returns false when an adaptive refinement fails the backward-error test.
// A team with active false takes part in the barriers only; the block leaves
// the sweep loop together (barriers stay paired across the teams of a block).
template <int N, int TEAM, class LAcc, class WAcc, class XAcc, class BFn, class MAcc>
__device__ __forceinline__ bool refine_cols(LAcc L, const float* Li, WAcc W, XAcc X, BFn B, MAcc Mf,
                                            const double* Sv, int ncol, int sweeps, double anrm, double* red,
                                            int lane, bool active) {
  constexpr int NW = TEAM / 64;
  const int w_id = lane / 64, l = lane % 64;
  const int CT = (ncol + 15) / 16;
  const bool adaptive = sweeps < 0;
  const int cap = adaptive ? kRefineMax : sweeps;
  const double tol = sqrt(double(N)) * 0x1p-53 * anrm;
  const int tot = active ? N * ncol : 0;
  __syncthreads();  // the team is done with red and W
  if (lane < 8) red[lane] = 0.0;
  for (int t = lane; t < tot; t += TEAM) {
    const int i = t / ncol, c = t % ncol;
    W(i, c) = float(Sv[i] * B(i, c));
  }
  __syncthreads();
  for (int ct = active ? w_id : CT; ct < CT; ct += NW)
    tile_solve<float, N>(L, Li, W, 16 * ct, ncol - 16 * ct < 16 ? ncol - 16 * ct : 16, l);
  __syncthreads();
  double xm = 0.0, zm = 0.0, zprev = 0.0;
  for (int t = lane; t < tot; t += TEAM) {
    const int i = t / ncol, c = t % ncol;
    const double x = Sv[i] * double(W(i, c));
    X(i, c) = x;
    xm = fmax(xm, fabs(x));
  }
  bool done = !active || (!adaptive && cap == 0), result = true;
  for (int sw = 1;; ++sw) {
    if (!__syncthreads_or(done ? 0 : 1)) return result;
    double* slot = red + 4 * (sw & 1);
    if (adaptive && !done) {
      team_max(slot + 1, xm);
      team_max(slot + 2, zm);
    }
    __syncthreads();  // X complete
    double rm = 0.0;
    if (!done)
      rm = residual_tiles<N, TEAM>(Mf, X, B, [&](int i, int c, double R) { W(i, c) = float(Sv[i] * R); }, ncol,
                                   lane);
    if (adaptive && !done) team_max(slot, rm);
    __syncthreads();
    // every lane has read the other slot in the previous sweep
    if (lane < 4) red[4 * ((sw + 1) & 1) + lane] = 0.0;
    if (!done) {
      if (adaptive) {
        // slot: residual and size of the current x, the correction that made it
        const bool backward_ok = slot[0] <= tol * slot[1];
        if ((sw >= 2 && slot[2] <= 0x1p-53 * slot[1]) || (sw >= 3 && slot[2] > 0.5 * zprev) || sw > cap) {
          done = true;
          result = backward_ok;
        }
        zprev = slot[2];
      } else if (sw >= cap) {
        done = true;   // the last correction below is still applied
      }
    }
    const bool solve_now = !done || (!adaptive && sw == cap);
    if (!__syncthreads_or(solve_now ? 1 : 0)) return result;
    for (int ct = solve_now ? w_id : CT; ct < CT; ct += NW)
      tile_solve<float, N>(L, Li, W, 16 * ct, ncol - 16 * ct < 16 ? ncol - 16 * ct : 16, l);
    __syncthreads();
    xm = zm = 0.0;
    for (int t = solve_now ? lane : tot; t < tot; t += TEAM) {
      const int i = t / ncol, c = t % ncol;
      const double z = Sv[i] * double(W(i, c));
      const double x = X(i, c) + z;
      X(i, c) = x;
      xm = fmax(xm, fabs(x));
      zm = fmax(zm, fabs(z));
    }
  }
}

template <int K>
struct MixedRec {
  using R = RT<K>;
  static constexpr int64_t x = 0;                        // X, n x nb column-major
  static constexpr int64_t len = int64_t(R::n) * R::nb;
};

// Per-element LDS (doubles) and, for k = 3, the per-workgroup HBM scratch
// slot.  Regions: M64 (packed FP64 element matrix; k = 3: in the slot), X64
// (n x nb row-major FP64; k = 3: the record), FW (the packed FP32 factor,
// then the FP32 work columns; the FP64 fallback factor over both; the
// assembly's staging tables before the factor), Li (inverses of the FP32
// factor's diagonal blocks; the FP64 ones where M64 cannot hold them),
// per-point terms, f_hat, S, y, corners, reduction slots.
template <int K, int TEAM, int EPB>
struct MixedLayout {
  using R = RT<K>;
  static constexpr int n = R::n, nb = R::nb, NT = (n + 15) / 16;
  static constexpr bool kGlobal = K >= 3;
  static constexpr int l32 = (R::npk + 1) / 2;            // packed FP32 factor
  static constexpr int w32 = (n * nb + 1) / 2;            // FP32 work columns
  static constexpr int fw_min = kGlobal ? l32 : (l32 + w32 > R::npk ? l32 + w32 : R::npk);
  static constexpr int QC = kGlobal ? kAsmQC : (fw_min / (2 * n) < kAsmQC ? fw_min / (2 * n) : kAsmQC);
  static constexpr int fw = fw_min > 2 * n * QC ? fw_min : 2 * n * QC;
  // FP64 inverses of the diagonal blocks: in M64 (k <= 2, when they fit), in
  // FW after the HBM Cholesky's panel (k = 3), else in Li
  static constexpr int li64 = NT * 256;
  static constexpr bool li64_in_m = !kGlobal && li64 <= R::npk;
  static constexpr int hbm_panel = 32 * (n | 1);
  static constexpr int li = (kGlobal || li64_in_m) ? NT * 128 : li64;
  static constexpr int m64 = kGlobal ? 0 : R::npk;
  static constexpr int x64 = kGlobal ? 0 : n * nb;
  static constexpr int per = m64 + x64 + fw + li + R::Q * 10 + 3 * n + 24 + 32;
  // HBM scratch per workgroup (k = 3): M64 and the FP32 work columns
  static constexpr int64_t slot = kGlobal ? int64_t(R::npk) + w32 : 0;
  static_assert(!kGlobal || fw >= hbm_panel + li64, "the HBM Cholesky's panel and FP64 block inverses fit in FW");
  static_assert(kGlobal || fw >= R::npk, "the FP64 fallback factor fits in FW");
  static_assert(!kGlobal || EPB == 1, "a scratch slot per element in flight: one element per block");
  static_assert(QC >= 1, "assembly staging");
};

// Workgroups of the k = 3 persistent launch (one scratch slot each).
constexpr int kMixedSlots = 512;

// The mixed element routine: setup (MODE_MATRIX: M_T, the FP32 factor, X,
// H_T into H) and/or right-hand side (MODE_RHS: f_hat, y, r_T into r; alone,
// M_T and the FP32 factor are derived again from the coefficients).  scratch:
// the workgroup's HBM slot (k = 3), fallbacks: counter of elements solved in
// FP64.
template <int K, int TEAM, int EPB>
__device__ __forceinline__ void setup_mixed_body(const SetupArgs& a, double* smem, int64_t blk, int sweeps,
                                                 double* scratch) {
  using R = RT<K>;
  using Lay = MixedLayout<K, TEAM, EPB>;
  using Rec = MixedRec<K>;
  constexpr int n = R::n, ni = R::ni, nb = R::nb, K1 = R::K1, K2 = R::K2, Q = R::Q, QD = 10, NT = Lay::NT;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int w_id = lane / 64, l = lane % 64;
  constexpr int NW = TEAM / 64;
  const int64_t e = blk * EPB + team;
  const bool live = e < a.ne;
  const int64_t es = live ? e : 0;  // safe index for loads of padding teams
  const bool matrix = (a.mode & MODE_MATRIX) != 0, rhs = (a.mode & MODE_RHS) != 0;
  double* rec = a.factor + es * Rec::len;
  double* base = smem + team * Lay::per;
  double* M64 = Lay::kGlobal ? scratch : base;
  double* X64 = Lay::kGlobal ? nullptr : base + Lay::m64;
  double* FW = base + Lay::m64 + Lay::x64;
  float* L32 = reinterpret_cast<float*>(FW);
  float* W32 = Lay::kGlobal ? reinterpret_cast<float*>(scratch + R::npk) : L32 + 2 * Lay::l32;
  double* Li = FW + Lay::fw;
  float* Li32 = reinterpret_cast<float*>(Li);
  double* qd = Li + Lay::li;
  double* fh = qd + Q * QD;
  double* Sv = fh + n;
  double* yv = Sv + n;
  double* xe = yv + n;
  double* red = xe + 24;
  int* flag = reinterpret_cast<int*>(red + 12);
  double* rdv = red + 16;   // the Cholesky's pivot reciprocals (16)
  const DeviceMaps& mp = a.mp;

  auto Mrow = [&](int i, int j) { return i >= j ? M64[pk(i, j)] : M64[pk(j, i)]; };
  auto L32a = [&](int i, int j) -> float { return L32[pk(i, j)]; };
  // X: n x nb, row-major in LDS (k <= 2) or the record's column-major array
  auto Xe = [&](int i, int c) -> double& { return Lay::kGlobal ? rec[int64_t(c) * n + i] : X64[i * nb + c]; };
  auto Wx = [&](int i, int c) -> float& { return W32[i * nb + c]; };
  auto Wy = [&](int i, int) -> float& { return W32[i]; };
  auto Y = [&](int i, int) -> double& { return yv[i]; };

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
  // sign of face dof b in C_T: +1 on the max side of an axis, -1 on the min side
  auto eps = [&](int b) { return ((b / K2) & 1) ? 1.0 : -1.0; };
  auto Bx = [&](int i, int c) { return i == ni + c ? eps(c) : 0.0; };
  auto By = [&](int i, int) { return fh[i]; };

  const double al = a.alpha ? a.alpha[es] : 0.0, be = a.beta ? a.beta[es] : 0.0;
  double fv[3] = {0.0, 0.0, 0.0};
  if (rhs) {
    fv[0] = a.f[es * 3 + 0]; fv[1] = a.f[es * 3 + 1]; fv[2] = a.f[es * 3 + 2];
  }
  element_qd<K, TEAM>(mp, es, al, be, fv, true, rhs, xe, qd, lane, live, a.status, e);

  // M_T (FP64, packed lower): by sum factorization (k = 3) or the dense sum
  // on the matrix cores; the partial sums or tables staged in FW
  if constexpr (use_sumfact<K>()) {
    static_assert(Lay::fw >= sumfact_stage<K>(), "the sum factorization's partial sums fit in FW");
    assemble_sumfact<K, TEAM>(mp, qd, FW, lane, [&](int i, int j, double v) { M64[pk(i, j)] = v; });
  } else {
    assemble_mfma<K, TEAM, Lay::QC>(mp, qd, FW, lane, [&](int i, int j, double v) { M64[pk(i, j)] = v; });
  }
  __syncthreads();
  if (rhs) {
    // f_hat, with f_r -= M_re g_e from the unmasked matrix
    for (int i = lane; i < n; i += TEAM) {
      const int d = R::comp(i);
      double s = 0.0;
#pragma unroll 8
      for (int q = 0; q < Q; ++q) s += mp.tab_s[q * n + i] * qd[q * QD + 7 + d];
      if (is_ess(i)) {
        s = a.g ? a.g[es * nb + (i - ni)] : 0.0;
      } else if (a.g) {
        for (int j = ni; j < n; ++j)
          if (is_ess(j)) s -= Mrow(i, j) * a.g[es * nb + (j - ni)];
      }
      fh[i] = s;
    }
    __syncthreads();
  }
  // essential rows/columns -> identity; power-of-two scaling; FP32 copy
  for (int p = lane; p < R::npk; p += TEAM) {
    int i, j;
    unpk(p, i, j);
    if (is_ess(i) || is_ess(j)) M64[p] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = lane; i < n; i += TEAM) {
    int ex;
    (void)frexp(M64[pk(i, i)], &ex);
    Sv[i] = ldexp(1.0, -(ex >> 1));
  }
  __syncthreads();
  for (int p = lane; p < R::npk; p += TEAM) {
    int i, j;
    unpk(p, i, j);
    L32[p] = float(Sv[i] * M64[p] * Sv[j]);
  }
  const double anrm = norm_inf<n, TEAM>(Mrow, red + 10, lane);
  // FP32 Cholesky of S M_T S; a breakdown means kappa(S M_T S) 2^-24 >= 1
  // (or M_T is not SPD): such an element is solved in FP64
  const bool broke = chol_mfma_t<float, n, TEAM>(L32, lane, true, flag, reinterpret_cast<float*>(rdv));
  diag_inverses<float, n, TEAM>(L32a, Li32, lane, !broke);
  __syncthreads();

  // (every team of the block runs the calls: they hold block barriers)
  bool ok_y = true, ok_x = true;
  if (rhs) {
    const bool r = refine_cols<n, TEAM>(L32a, Li32, Wy, Y, By, Mrow, Sv, 1, sweeps, anrm, red, lane, !broke);
    ok_y = !broke && r;
  }
  if (matrix) {
    const bool r = refine_cols<n, TEAM>(L32a, Li32, Wx, Xe, Bx, Mrow, Sv, nb, sweeps, anrm, red, lane, !broke);
    ok_x = !broke && r;
  }

  // FP64 for what FP32 could not do: Cholesky of M_T (FP64 matrix cores), the
  // same tile solves in FP64 (block-uniform branch; the other teams of the
  // block take part in the barriers)
  const bool fb = !(ok_x && ok_y);
  if (__syncthreads_or(fb ? 1 : 0)) {
    double* F = Lay::kGlobal ? M64 : FW;
    double* Li64 = Lay::kGlobal ? FW + Lay::hbm_panel : (Lay::li64_in_m ? M64 : Li);
    bool notspd;
    if constexpr (Lay::kGlobal) {
      notspd = chol_hbm32<n, TEAM>(F, FW, lane, fb);
      __syncthreads();
    } else {
      for (int p = fb ? lane : R::npk; p < R::npk; p += TEAM) F[p] = M64[p];
      notspd = chol_mfma_t<double, n, TEAM>(F, lane, fb, flag, rdv);
    }
    if (fb && notspd && live && lane == 0) report_error(a.status, HYB_E_NOT_SPD, e);
    auto Fa = [&](int i, int j) -> double { return F[pk(i, j)]; };
    diag_inverses<double, n, TEAM>(Fa, Li64, lane, fb);
    __syncthreads();
    if (fb && !ok_y) {
      for (int i = lane; i < n; i += TEAM) yv[i] = fh[i];
    }
    if (fb && !ok_x) {
      for (int t = lane; t < n * nb; t += TEAM) Xe(t / nb, t % nb) = Bx(t / nb, t % nb);
    }
    __syncthreads();
    if (fb && !ok_y && w_id == 0) tile_solve<double, n>(Fa, Li64, Y, 0, 1, l);
    if (fb && !ok_x) {
      constexpr int CT = (nb + 15) / 16;
      for (int ct = w_id; ct < CT; ct += NW) tile_solve<double, n>(Fa, Li64, Xe, 16 * ct, nb - 16 * ct < 16 ? nb - 16 * ct : 16, l);
    }
    __syncthreads();
    if (fb && live && lane == 0) atomicAdd(reinterpret_cast<int*>(a.status) + 2, 1);
  }

  if (matrix && live) {
    // H_T = D (M^{-1})_bb D = D E_b^T X, symmetrized, scattered into H (same-
    // face blocks receive two element terms by atomic add)
    for (int t = lane; t < R::nbpk; t += TEAM) {
      int aa, bb;
      unpk(t, aa, bb);
      const int fa = aa / K2, fb2 = bb / K2;
      if (fid[fa] < 0 || fid[fb2] < 0) continue;
      const double v = 0.5 * (eps(aa) * Xe(ni + aa, bb) + eps(bb) * Xe(ni + bb, aa));
      int a0 = (aa % K2) % K1, a1 = (aa % K2) / K1, b0 = (bb % K2) % K1, b1 = (bb % K2) / K1;
      frame_map(pic[fa], K, a0, a1);
      frame_map(pic[fb2], K, b0, b1);
      const int ja = a0 + K1 * a1, jb = b0 + K1 * b1;
      const int Fa = fid[fa], Fb = fid[fb2];
      const double vw = v * (mp.face_w[ja] * mp.face_w[jb]);   // M_s H_T M_s (weighted C)
      const int64_t pab = mp.face_rowbase[Fa] + int64_t(ja) * mp.face_nslots[Fa] * K2 +
                          mp.elem_slot[e * 36 + fa * 6 + fb2] * K2 + jb;
      const int64_t pba = mp.face_rowbase[Fb] + int64_t(jb) * mp.face_nslots[Fb] * K2 +
                          mp.elem_slot[e * 36 + fb2 * 6 + fa] * K2 + ja;
      if (fa == fb2) {
        atomicAdd(&a.Hval[pab], vw);
        if (aa != bb) atomicAdd(&a.Hval[pba], vw);
      } else {
        a.Hval[pab] = vw;
        a.Hval[pba] = vw;
      }
    }
    if constexpr (!Lay::kGlobal) {
      for (int t = lane; t < n * nb; t += TEAM) rec[t] = X64[(t % n) * nb + t / n];
    }
  }
  if (rhs && live) {
    for (int i = lane; i < n; i += TEAM) a.y[e * n + i] = yv[i];
    // r_T = D y_b
    for (int b = lane; b < nb; b += TEAM) {
      const int fb2 = b / K2;
      if (fid[fb2] < 0) continue;
      int b0 = (b % K2) % K1, b1 = (b % K2) / K1;
      frame_map(pic[fb2], K, b0, b1);
      atomicAdd(&a.r[int64_t(fid[fb2]) * K2 + b0 + K1 * b1], eps(b) * yv[ni + b] * mp.face_w[b0 + K1 * b1]);
    }
  }
}

template <int K, int TEAM, int EPB>
__global__ __launch_bounds__(TEAM* EPB) void k_setup_mixed(SetupArgs a, int sweeps) {
  __shared__ double smem[EPB * MixedLayout<K, TEAM, EPB>::per];
  setup_mixed_body<K, TEAM, EPB>(a, smem, blockIdx.x, sweeps, nullptr);
}

// k = 3: a persistent grid, workgroup b owning scratch slot b.
template <int K, int TEAM>
__global__ __launch_bounds__(TEAM) void k_setup_mixed_slots(SetupArgs a, int sweeps, double* scratch) {
  __shared__ double smem[MixedLayout<K, TEAM, 1>::per];
  double* slot = scratch + int64_t(blockIdx.x) * MixedLayout<K, TEAM, 1>::slot;
  for (int64_t e = blockIdx.x; e < a.ne; e += gridDim.x) {
    setup_mixed_body<K, TEAM, 1>(a, smem, e, sweeps, slot);
    __syncthreads();
  }
}

// u_T = y - X lambda_T, lambda_T the element's face multipliers in its own
// frame (0 on boundary faces); X carries the signs of C_T.  smem: EPB * nb
// doubles.
template <int K, int TEAM, int EPB>
__device__ __forceinline__ void recover_mixed_body(const RecoverArgs& a, double* smem, int64_t blk) {
  using R = RT<K>;
  using Rec = MixedRec<K>;
  constexpr int n = R::n, nb = R::nb, K1 = R::K1, K2 = R::K2;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t e = blk * EPB + team;
  const bool live = e < a.ne;
  const int64_t es = live ? e : 0;
  double* tl = smem + team * nb;
  const DeviceMaps& mp = a.mp;
  for (int b = lane; b < nb; b += TEAM) {
    const int fb = b / K2;
    const int F = mp.elem_face[es * 6 + fb];
    double v = 0.0;
    if (F >= 0) {
      int b0 = (b % K2) % K1, b1 = (b % K2) / K1;
      frame_map(mp.elem_pi[es * 8 + fb], K, b0, b1);
      v = a.lambda[int64_t(F) * K2 + b0 + K1 * b1] * mp.face_w[b0 + K1 * b1];
    }
    tl[b] = v;
  }
  __syncthreads();
  if (live) {
    const double* X = a.factor + es * Rec::len + Rec::x;
    for (int i = lane; i < n; i += TEAM) {
      double s = a.y[es * n + i];
      for (int b = 0; b < nb; ++b) s -= X[int64_t(b) * n + i] * tl[b];
      a.u[es * n + i] = s;
    }
  }
}

template <int K, int TEAM, int EPB>
__global__ __launch_bounds__(TEAM* EPB) void k_recover_mixed(RecoverArgs a) {
  __shared__ double tl_all[EPB * RT<K>::nb];
  recover_mixed_body<K, TEAM, EPB>(a, tl_all, blockIdx.x);
}

}  // namespace hyb
