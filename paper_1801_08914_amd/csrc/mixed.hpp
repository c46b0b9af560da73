// Mixed-precision form of the element kernels.  The element matrix M_T is
// assembled in FP64 (as in the plain form); its Cholesky factor is computed
// in FP32 after an exact power-of-two diagonal scaling S (S M_T S has its
// diagonal in [0.5, 2)).  X = M_T^{-1} C_T^T (the columns that give H_T) and
// y = M_T^{-1} f_hat are solved with the FP32 factor and refined: each sweep
// forms the residual against the FP64 M_T in FP64, solves for the correction
// in FP32 and adds it in FP64 (a fixed number of sweeps, or while the
// correction keeps shrinking).  H_T = C_T X (symmetrized), its scatter into
// H, r_T = C_T y and the recovery u_T = y - X lambda_T are FP64.
//
// Element record (offsets in doubles): X (n x nb, column-major, FP64), M_T
// (packed lower, FP64, essential rows and columns replaced by the identity),
// the FP32 factor of S M_T S (packed lower, two per double) and S (n).
#pragma once

#include "setup_generic.hpp"

namespace hyb {

template <int K>
struct MixedRec {
  using R = RT<K>;
  static constexpr int64_t x = 0;
  static constexpr int64_t m64 = int64_t(R::n) * R::nb;
  static constexpr int64_t l32 = m64 + R::npk;
  static constexpr int64_t sc = l32 + (R::npk + 1) / 2;
  static constexpr int64_t len = sc + R::n;
};

// Per-element LDS (doubles).  From k = 3 on, M_T and X stay in the element's
// HBM record (L2-resident while the element is processed) and the FP32 solves
// run over chunks of CH columns.  X's column stride in LDS is odd, so that
// lanes on consecutive columns hit different banks.
template <int K, int TEAM, int EPB>
struct MixedLayout {
  using R = RT<K>;
  static constexpr bool kGlobal = K >= 3;
  static constexpr int CH = K >= 3 ? 16 : R::nb;
  static constexpr int XS = kGlobal ? R::n : (R::n | 1);
  static constexpr int l32 = (R::npk + 1) / 2;
  static constexpr int w32 = (R::n * CH + 1) / 2;
  static constexpr int d32 = (R::n + 1) / 2;
  // the assembly stages its tables in W (free until the solves): QC points
  static constexpr int QC = (2 * w32) / (4 * R::n) >= 1 ? (2 * w32) / (4 * R::n) : 1;
  static constexpr int per = l32 + w32 + d32 + (kGlobal ? 0 : R::npk + XS * R::nb) + R::Q * 10 + 3 * R::n + 24 + 10;
  static_assert(2 * R::n * QC <= w32, "assembly staging fits in W");
  static_assert(!kGlobal || EPB == 1, "an HBM-resident element matrix needs one element per block");
  static_assert(R::nb % CH == 0, "whole column chunks");
};

// Inverse of pk in FP32 arithmetic (exact after the correction steps for the
// packed sizes here, t < 2^24).
__device__ __forceinline__ void unpk_f(int t, int& i, int& j) {
  int r = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  i = r;
  j = t - r * (r + 1) / 2;
}

// W (N x NC, row-major, FP32) := (L L^T)^{-1} W with the packed FP32 factor
// L and the reciprocals dinv of its diagonal; one barrier per column in each
// direction.  Expects W complete on entry, ends with a barrier.  A team with
// active false only takes part in the barriers.
template <int N, int TEAM, int NC>
__device__ __forceinline__ void chol_solve32(const float* L, const float* dinv, float* W, int lane,
                                             bool active = true) {
  const int l0 = active ? lane : (1 << 30);
  for (int c = 0; c < N; ++c) {
    const float rc = dinv[c];
    for (int t = l0; t < (N - c - 1) * NC; t += TEAM) {
      const int i = c + 1 + t / NC, col = t % NC;
      W[i * NC + col] -= L[pk(i, c)] * (W[c * NC + col] * rc);
    }
    __syncthreads();
    // row c is not touched by later forward steps
    for (int col = l0; col < NC; col += TEAM) W[c * NC + col] *= rc;
  }
  __syncthreads();
  for (int c = N - 1; c >= 0; --c) {
    const float rc = dinv[c];
    for (int t = l0; t < c * NC; t += TEAM) {
      const int i = t / NC, col = t % NC;
      W[i * NC + col] -= L[pk(c, i)] * (W[c * NC + col] * rc);
    }
    __syncthreads();
    for (int col = l0; col < NC; col += TEAM) W[c * NC + col] *= rc;
  }
  __syncthreads();
}

// Sweep control of the refinement.  sweeps >= 0: exactly that many sweeps
// after the FP32 solve.  sweeps < 0 (adaptive): sweep while the correction
// keeps shrinking (the classical forward-error rule: stop once
// ||dx||_inf <= 2^-53 ||x||_inf, or once a correction is more than half the
// previous one, the FP64 floor kappa 2^-53 reached), at most kRefineMax
// sweeps; the result is accepted if the FP64 residual then passes the
// backward-error test ||b - M x||_inf <= sqrt(n) 2^-53 ||M||_inf ||x||_inf
// (the test of LAPACK's mixed-precision Cholesky solver), otherwise the
// element is reported (kappa(S M_T S) 2^-24 near 1), not hidden.
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

// Solve M X = B for NC columns with the FP32 factor and FP64 refinement:
// sweep 0 solves for B, every later sweep for the residual B - M X (FP64,
// from mrow), the correction added in FP64.  bcol(i, c) and xel(i, c) give
// B and X for local column c; anrm = ||M||_inf; red holds 8 doubles of team
// scratch (two slots of max |residual|, max |x|, max |correction|).  Returns
// false when an adaptive refinement did not pass the backward-error test.
template <int N, int TEAM, int NC, class MRow, class BCol, class XEl>
__device__ __forceinline__ bool refine_solve(const float* L, const float* dinv, float* W, const double* Sv,
                                             MRow mrow, BCol bcol, XEl xel, int sweeps, double anrm, double* red,
                                             int lane) {
  const bool adaptive = sweeps < 0;
  const int cap = adaptive ? kRefineMax : sweeps;
  const double tol = sqrt(double(N)) * 0x1p-53 * anrm;
  __syncthreads();  // the team is done with red and W
  if (lane < 8) red[lane] = 0.0;
  for (int t = lane; t < N * NC; t += TEAM) {
    const int i = t / NC, c = t % NC;
    W[i * NC + c] = float(Sv[i] * bcol(i, c));
  }
  __syncthreads();
  chol_solve32<N, TEAM, NC>(L, dinv, W, lane);
  double xm = 0.0, zm = 0.0, zprev = 0.0;
  for (int t = lane; t < N * NC; t += TEAM) {
    const int i = t / NC, c = t % NC;
    const double x = Sv[i] * double(W[i * NC + c]);
    xel(i, c) = x;
    xm = fmax(xm, fabs(x));
  }
  // A team whose refinement has ended keeps taking part in the block's
  // barriers (its work masked off) until every team of the block is done:
  // the block leaves the loop together, so barriers stay paired across teams
  // (in a persistent batch block the teams go on to other work items, whose
  // LDS layout may differ).
  bool done = false, result = true;
  for (int sw = 1;; ++sw) {
    double* slot = red + 4 * (sw & 1);
    if (adaptive && !done) {
      team_max(slot + 1, xm);
      team_max(slot + 2, zm);
    }
    __syncthreads();  // x complete
    double rm = 0.0;
    for (int t = done ? N * NC : lane; t < N * NC; t += TEAM) {
      const int i = t / NC, c = t % NC;
      double res = bcol(i, c);
      for (int j = 0; j < N; ++j) res -= mrow(i, j) * xel(j, c);
      rm = fmax(rm, fabs(res));
      W[i * NC + c] = float(Sv[i] * res);
    }
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
      } else if (sw > cap) {
        done = true;
      }
    }
    if (!__syncthreads_or(done ? 0 : 1)) return result;
    chol_solve32<N, TEAM, NC>(L, dinv, W, lane, !done);
    xm = zm = 0.0;
    for (int t = done ? N * NC : lane; t < N * NC; t += TEAM) {
      const int i = t / NC, c = t % NC;
      const double z = Sv[i] * double(W[i * NC + c]);
      const double x = xel(i, c) + z;
      xel(i, c) = x;
      xm = fmax(xm, fabs(x));
      zm = fmax(zm, fabs(z));
    }
  }
}

template <int K, int TEAM, int EPB>
__device__ __forceinline__ void setup_mixed_body(const SetupArgs& a, double* smem, int64_t blk, int sweeps) {
  using R = RT<K>;
  using Lay = MixedLayout<K, TEAM, EPB>;
  using Rec = MixedRec<K>;
  constexpr int n = R::n, ni = R::ni, nb = R::nb, K1 = R::K1, K2 = R::K2, Q = R::Q, QD = 10;
  constexpr int CH = Lay::CH, XS = Lay::XS;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t e = blk * EPB + team;
  const bool live = e < a.ne;
  const int64_t es = live ? e : 0;  // safe index for loads of padding teams
  const bool matrix = (a.mode & MODE_MATRIX) != 0, rhs = (a.mode & MODE_RHS) != 0;
  double* rec = a.factor + es * Rec::len;
  double* base = smem + team * Lay::per;
  float* L = reinterpret_cast<float*>(base);
  float* W = reinterpret_cast<float*>(base + Lay::l32);
  float* dinv = reinterpret_cast<float*>(base + Lay::l32 + Lay::w32);
  double* rest = base + Lay::l32 + Lay::w32 + Lay::d32;
  double* Ml = rest;
  double* Xl = rest + (Lay::kGlobal ? 0 : R::npk);
  double* qd = Xl + (Lay::kGlobal ? 0 : XS * nb);
  double* fh = qd + Q * QD;
  double* yv = fh + n;
  double* Sv = yv + n;
  double* xe = Sv + n;
  double* red = xe + 24;
  // the FP64 matrix: in LDS while a setup assembles it (k <= 2), else the record's
  double* M = (matrix && !Lay::kGlobal) ? Ml : rec + Rec::m64;
  double* X = Lay::kGlobal ? rec + Rec::x : Xl;
  auto Mrow = [&](int i, int j) { return i >= j ? M[pk(i, j)] : M[pk(j, i)]; };
  auto Xe = [&](int i, int b) -> double& { return X[b * XS + i]; };
  const DeviceMaps& mp = a.mp;

  int fid[6], pic[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    fid[f] = mp.elem_face[es * 6 + f];
    pic[f] = mp.elem_pi[es * 8 + f];
  }
  auto is_ess = [&](int i) { return i >= ni && fid[(i - ni) / K2] < 0; };
  // sign of face dof b in C_T: +1 on the max side of an axis, -1 on the min side
  auto eps = [&](int b) { return ((b / K2) & 1) ? 1.0 : -1.0; };
  double anrm = 0.0;  // ||M_T||_inf (masked), for the refinement's stopping test

  const double al = a.alpha ? a.alpha[es] : 0.0, be = a.beta ? a.beta[es] : 0.0;
  double fv[3] = {0.0, 0.0, 0.0};
  if (rhs) {
    fv[0] = a.f[es * 3 + 0]; fv[1] = a.f[es * 3 + 1]; fv[2] = a.f[es * 3 + 2];
  }
  const bool need_matrix = matrix || (rhs && a.g);
  element_qd<K, TEAM>(mp, es, al, be, fv, need_matrix, rhs, xe, qd, lane, live, a.status, e);

  if (matrix) {
    if constexpr (TEAM % 64 == 0) {
      assemble_mfma<K, TEAM, Lay::QC>(mp, qd, reinterpret_cast<double*>(W), lane,
                                      [&](int i, int j, double v) { M[pk(i, j)] = v; });
    } else {
      for (int p = lane; p < R::npk; p += TEAM) {
        int i, j;
        unpk_f(p, i, j);
        M[p] = m_entry<K>(mp, qd, i, j);
      }
    }
    __syncthreads();
  } else {
    // right-hand side only: the stored factor and scaling
    const float* Lr = reinterpret_cast<const float*>(rec + Rec::l32);
    for (int p = lane; p < R::npk; p += TEAM) L[p] = Lr[p];
    for (int i = lane; i < n; i += TEAM) Sv[i] = rec[Rec::sc + i];
    __syncthreads();
    for (int c = lane; c < n; c += TEAM) dinv[c] = 1.0f / L[pk(c, c)];
    __syncthreads();
  }
  if (rhs) {
    // f_hat, with f_r -= M_re g_e from the unmasked matrix
    for (int i = lane; i < n; i += TEAM) {
      const int d = R::comp(i);
      double s = 0.0;
      for (int q = 0; q < Q; ++q) s += mp.tab_s[q * n + i] * qd[q * QD + 7 + d];
      if (is_ess(i)) {
        s = a.g ? a.g[es * nb + (i - ni)] : 0.0;
      } else if (a.g) {
        for (int j = ni; j < n; ++j)
          if (is_ess(j)) s -= (matrix ? Mrow(i, j) : (i > j ? m_entry<K>(mp, qd, i, j) : m_entry<K>(mp, qd, j, i))) *
                              a.g[es * nb + (j - ni)];
      }
      fh[i] = s;
    }
    __syncthreads();
  }

  if (matrix) {
    // essential rows/columns -> identity; power-of-two scaling; FP32 copy
    for (int p = lane; p < R::npk; p += TEAM) {
      int i, j;
      unpk_f(p, i, j);
      if (is_ess(i) || is_ess(j)) M[p] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int i = lane; i < n; i += TEAM) {
      int ex;
      (void)frexp(M[pk(i, i)], &ex);
      Sv[i] = ldexp(1.0, -(ex >> 1));
    }
    __syncthreads();
    for (int p = lane; p < R::npk; p += TEAM) {
      int i, j;
      unpk_f(p, i, j);
      L[p] = float(Sv[i] * M[p] * Sv[j]);
    }
    __syncthreads();
    // FP32 Cholesky; a breakdown means kappa(S M_T S) 2^-24 >= 1 (or M_T is
    // not SPD): the plain FP64 form is the one to use for this element
    if (chol_packed<float, n, TEAM>(L, lane) && live && lane == 0) report_error(a.status, HYB_E_REFINE, e);
    for (int c = lane; c < n; c += TEAM) dinv[c] = 1.0f / L[pk(c, c)];
    __syncthreads();

    // X = M^{-1} C_T^T by chunks of CH columns
    anrm = norm_inf<n, TEAM>(Mrow, red + 8, lane);
    bool ok = true;
    for (int c0 = 0; c0 < nb; c0 += CH) {
      ok &= refine_solve<n, TEAM, CH>(
          L, dinv, W, Sv, Mrow, [&](int i, int c) { return (i == ni + c0 + c) ? eps(c0 + c) : 0.0; },
          [&](int i, int c) -> double& { return Xe(i, c0 + c); }, sweeps, anrm, red, lane);
    }
    if (!ok && live && lane == 0) report_error(a.status, HYB_E_REFINE, e);

    // H_T = D (M^{-1})_bb D = D E_b^T X, symmetrized, scattered into H (same-
    // face blocks receive two element terms by atomic add)
    if (live) {
      for (int t = lane; t < R::nbpk; t += TEAM) {
        int aa, bb;
        unpk_f(t, aa, bb);
        const int fa = aa / K2, fb = bb / K2;
        if (fid[fa] < 0 || fid[fb] < 0) continue;
        const double v = 0.5 * (eps(aa) * Xe(ni + aa, bb) + eps(bb) * Xe(ni + bb, aa));
        int a0 = (aa % K2) % K1, a1 = (aa % K2) / K1, b0 = (bb % K2) % K1, b1 = (bb % K2) / K1;
        frame_map(pic[fa], K, a0, a1);
        frame_map(pic[fb], K, b0, b1);
        const int ja = a0 + K1 * a1, jb = b0 + K1 * b1;
        const int Fa = fid[fa], Fb = fid[fb];
        const double vw = v * (mp.face_w[ja] * mp.face_w[jb]);   // M_s H_T M_s (weighted C)
        const int64_t pab = mp.face_rowbase[Fa] + int64_t(ja) * mp.face_nslots[Fa] * K2 +
                            mp.elem_slot[e * 36 + fa * 6 + fb] * K2 + jb;
        const int64_t pba = mp.face_rowbase[Fb] + int64_t(jb) * mp.face_nslots[Fb] * K2 +
                            mp.elem_slot[e * 36 + fb * 6 + fa] * K2 + ja;
        if (fa == fb) {
          atomicAdd(&a.Hval[pab], vw);
          if (aa != bb) atomicAdd(&a.Hval[pba], vw);
        } else {
          a.Hval[pab] = vw;
          a.Hval[pba] = vw;
        }
      }
    }
  }

  if (rhs) {
    // y = M^{-1} f_hat, refined the same way (one column)
    if (!matrix) anrm = norm_inf<n, TEAM>(Mrow, red + 8, lane);
    const bool oky = refine_solve<n, TEAM, 1>(
        L, dinv, W, Sv, Mrow, [&](int i, int) { return fh[i]; }, [&](int i, int) -> double& { return yv[i]; },
        sweeps, anrm, red, lane);
    if (!oky && live && lane == 0) report_error(a.status, HYB_E_REFINE, e);
    if (live) {
      for (int i = lane; i < n; i += TEAM) a.y[e * n + i] = yv[i];
      // r_T = D y_b
      for (int b = lane; b < nb; b += TEAM) {
        const int fb = b / K2;
        if (fid[fb] < 0) continue;
        int b0 = (b % K2) % K1, b1 = (b % K2) / K1;
        frame_map(pic[fb], K, b0, b1);
        atomicAdd(&a.r[int64_t(fid[fb]) * K2 + b0 + K1 * b1], eps(b) * yv[ni + b] * mp.face_w[b0 + K1 * b1]);
      }
    }
  }

  if (matrix && live) {
    float* Lr = reinterpret_cast<float*>(rec + Rec::l32);
    for (int p = lane; p < R::npk; p += TEAM) Lr[p] = L[p];
    for (int i = lane; i < n; i += TEAM) rec[Rec::sc + i] = Sv[i];
    if constexpr (!Lay::kGlobal) {
      for (int p = lane; p < R::npk; p += TEAM) rec[Rec::m64 + p] = Ml[p];
      for (int t = lane; t < n * nb; t += TEAM) rec[Rec::x + t] = Xl[(t / n) * XS + t % n];
    }
  }
}

template <int K, int TEAM, int EPB>
__global__ __launch_bounds__(TEAM* EPB) void k_setup_mixed(SetupArgs a, int sweeps) {
  __shared__ double smem[EPB * MixedLayout<K, TEAM, EPB>::per];
  setup_mixed_body<K, TEAM, EPB>(a, smem, blockIdx.x, sweeps);
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
