// RT_3 element setup (n = 240 broken dofs, 144 interior, 96 on faces) by
// the blocks of the interior-first order, M_T = [[A_ii, A_ib], [A_bi, A_bb]]:
//   L_ii = chol(A_ii)                    in LDS (83.5 KB), FP64 matrix cores,
//   L_bi = A_bi L_ii^{-T}                forward tile solves, in place in HBM,
//   S    = A_bb - L_bi L_bi^T            the face Schur complement, FP64
//                                        matrix-core SYRK into LDS,
//   L_bb = chol(S), then L_bb^{-1}       in LDS,
// so that H_T = D L_bb^{-T} L_bb^{-1} D (Sec. 3.1, Sec. 5) needs no pass
// over the whole 231 KB matrix in HBM per panel.  The element matrix is
// assembled by sum factorization: the interior block straight into LDS, the
// rows of the face dofs into the element's record (the packed factor, where
// L_bi stays and the face block is written back inverted, the layout of the
// generic kernels, which recover from it).
#pragma once

#include "mixed.hpp"

namespace hyb {

struct K3Layout {
  using R = RT<3>;
  static constexpr int n = R::n, ni = R::ni, nb = R::nb;
  static constexpr int npi = ni * (ni + 1) / 2;                 // packed interior block
  // staging: the sum factorization's partial sums, then the inverses of the
  // diagonal blocks of L_ii, then S (its factor L_bb) and the inverses of
  // L_bb's diagonal blocks; L_bb^{-1} (full nb x nb) goes where L_ii was
  static constexpr int stage0 = sumfact_stage<3>();
  static constexpr int stage1 = ((ni + 15) / 16) * 256;
  static constexpr int stage2 = R::nbpk + (nb / 16) * 256;   // L_bb and its diagonal blocks' inverses
  // row strides of L_bb^{-1} (nb + 1: a lane per row reads conflict-free) and
  // of L_bi^T (rows of the four lane groups 32 banks apart)
  static constexpr int XLD = nb + 1, LDE = nb + 16;
  static_assert(nb * XLD <= npi, "the full inverse of L_bb fits where L_ii was");
  static constexpr int stage = stage0 > stage1 ? (stage0 > stage2 ? stage0 : stage2) : (stage1 > stage2 ? stage1 : stage2);
  static_assert(load_sumfact_stage<3>() <= stage, "the load vector's partial sums fit in the staging area");
  static_assert(ni % 16 == 0 && nb % 16 == 0, "whole 16-row blocks");
  static_assert(ni * LDE <= npi + stage, "L_bi^T fits where L_ii and the staging area were");
  static constexpr int per = npi + stage + R::Q * 10 + n + 24 + nb + 8;
};

template <int TEAM>
__device__ __forceinline__ void setup_k3_body(const SetupArgs& a, double* smem, int64_t e) {
  using R = RT<3>;
  using Lay = K3Layout;
  constexpr int K = 3, n = R::n, ni = R::ni, nb = R::nb, K1 = R::K1, K2 = R::K2, Q = R::Q, QD = 10;
  constexpr int NW = TEAM / 64;
  static_assert(TEAM % 64 == 0 && TEAM >= nb, "whole waves, a lane per face row");
  const int lane = threadIdx.x % TEAM, w_id = lane / 64, l = lane % 64;
  const bool live = e < a.ne;
  const int64_t es = live ? e : 0;
  const bool own = live;   // a padding team (none in the launches here) writes nothing to the record
  double* A = smem;                  // L_ii (packed), LDS
  double* stg = A + Lay::npi;        // staging (see K3Layout)
  double* qd = stg + Lay::stage;
  double* fh = qd + Q * QD;
  double* xe = fh + n;
  double* tb = xe + 24;
  int* flag = reinterpret_cast<int*>(tb + nb);
  double* rec = a.factor + es * R::npk;   // the packed factor of the element (HBM)
  double* Sb = stg;                       // S, then L_bb (packed nb x nb)
  double* Xb = A;                         // L_bb^{-1}, full nb x nb, rows XLD apart (setup)
  double* E = A;                          // L_bi^T, rows LDE apart (setup, before S is factored)
  using M = MfmaT<double>;
  constexpr int NTi = ni / 16;
  const int li = l & 15, lk = l >> 4;
  const bool tw = w_id < nb / 16;         // the waves of the column tiles of L_bi^T and L_bb^{-1}
  const DeviceMaps& mp = a.mp;
  const bool matrix = (a.mode & MODE_MATRIX) != 0, rhs = (a.mode & MODE_RHS) != 0;
  // L_bb^{-1}: full in LDS after a setup, packed (from the record) for a right-hand side alone

  int fid[6], pic[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    fid[f] = mp.elem_face[es * 6 + f];
    pic[f] = mp.elem_pi[es * 8 + f];
  }
  const int nat = mp.elem_pi[es * 8 + 6];
  auto is_ess = [&](int i) {
    const int f = (i - ni) / K2;
    return i >= ni && fid[f] < 0 && !((nat >> f) & 1);
  };
  auto sigma = [&](int b) {
    const int f = b / K2;
    const double eps = (f & 1) ? 1.0 : -1.0;
    return mp.face_owner[fid[f]] == e ? eps : -eps;
  };

  // tb = f_b - L_bi y_i on the face rows of one column tile (the calling
  // wave's, 16 w_id ..) from the tile of L_bi^T in registers: per lane the
  // products over its rows in register order, then the sum over the lanes
  // of the column (the same order in a setup and for a right-hand side alone)
  auto lbi_yi = [&](const dx4(&X)[NTi]) {
    double p = 0.0;
#pragma unroll
    for (int I = 0; I < NTi; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) p += X[I][r] * fh[16 * I + M::row(l, r)];
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    if (lk == 0) tb[16 * w_id + li] = fh[ni + 16 * w_id + li] - p;
  };

  const double al = a.alpha ? a.alpha[es] : 0.0, be = a.beta ? a.beta[es] : 0.0;
  double fv[3] = {0.0, 0.0, 0.0};
  if (rhs) {
    fv[0] = a.f[es * 3 + 0]; fv[1] = a.f[es * 3 + 1]; fv[2] = a.f[es * 3 + 2];
  }
  const bool need_matrix = matrix || (rhs && a.g);
  element_qd<K, TEAM>(mp, es, al, be, fv, need_matrix, rhs, xe, qd, lane, live, a.status, e);
  // entry (i, j) of M_T by Gauss quadrature (the right-hand side alone, for
  // the boundary correction)
  auto mij = [&](int i, int j) {
    const int gi = gidx(R::comp(i), R::comp(j));
    double s = 0.0;
    for (int q = 0; q < Q; ++q)
      s += qd[q * QD + gi] * mp.tab_s[q * n + i] * mp.tab_s[q * n + j] +
           qd[q * QD + 6] * mp.tab_d[q * n + i] * mp.tab_d[q * n + j];
    return s;
  };

  if (matrix) {
    // (the interior entries through an LDS-qualified pointer: the two stores
    // are not merged into one flat store)
    lds_double* As = (lds_double*)(A);
    assemble_sumfact<K, TEAM>(mp, qd, stg, lane, [=](int i, int j, double v) {
      if (i < ni) As[pk(i, j)] = v;
      else if (own) rec[pk(i, j)] = v;
    });
    __syncthreads();
  }
  if (rhs) {
    // the load vector by sum factorization, then the boundary data
    load_sumfact<K, TEAM>(mp, qd, stg, lane, [=](int i, double v) { fh[i] = v; });
    for (int i = lane; i < n; i += TEAM) {
      double s = fh[i];
      if (is_ess(i)) {
        s = a.g ? a.g[es * nb + (i - ni)] : 0.0;
      } else if (a.g) {
        // f_r -= M_re g_e (unmasked matrix; the essential dofs are face dofs)
        for (int j = ni; j < n; ++j)
          if (is_ess(j)) s -= (matrix ? rec[i > j ? pk(i, j) : pk(j, i)] : (i > j ? mij(i, j) : mij(j, i))) *
                              a.g[es * nb + (j - ni)];
      }
      fh[i] = s;
    }
    __syncthreads();
  }

  if (matrix) {
    // essential face dofs: identity rows and columns (the interior block has
    // none), face by face; an entry between two essential faces is cleared
    // by both passes, a diagonal entry set by its own face's pass only
    for (int f = 0; f < 6; ++f) {
      if (!is_ess(ni + f * K2)) continue;   // uniform across the team
      for (int t = lane; t < K2 * n; t += TEAM) {
        const int i = ni + f * K2 + t / n, j = t % n;
        if (own) rec[i >= j ? pk(i, j) : pk(j, i)] = (i == j) ? 1.0 : 0.0;
      }
    }
    // L_ii = chol(A_ii) in LDS; the inverses of its diagonal blocks
    const bool bad_i = chol_mfma_t<double, ni, TEAM>(A, lane, true, flag, stg);
    auto Lii = [=](int i, int j) -> double { return A[pk(i, j)]; };
    diag_inverses<double, ni, TEAM>(Lii, stg, lane, true);
    __syncthreads();
    // L_bi^T = L_ii^{-1} A_bi^T by forward tile solves held in registers (the
    // record's face rows: column c of the tile is face row ni + c), six
    // column tiles over the waves, stored to the record and kept; y_i =
    // L_ii^{-1} f_i as a seventh (one column) while L_ii is in LDS
    dx4 Xr[NTi];
    if (tw) {
      tile_forward_regs<ni>(Lii, stg, [=](int i, int c) { return rec[pk(ni + c, i)]; }, Xr, 16 * w_id, 16, l);
#pragma unroll
      for (int I = 0; I < NTi; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (own) rec[pk(ni + 16 * w_id + li, 16 * I + M::row(l, r))] = Xr[I][r];
    } else if (w_id == nb / 16 && rhs) {
      tile_forward_reg<ni>(Lii, stg, [=](int i, int) { return fh[i]; }, [=](int i, int, double v) { fh[i] = v; }, 0, 1,
                           l);
    }
    __syncthreads();
    // L_ii back to the record; then L_bi^T from the registers into LDS where
    // L_ii was (E[k * LDE + c] = L_bi(c, k)), and f_b - L_bi y_i
    for (int t = lane; t < Lay::npi; t += TEAM)
      if (own) rec[t] = A[t];
    __syncthreads();
    if (tw) {
#pragma unroll
      for (int I = 0; I < NTi; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) E[(16 * I + M::row(l, r)) * Lay::LDE + 16 * w_id + li] = Xr[I][r];
      if (rhs) lbi_yi(Xr);
    }
    __syncthreads();
    // S = A_bb - L_bi L_bi^T: the 21 lower 16 x 16 tiles over the waves on the
    // FP64 matrix cores, operands from E; the accumulators stay in registers
    // until every wave is done with E (S goes where E ends)
    {
      constexpr int NT = nb / 16, NS = NT * (NT + 1) / 2, SU = (NS + NW - 1) / NW;
      dx4 Sacc[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int t = w_id + NW * u;
        if (t >= NS) continue;   // uniform
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        const int J = t - I * (I + 1) / 2;
        dx4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + M::row(l, r), j = 16 * J + li;
          acc[r] = j <= i ? rec[pk(ni + i, ni + j)] : 0.0;
        }
        const double* ea = E + lk * Lay::LDE + 16 * I + li;
        const double* eb = E + lk * Lay::LDE + 16 * J + li;
#pragma unroll 4
        for (int k0 = 0; k0 < ni; k0 += 4) acc = M::op(-ea[k0 * Lay::LDE], eb[k0 * Lay::LDE], acc);
        Sacc[u] = acc;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int t = w_id + NW * u;
        if (t >= NS) continue;
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        const int J = t - I * (I + 1) / 2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + M::row(l, r), j = 16 * J + li;
          if (j <= i) Sb[pk(i, j)] = Sacc[u][r];
        }
      }
    }
    // L_bb = chol(S) in LDS
    const bool bad_b = chol_mfma_t<double, nb, TEAM>(Sb, lane, true, flag, Sb + R::nbpk);
    if ((bad_i || bad_b) && live && lane == 0) report_error(a.status, HYB_E_NOT_SPD, e);
    if (a.stat) {
      // static condensation: S_hat_T = L_bb L_bb^T (lower triangle), sigma-signed, into S
      auto Lbb = [=](int i, int j) { return Sb[pk(i, j)]; };
      if (live) {
        for (int t = lane; t < R::nbpk; t += TEAM) {
          int aa, bb;
          unpk(t, aa, bb);
          const int fa = aa / K2, fb = bb / K2;
          if (fid[fa] < 0 || fid[fb] < 0) continue;
          double h = 0.0;
          for (int c = 0; c <= bb; ++c) h += Lbb(aa, c) * Lbb(bb, c);
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
      __syncthreads();
      for (int t = lane; t < R::nbpk; t += TEAM) {
        int i, j;
        unpk(t, i, j);
        if (own) rec[pk(ni + i, ni + j)] = Sb[t];
      }
      __syncthreads();
    } else {
      // L_bb^{-1} = L_bb^{-1} I by forward tile solves (one wave per column
      // tile, every 16-row block on the matrix cores), into Xb where L_ii was
      double* LiB = Sb + R::nbpk;
      auto Lbb = [=](int i, int j) -> double { return Sb[pk(i, j)]; };
      diag_inverses<double, nb, TEAM>(Lbb, LiB, lane, true);
      __syncthreads();
      if (tw)
        tile_forward_reg<nb>(Lbb, LiB, [=](int i, int c) { return i == c ? 1.0 : 0.0; },
                             [=](int i, int c, double v) { Xb[i * Lay::XLD + c] = v; }, 16 * w_id, 16, l, w_id);
      __syncthreads();
      // H_T = D L_bb^{-T} L_bb^{-1} D: the lower 16 x 16 tiles of X^T X on the
      // FP64 matrix cores (X lower triangular: the sum starts at row block I),
      // scattered into H from the accumulators (same-face blocks receive two
      // element terms by atomic add; the mirror entry written as well)
      {
        constexpr int NT = nb / 16;
        for (int t = w_id; t < NT * (NT + 1) / 2; t += NW) {
          int I = 0;
          while ((I + 1) * (I + 2) / 2 <= t) ++I;
          const int J = t - I * (I + 1) / 2;
          dx4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
          for (int c0 = 16 * I; c0 < nb; c0 += 4)
            acc = M::op(Xb[(c0 + lk) * Lay::XLD + 16 * I + li], Xb[(c0 + lk) * Lay::XLD + 16 * J + li], acc);
          // tile (I, J) couples faces I and J (K2 = 16 dofs per face): the
          // face data are the tile's, the frame maps the lane's
          static_assert(K2 == 16, "a 16 x 16 tile per face pair");
          const int Fa = fid[I], Fb = fid[J];
          if (!live || Fa < 0 || Fb < 0) continue;   // uniform
          const int64_t rba = mp.face_rowbase[Fa], rbb = mp.face_rowbase[Fb];
          const int64_t nsa = int64_t(mp.face_nslots[Fa]) * K2, nsb = int64_t(mp.face_nslots[Fb]) * K2;
          const int64_t sab = int64_t(mp.elem_slot[e * 36 + I * 6 + J]) * K2;
          const int64_t sba = int64_t(mp.elem_slot[e * 36 + J * 6 + I]) * K2;
          const bool flip = ((I ^ J) & 1) != 0;
          int b0 = li % K1, b1 = li / K1;
          frame_map(pic[J], K, b0, b1);
          const int jb = b0 + K1 * b1;
          const double wb = mp.face_w[jb];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ra = M::row(l, r);   // row of the tile: dof ra of face I
            if (I == J && li > ra) continue;
            int a0 = ra % K1, a1 = ra / K1;
            frame_map(pic[I], K, a0, a1);
            const int ja = a0 + K1 * a1;
            const double vw = (flip ? -acc[r] : acc[r]) * (mp.face_w[ja] * wb);   // M_s H_T M_s (weighted C)
            const int64_t pab = rba + ja * nsa + sab + jb;
            const int64_t pba = rbb + jb * nsb + sba + ja;
            if (I == J) {
              atomicAdd(&a.Hval[pab], vw);
              if (li != ra) atomicAdd(&a.Hval[pba], vw);
            } else {
              a.Hval[pab] = vw;
              a.Hval[pba] = vw;
            }
          }
        }
      }
      // the face block of the record: L_bb^{-1} (lower)
      for (int t = lane; t < R::nbpk; t += TEAM) {
        int i, j;
        unpk(t, i, j);
        if (own) rec[pk(ni + i, ni + j)] = Xb[i * Lay::XLD + j];
      }
      __syncthreads();
    }
  } else if (rhs) {
    // a right-hand side alone: y_i = L_ii^{-1} f_i from the stored L_ii and
    // f_b - L_bi y_i from the stored L_bi, as the setup computes them, then
    // the stored face block into LDS
    for (int t = lane; t < Lay::npi; t += TEAM) A[t] = rec[t];
    __syncthreads();
    auto Lii = [=](int i, int j) -> double { return A[pk(i, j)]; };
    diag_inverses<double, ni, TEAM>(Lii, stg, lane, true);
    __syncthreads();
    if (w_id == 0)
      tile_forward_reg<ni>(Lii, stg, [=](int i, int) { return fh[i]; }, [=](int i, int, double v) { fh[i] = v; }, 0, 1,
                           l);
    __syncthreads();
    if (tw) {
      dx4 Xr[NTi];
#pragma unroll
      for (int I = 0; I < NTi; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) Xr[I][r] = rec[pk(ni + 16 * w_id + li, 16 * I + M::row(l, r))];
      lbi_yi(Xr);
    }
    for (int t = lane; t < R::nbpk; t += TEAM) {
      int i, j;
      unpk(t, i, j);
      Sb[t] = rec[pk(ni + i, ni + j)];
    }
    __syncthreads();
  }

  if (rhs) {
    // y_b = L_bb^{-1} (f_b - L_bi y_i); static condensation keeps
    // f_b - L_bi y_i (on boundary faces: their data g)
    for (int b = lane; b < nb; b += TEAM) {
      double s = tb[b];
      if (!a.stat) {
        // row b of L_bb^{-1}: full rows after a setup, packed from the record
        // (the same products in the same order; loops unrolled so that the
        // loads run ahead of the chain of sums)
        s = 0.0;
        const double* lr = matrix ? Xb + b * Lay::XLD : Sb + pk(b, 0);
#pragma unroll 8
        for (int c = 0; c <= b; ++c) s += lr[c] * tb[c];
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
          // column b of L_bb^{-1}
          s = 0.0;
          if (matrix) {
            const double* lc = Xb + b;
#pragma unroll 8
            for (int c = b; c < nb; ++c) s += lc[c * Lay::XLD] * fh[ni + c];
          } else {
            int p = pk(b, b);
#pragma unroll 8
            for (int c = b; c < nb; ++c) {
              s += Sb[p] * fh[ni + c];
              p += c + 1;
            }
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
}

template <int TEAM>
__global__ __launch_bounds__(TEAM) void k_setup_k3(SetupArgs a) {
  __shared__ double smem[K3Layout::per];
  setup_k3_body<TEAM>(a, smem, blockIdx.x);
}

}  // namespace hyb
