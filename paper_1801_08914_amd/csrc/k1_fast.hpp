// RT_1 kernels for affine hexahedra (n = 36 broken dofs, 12 interior, 24 on
// faces).  Setup: a team of 8 lanes per element, 8 elements per wave, every
// matrix row set held in registers, one LDS barrier per eliminated column.
// Right-hand side and recovery: one element per lane.
//
// Per element the setup computes, in the i-first order of Sec. 5:
//   M_T (affine: alpha G[d_i][d_j] T_ij + beta/detJ Dv_ij with the reference
//        integrals T_ij = int s_i s_j and Dv_ij = int div_i div_j, exact for
//        a constant Jacobian),
//   the upper Cholesky rows of the interior block, U_ii, and W = U_ii^{-T} A_ib
//        (interior elimination, column-cyclic over the team),
//   S = A_bb - W^T W, its Cholesky factor L and L^{-1} (in place),
//   H_T = D L^{-T} L^{-1} D in 4x4 face blocks, scattered into CSR H,
//   y = (U_ii^{-T} f_i, L^{-1}(f_b - W^T y_i)) and r_T = D L^{-T} y_b.
//
// Factor layout in HBM ("64-interleaved"): entry x of element e at
//   ((e / 64) * 666 + x) * 64 + e % 64, with x in
//   [0, 78)    U_ii, upper triangle packed by rows,
//   [78, 366)  W, 12 x 24 row-major,
//   [366, 666) L^{-1}, lower triangle packed by rows.
// y uses the same interleaving with 36 entries per element (local order).
#pragma once

#include "kernels_common.hpp"
#include "setup_generic.hpp"

namespace hyb {
namespace k1 {

constexpr int N = 36, NI = 12, NB = 24, FLEN = 666, OFF_W = 78, OFF_LI = 366;

__device__ __forceinline__ int64_t fidx(int64_t e, int x) { return ((e >> 6) * FLEN + x) * 64 + (e & 63); }
__device__ __forceinline__ int64_t yidx(int64_t e, int i) { return ((e >> 6) * N + i) * 64 + (e & 63); }
// start of row c of the packed upper interior factor
__device__ __host__ constexpr int uoff(int c) { return c * 12 - c * (c - 1) / 2; }
// component of local dof i (interior: i / 4, face dof 12 + a: a / 8)
__device__ __host__ constexpr int comp(int i) { return i < 12 ? i / 4 : (i - 12) / 8; }

// Affine geometry of one element from vertices 0, 1, 2 and 4: J columns are
// the edge vectors.  Returns det J and fills G = J^T J / det J (symmetric).
__device__ __forceinline__ double affine_geometry(const DeviceMaps& mp, int64_t e, double J[3][3], double G[3][3]) {
  const int32_t* ev = mp.e2v + e * 8;
  const int v0 = ev[0];
  const int vs[3] = {ev[1], ev[2], ev[4]};
  double x0[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) x0[r] = mp.xyz[3 * int64_t(v0) + r];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r) J[r][c] = mp.xyz[3 * int64_t(vs[c]) + r] - x0[r];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double id = 1.0 / det;
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int c = 0; c < 3; ++c) G[d][c] = (J[0][d] * J[0][c] + J[1][d] * J[1][c] + J[2][d] * J[2][c]) * id;
  return det;
}

// Static assignment of the 21 lower 4x4 face blocks (fa >= fb) of H_T to the
// 8 lanes of a team, balanced by the length of their row loops (24 - 4 fa).
// Entry = fa * 8 + fb, terminated by 255.
__constant__ uint8_t c_blocks[8][4] = {
    {0 * 8 + 0, 5 * 8 + 5, 3 * 8 + 3, 255},
    {1 * 8 + 0, 5 * 8 + 4, 4 * 8 + 4, 255},
    {1 * 8 + 1, 5 * 8 + 3, 4 * 8 + 3, 255},
    {2 * 8 + 0, 5 * 8 + 2, 4 * 8 + 2, 255},
    {2 * 8 + 1, 5 * 8 + 1, 4 * 8 + 1, 255},
    {2 * 8 + 2, 5 * 8 + 0, 4 * 8 + 0, 255},
    {3 * 8 + 0, 3 * 8 + 2, 255, 255},
    {3 * 8 + 1, 255, 255, 255},
};

// per team: [0, 96) row/column broadcast buffers, [96, 400) W + y_i, then
// L^{-1} (packed rows + pad), [400, 424) y_b
constexpr int LDS_PER_TEAM = 424;

__global__ __launch_bounds__(64) void k_setup_k1(SetupArgs a) {
  __shared__ double lds[8][LDS_PER_TEAM];
  const int lane = threadIdx.x, tau = lane >> 3, t = lane & 7;
  const int64_t e = int64_t(blockIdx.x) * 8 + tau;
  const bool live = e < a.ne;
  const int64_t es = live ? e : 0;
  double* bcast = lds[tau];             // 2 x 48
  double* wbuf = bcast + 96;            // W (12 x 24) then y_i (12)
  double* lin = wbuf;                   // L^{-1} packed rows, after W is consumed
  double* ybuf = bcast + 400;           // y_b (24)
  const DeviceMaps& mp = a.mp;
  const bool rhs = (a.mode & MODE_RHS) != 0;

  double J[3][3], G[3][3];
  const double det = affine_geometry(mp, es, J, G);
  if (live && t == 0 && !(det > 0.0)) report_error(a.status, HYB_E_JACOBIAN, e);
  const double al = a.alpha[es], bd = a.beta[es] / det;
  double jtf[3] = {0.0, 0.0, 0.0};
  if (rhs) {
    const double f0 = a.f[es * 3], f1 = a.f[es * 3 + 1], f2 = a.f[es * 3 + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d) jtf[d] = J[0][d] * f0 + J[1][d] * f1 + J[2][d] * f2;
  }
  unsigned ess = 0;
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (mp.elem_face[es * 6 + f] < 0) ess |= 1u << f;
  const double* Tr = mp.tab_ref;           // T (symmetric, 36 x 36)
  const double* Dr = mp.tab_ref + N * N;   // Dv (symmetric)
  const double* sr = mp.tab_ref + 2 * N * N;
  const double* gb = (rhs && a.g) ? a.g + es * NB : nullptr;
  // unmasked M_T[i][j] for dofs of components di, dj (di compile-time)
  auto entry = [&](int i, int j, double gij) -> double {
    return al * gij * Tr[j * N + i] + bd * Dr[j * N + i];
  };
  auto gsel = [&](int di, int dj) -> double {   // G[di][dj] with a runtime dj
    return dj == 0 ? G[di][0] : (dj == 1 ? G[di][1] : G[di][2]);
  };
  auto ess_dof = [&](int j) -> bool { return j >= 12 && ((ess >> ((j - 12) >> 2)) & 1u); };

  // ======== pass 1: interior rows, column-cyclic (lane t owns the columns
  // j = base + 8 m, m = 0..4, j = 36 being the right-hand side) ========
  {
    const int base = (t + 4) & 7;
    double R[12][5];
#pragma unroll
    for (int r = 0; r < 12; ++r)
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int j = base + 8 * m;
        R[r][m] = (j < 36 && !ess_dof(j)) ? entry(r, j, gsel(r / 4, comp(j))) : 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);
    if (rhs) {
#pragma unroll
      for (int r = 0; r < 12; ++r) {
        double corr = 0.0;
        if (gb) {
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            const int j = base + 8 * m;
            if (j < 36 && ess_dof(j)) corr += entry(r, j, gsel(r / 4, comp(j))) * gb[j - 12];
          }
          corr += __shfl_xor(corr, 1, 8);
          corr += __shfl_xor(corr, 2, 8);
          corr += __shfl_xor(corr, 4, 8);
        }
        if (t == 0) R[r][4] = jtf[r / 4] * sr[r] - corr;
      }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      double* buf = bcast + 48 * (c & 1);
#pragma unroll
      for (int m = 0; m < 5; ++m)
        if (base + 8 * m <= 36) buf[base + 8 * m] = R[c][m];
      __syncthreads();
      double d = buf[c];
      if (!(d > 0.0)) {
        if (live && t == 0) report_error(a.status, HYB_E_NOT_SPD, e);
        d = 1.0;
      }
      const double sq = sqrt(d), is = 1.0 / sq;
#pragma unroll
      for (int m = 0; m < 5; ++m) R[c][m] = (base + 8 * m == c) ? sq : R[c][m] * is;
#pragma unroll
      for (int r = 0; r < 12; ++r) {
        if (r <= c) continue;
        const double ur = buf[r] * is;
#pragma unroll
        for (int m = 0; m < 5; ++m) R[r][m] -= ur * R[c][m];
      }
#pragma unroll
      for (int r = 0; r < 12; ++r)
#pragma unroll
        for (int m = 0; m < 5; ++m) __asm__ volatile("" : "+v"(R[r][m]));
      // finished row c: U_ii and W to HBM, W and y_c to LDS for pass 2
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int j = base + 8 * m;
        if (j < c || j > 36) continue;
        const double v = R[c][m];
        if (j < 12) {
          if (live) a.factor[fidx(e, uoff(c) + (j - c))] = v;
        } else if (j < 36) {
          wbuf[24 * c + (j - 12)] = v;
          if (live) a.factor[fidx(e, OFF_W + 24 * c + (j - 12))] = v;
        } else {
          wbuf[288 + c] = v;
          if (rhs && live) a.y[yidx(e, c)] = v;
        }
      }
    }
  }
  __syncthreads();

  // ======== pass 2: face rows a = 8 s + t (component s), lower part
  // b <= 8 s + 7: S = A_bb - W^T W and t = f_b - W^T y_i ========
  // rows of the three slots stored back to back: slot s starts at 4 s (s + 1)
  double Sr[48], ts[3];
#define SROW(s, b) Sr[4 * (s) * ((s) + 1) + (b)]
  // Keep every row value materialized here: without it the compiler sinks
  // each row's chain of updates down to its first reader and keeps all the
  // operands alive meanwhile.
#define PIN_ROWS()                                         \
  do {                                                     \
    _Pragma("unroll") for (int q_ = 0; q_ < 48; ++q_)      \
      __asm__ volatile("" : "+v"(Sr[q_]));                 \
    __asm__ volatile("" : "+v"(ts[0]), "+v"(ts[1]), "+v"(ts[2])); \
  } while (0)
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int arow = 8 * s + t, ia = 12 + arow;
    const bool ess_a = ess_dof(ia);
#pragma unroll
    for (int b = 0; b < 24; ++b) {
      if (b > 8 * s + 7) break;
      double v;
      if (ess_a || ess_dof(12 + b)) v = (b == arow) ? 1.0 : 0.0;
      else v = entry(ia, 12 + b, G[s][b >> 3]);
      SROW(s, b) = v;
    }
    double tv = 0.0;
    if (rhs) {
      if (ess_a) {
        tv = gb ? gb[arow] : 0.0;
      } else {
        tv = jtf[s] * sr[ia];
        if (gb) {
#pragma unroll
          for (int b = 0; b < 24; ++b)
            if (ess_dof(12 + b)) tv -= entry(ia, 12 + b, G[s][b >> 3]) * gb[b];
        }
      }
    }
    ts[s] = tv;
    __builtin_amdgcn_sched_barrier(0);
  }
  // S -= W^T W and t -= W^T y_i, one interior row c at a time (W entries of
  // boundary faces are zero, so identity rows stay identity)
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double w0 = wbuf[24 * c + t], w1 = wbuf[24 * c + 8 + t], w2 = wbuf[24 * c + 16 + t];
    const double yc = wbuf[288 + c];
#pragma unroll
    for (int b = 0; b < 24; ++b) {
      const double u = wbuf[24 * c + b];
      if (b < 8) SROW(0, b) -= w0 * u;
      if (b < 16) SROW(1, b) -= w1 * u;
      SROW(2, b) -= w2 * u;
    }
    if (rhs) {
      ts[0] -= w0 * yc;
      ts[1] -= w1 * yc;
      ts[2] -= w2 * yc;
    }
    PIN_ROWS();
  }

  // ======== Cholesky of S (lower rows in registers), forward solve y_b ========
#pragma unroll
  for (int c = 0; c < 24; ++c) {
    double* buf = bcast + 48 * (c & 1);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (c <= 8 * s + 7) buf[8 * s + t] = SROW(s, c);
      buf[24 + 8 * s + t] = ts[s];
    }
    __syncthreads();
    double d = buf[c];
    if (!(d > 0.0)) {
      if (live && t == 0) report_error(a.status, HYB_E_NOT_SPD, e);
      d = 1.0;
    }
    const double sq = sqrt(d), is = 1.0 / sq, inv = 1.0 / d;
    const double yc = buf[24 + c] * is;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int arow = 8 * s + t;
      if (c < 8 * s + 7) {
        const double la = SROW(s, c);
        const double lai = la * inv;
#pragma unroll
        for (int j = 0; j < 24; ++j)
          if (j > c && j <= 8 * s + 7) SROW(s, j) -= lai * buf[j];
        if (rhs) ts[s] -= (arow > c ? la * is : 0.0) * yc;
      }
      if (c <= 8 * s + 7) {
        const double v = SROW(s, c);
        SROW(s, c) = (arow == c) ? sq : (arow > c ? v * is : v);
      }
    }
    if (t == (c & 7)) {
      ybuf[c] = yc;
      if (rhs && live) a.y[yidx(e, 12 + c)] = yc;
    }
    PIN_ROWS();
  }
  // clear the upper parts of the rows (the in-place inversion sums over them)
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int b = 0; b < 24; ++b)
      if (b <= 8 * s + 7 && b > 8 * s + t) SROW(s, b) = 0.0;

  // ======== in-place inversion L -> L^{-1}, columns right to left ========
#pragma unroll
  for (int j = 23; j >= 0; --j) {
    double* buf = bcast + 48 * (j & 1);
#pragma unroll
    for (int s = 0; s < 3; ++s)
      if (j <= 8 * s + 7) buf[8 * s + t] = SROW(s, j);
    __syncthreads();
    const double rinv = 1.0 / buf[j];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (j > 8 * s + 7) continue;
      const int arow = 8 * s + t;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 24; ++k)
        if (k > j && k <= 8 * s + 7) acc += SROW(s, k) * buf[k];
      const double v = SROW(s, j);
      SROW(s, j) = (arow > j) ? -rinv * acc : (arow == j ? rinv : v);
    }
    PIN_ROWS();
  }
  // L^{-1} rows to LDS (packed lower rows; W is no longer needed)
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int arow = 8 * s + t;
#pragma unroll
    for (int b = 0; b < 24; ++b)
      if (b <= 8 * s + 7 && b <= arow) lin[arow * (arow + 1) / 2 + b] = SROW(s, b);
  }
  if (t < 4) lin[300 + t] = 0.0;
  __syncthreads();

  if (!live) return;
  // face ids and frame codes, indexed by runtime face numbers below
  const int* fid = mp.elem_face + e * 6;
  const uint8_t* pic = mp.elem_pi + e * 8;
  // L^{-1} to HBM, team-cooperative
  for (int p = t; p < 300; p += 8) a.factor[fidx(e, OFF_LI + p)] = lin[p];
#undef SROW
#undef PIN_ROWS
  // H_T = D L^{-T} L^{-1} D in 4x4 face blocks
  for (int q = 0; q < 4; ++q) {
    const int code = c_blocks[t][q];
    if (code == 255) break;
    const int fa = code >> 3, fb = code & 7;
    if (fid[fa] < 0 || fid[fb] < 0) continue;
    double h[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) h[i][jj] = 0.0;
    const int a0 = 4 * fa, b0 = 4 * fb;
    for (int c = a0; c < 24; ++c) {
      const double* row = lin + c * (c + 1) / 2;
      double va[4], vb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        va[i] = (a0 + i <= c) ? row[a0 + i] : 0.0;
        vb[i] = (b0 + i <= c) ? row[b0 + i] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) h[i][jj] += va[i] * vb[jj];
    }
    const double sgn = ((fa ^ fb) & 1) ? -1.0 : 1.0;
    const int Fa = fid[fa], Fb = fid[fb];
    const int64_t rba = mp.face_rowbase[Fa], rbb = mp.face_rowbase[Fb];
    const int lena = mp.face_nslots[Fa] * 4, lenb = mp.face_nslots[Fb] * 4;
    const int sab = mp.elem_slot[e * 36 + fa * 6 + fb] * 4, sba = mp.elem_slot[e * 36 + fb * 6 + fa] * 4;
    // owner-frame index of each local face dof
    int pa[4], pb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int x0 = i & 1, x1 = i >> 1;
      frame_map(pic[fa], 1, x0, x1);
      pa[i] = x0 + 2 * x1;
      int y0 = i & 1, y1 = i >> 1;
      frame_map(pic[fb], 1, y0, y1);
      pb[i] = y0 + 2 * y1;
    }
    if (fa == fb) {
      // same face: the neighbour element adds its own term
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          atomicAdd(&a.Hval[rba + int64_t(pa[i]) * lena + sab + pb[jj]], sgn * h[i][jj]);
    } else if (pic[fa] == 0 && pic[fb] == 0) {
      // both faces in the owner's frame: contiguous row segments
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double* dst = a.Hval + rba + int64_t(i) * lena + sab;
        dst[0] = sgn * h[i][0]; dst[1] = sgn * h[i][1]; dst[2] = sgn * h[i][2]; dst[3] = sgn * h[i][3];
        double* dst2 = a.Hval + rbb + int64_t(i) * lenb + sba;
        dst2[0] = sgn * h[0][i]; dst2[1] = sgn * h[1][i]; dst2[2] = sgn * h[2][i]; dst2[3] = sgn * h[3][i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          a.Hval[rba + int64_t(pa[i]) * lena + sab + pb[jj]] = sgn * h[i][jj];
          a.Hval[rbb + int64_t(pb[jj]) * lenb + sba + pa[i]] = sgn * h[i][jj];
        }
    }
  }
  // r_T = D L^{-T} y_b
  if (rhs) {
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int arow = 8 * s + t, fa = arow >> 2;
      if (fid[fa] < 0) continue;
      double acc = 0.0;
      for (int c = arow; c < 24; ++c) acc += lin[c * (c + 1) / 2 + arow] * ybuf[c];
      if (!(fa & 1)) acc = -acc;
      int x0 = arow & 1, x1 = (arow >> 1) & 1;
      frame_map(pic[fa], 1, x0, x1);
      atomicAdd(&a.r[int64_t(fid[fa]) * 4 + x0 + 2 * x1], acc);
    }
  }
}

// ---------------------------------------------------------------------------
// One element per lane: right-hand side on stored factors.
struct SimtArgs {
  DeviceMaps mp;
  int64_t ne;
  const double* alpha;
  const double* beta;
  const double* f;
  const double* g;
  const double* factor;
  double* y;
  double* r;
  const double* lambda;
  double* u;
};

// Per-lane vectors live in LDS columns (v[i * 64 + lane]) so every loop can
// run with a runtime index without spilling registers.
__global__ __launch_bounds__(64) void k_rhs_k1(SimtArgs a) {
  __shared__ double vec[60 * 64];   // y (36) then r_T accumulators (24)
  const int L = threadIdx.x;
  const int64_t e = int64_t(blockIdx.x) * 64 + L;
  if (e >= a.ne) return;
  const DeviceMaps& mp = a.mp;
  double J[3][3], G[3][3];
  const double det = affine_geometry(mp, e, J, G);
  const double f0 = a.f[e * 3], f1 = a.f[e * 3 + 1], f2 = a.f[e * 3 + 2];
  double jtf[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) jtf[d] = J[0][d] * f0 + J[1][d] * f1 + J[2][d] * f2;
  unsigned ess = 0;
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (mp.elem_face[e * 6 + f] < 0) ess |= 1u << f;
  const double* Tr = mp.tab_ref;
  const double* Dr = mp.tab_ref + N * N;
  const double* sr = mp.tab_ref + 2 * N * N;
  const double* gb = a.g ? a.g + e * NB : nullptr;
  const double al = gb ? a.alpha[e] : 0.0, bd = gb ? a.beta[e] / det : 0.0;
  double* y = vec;
  double* rt = vec + 36 * 64;
  for (int i = 0; i < 36; ++i) {
    const int ci = comp(i);
    double v = (ci == 0 ? jtf[0] : (ci == 1 ? jtf[1] : jtf[2])) * sr[i];
    const bool ei = i >= 12 && ((ess >> ((i - 12) >> 2)) & 1u);
    if (ei) {
      v = gb ? gb[i - 12] : 0.0;
    } else if (gb) {
      for (int j = 12; j < 36; ++j)
        if ((ess >> ((j - 12) >> 2)) & 1u)
          v -= (al * G[ci][comp(j)] * Tr[j * N + i] + bd * Dr[j * N + i]) * gb[j - 12];
    }
    y[i * 64 + L] = v;
  }
  // y_i = U_ii^{-T} f_i
  for (int c = 0; c < 12; ++c) {
    double v = y[c * 64 + L];
    for (int k = 0; k < c; ++k) v -= a.factor[fidx(e, uoff(k) + (c - k))] * y[k * 64 + L];
    y[c * 64 + L] = v / a.factor[fidx(e, uoff(c))];
  }
  // t_b = f_b - W^T y_i
  for (int c = 0; c < 12; ++c) {
    const double yc = y[c * 64 + L];
#pragma unroll 8
    for (int b = 0; b < 24; ++b) y[(12 + b) * 64 + L] -= a.factor[fidx(e, OFF_W + 24 * c + b)] * yc;
  }
  // y_b = L^{-1} t_b, from the bottom row up so t_b is overwritten in place
  for (int b = 23; b >= 0; --b) {
    double v = 0.0;
    for (int c = 0; c <= b; ++c) v += a.factor[fidx(e, OFF_LI + b * (b + 1) / 2 + c)] * y[(12 + c) * 64 + L];
    y[(12 + b) * 64 + L] = v;
  }
  for (int i = 0; i < 36; ++i) a.y[yidx(e, i)] = y[i * 64 + L];
  // r_T = D L^{-T} y_b
  for (int b = 0; b < 24; ++b) rt[b * 64 + L] = 0.0;
  for (int c = 0; c < 24; ++c) {
    const double yc = y[(12 + c) * 64 + L];
    for (int b = 0; b <= c; ++b) rt[b * 64 + L] += a.factor[fidx(e, OFF_LI + c * (c + 1) / 2 + b)] * yc;
  }
  for (int f = 0; f < 6; ++f) {
    const int F = mp.elem_face[e * 6 + f];
    if (F < 0) continue;
    const int pi = mp.elem_pi[e * 8 + f];
    for (int i = 0; i < 4; ++i) {
      int x0 = i & 1, x1 = i >> 1;
      frame_map(pi, 1, x0, x1);
      const double v = rt[(4 * f + i) * 64 + L];
      atomicAdd(&a.r[int64_t(F) * 4 + x0 + 2 * x1], (f & 1) ? v : -v);
    }
  }
}

// One element per lane: u_b = L^{-T}(y_b - L^{-1} D lambda_b),
// u_i = U_ii^{-1}(y_i - W u_b).  The per-lane vector (36 entries, the local
// order of u) stays in an LDS column and is written out coalesced.
__global__ __launch_bounds__(64) void k_recover_k1(SimtArgs a) {
  __shared__ double vec[36 * 64 + 64];
  const int L = threadIdx.x;
  const int64_t e0 = int64_t(blockIdx.x) * 64;
  const int64_t e = e0 + L;
  const DeviceMaps& mp = a.mp;
  double* v = vec;   // v[i * 64 + L]: [0,12) interior, [12,36) face block
  if (e < a.ne) {
    for (int f = 0; f < 6; ++f) {
      const int F = mp.elem_face[e * 6 + f];
      const int pi = mp.elem_pi[e * 8 + f];
      for (int i = 0; i < 4; ++i) {
        double x = 0.0;
        if (F >= 0) {
          int x0 = i & 1, x1 = i >> 1;
          frame_map(pi, 1, x0, x1);
          x = a.lambda[int64_t(F) * 4 + x0 + 2 * x1];
          if (!(f & 1)) x = -x;
        }
        v[(12 + 4 * f + i) * 64 + L] = x;
      }
    }
    // z_b = y_b - L^{-1} t, bottom row first (in place over t)
    for (int b = 23; b >= 0; --b) {
      double s = a.y[yidx(e, 12 + b)];
      for (int c = 0; c <= b; ++c) s -= a.factor[fidx(e, OFF_LI + b * (b + 1) / 2 + c)] * v[(12 + c) * 64 + L];
      v[(12 + b) * 64 + L] = s;
    }
    // u_b = L^{-T} z_b, top row first (in place over z)
    for (int b = 0; b < 24; ++b) {
      double s = 0.0;
      for (int c = b; c < 24; ++c) s += a.factor[fidx(e, OFF_LI + c * (c + 1) / 2 + b)] * v[(12 + c) * 64 + L];
      v[(12 + b) * 64 + L] = s;
    }
    // u_i = U_ii^{-1} (y_i - W u_b), backward
    for (int c = 11; c >= 0; --c) {
      double s = a.y[yidx(e, c)];
#pragma unroll 8
      for (int b = 0; b < 24; ++b) s -= a.factor[fidx(e, OFF_W + 24 * c + b)] * v[(12 + b) * 64 + L];
      for (int k = c + 1; k < 12; ++k) s -= a.factor[fidx(e, uoff(c) + (k - c))] * v[k * 64 + L];
      v[c * 64 + L] = s / a.factor[fidx(e, uoff(c))];
    }
  }
  __syncthreads();
  const int64_t cnt = (a.ne - e0) < 64 ? (a.ne - e0) : 64;
  for (int p = L; p < cnt * 36; p += 64) {
    const int el = p / 36, i = p % 36;
    a.u[e0 * 36 + p] = v[i * 64 + el];
  }
}

}  // namespace k1
}  // namespace hyb
