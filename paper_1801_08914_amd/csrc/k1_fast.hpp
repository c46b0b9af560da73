// RT_1 kernels for affine hexahedra (n = 36 broken dofs: 12 interior, 24 on
// faces).
//
// Setup: one element per 16-lane row of the wave (4 elements per wave; lanes
// 12..15 of each row shadow lane 0 and store nothing).  Lane t holds three
// rows of the element matrix in registers: interior row t and face rows t and
// 12 + t, each with all 36 columns and the right-hand side.
//  1. Assembly (affine: M = alpha G[d_i][d_j] T_ij + beta/detJ Dv_ij with the
//     reference integrals T_ij = int s_i s_j, Dv_ij = int div_i div_j, exact
//     for a constant Jacobian); boundary-face rows and columns become
//     identity, their values move to the right-hand side.
//  2. Exact power-of-two diagonal scaling, so every pivot lies in (0, 2).
//  3. Gauss-Jordan sweep of the 12 interior pivots: the interior block
//     becomes -A_ii^{-1}, the interior-face block E = A_ii^{-1} A_ib, the face
//     block S = A_bb - A_bi A_ii^{-1} A_ib and the right-hand side
//     (A_ii^{-1} f_i, f_b - E^T f_i): the static condensation of the interior
//     dofs (Sec. 5) in sweep form.
//  4. Gauss-Jordan sweep of the 24 face pivots over the face rows:
//     S -> -S^{-1}, t -> S^{-1} t.  H_T = D S^{-1} D and r_T = D S^{-1} t
//     (Theorem 2.1 with the interior dofs condensed).
// The pivot row k of a step lives in one lane; its entries reach the other
// lanes of the row by DPP row broadcast, fused into no memory traffic.  Row r
// is updated as r_j -= (r_k / d) p_j.  The pivot lane uses the multiplier
// 1 - 1/d and every lane substitutes d - 1 for the pivot entry p_k, which
// leaves p / d in the pivot row and r_k / d in the pivot column without
// indexing a register by k; the swept diagonal entry then holds 2 - 1/d
// instead of -1/d (corrected on output).  With pivots below 2 the
// cancellation in these updates costs at most a few ulps.
//
// Per-element record in HBM (672 doubles, 128-byte aligned):
//   [0, 78)    A_ii^{-1}, lower triangle packed by rows,
//   [78, 366)  E, 12 x 24 row-major,
//   [366, 666) S^{-1}, lower triangle packed by rows.
// y (36 per element): (A_ii^{-1} f_i, S^{-1} t).
// Recovery: u_b = y_b - S^{-1} D lambda, u_i = y_i - E u_b.
//
// The same-face blocks of H and the entries of r receive one term from each
// of the face's two elements: the owner stores its term in place, the
// neighbour into a side buffer, and k_finalize_k1 adds the two, so H and r
// are bitwise reproducible and no atomics are used.
#pragma once

#include <type_traits>
#include <utility>

#include "kernels_common.hpp"
#include "setup_generic.hpp"

namespace hyb {
namespace k1 {

constexpr int N = 36, NB = 24, OFF_E = 78, OFF_SI = 366, REC = 672;
constexpr int TEAM = 12;       // rows per element handled by 12 lanes
constexpr int SETUP_EPW = 4;   // setup: one element per 16-lane DPP row
constexpr int SOLVE_EPW = 5;   // right-hand side and recovery: 5 teams of 12

// component (axis) of local dof i: interior i / 4, face dof 12 + a: a / 8
__device__ __host__ constexpr int comp(int i) { return i < 12 ? i / 4 : (i - 12) / 8; }
// packed lower index of a symmetric pair
__device__ __forceinline__ int spk(int a, int b) { return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a; }

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of elements so that face neighbours share an L2.
__device__ __forceinline__ int64_t xcd_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned q = nb / 8, rem = nb % 8, x = b % 8, i = b / 8;
  return int64_t(x) * q + (x < rem ? x : rem) + i;
}

// Owner-frame index of face dof i (0..3) of a face with frame code pi.
__device__ __forceinline__ int own_idx(int pi, int i) {
  int p0 = i & 1, p1 = i >> 1;
  frame_map(pi, 1, p0, p1);
  return p0 + 2 * p1;
}

// Lane L of each 16-lane row, broadcast to the whole row (DPP row_newbcast).
template <int L>
__device__ __forceinline__ double row_bcast(double x) {
  return __builtin_amdgcn_update_dpp(x, x, 0x150 + L, 0xF, 0xF, true);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Per-element affine data shared by the three kernels.
struct Elem {
  double g00, g01, g02, g11, g12, g22;   // G = J^T J / det J
  double jtf[3];                         // J^T f
  double al, bd;                         // alpha, beta / det J
  double det;
  unsigned ess;                          // bit f: face f is on the boundary

  __device__ __forceinline__ void load(const DeviceMaps& mp, int64_t e, const double* alpha, const double* beta,
                                       const double* f, bool need_matrix) {
    const int32_t* ev = mp.e2v + e * 8;
    const int v0 = ev[0];
    const int vs[3] = {ev[1], ev[2], ev[4]};
    double J[3][3], x0[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) x0[r] = mp.xyz[3 * int64_t(v0) + r];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) J[r][c] = mp.xyz[3 * int64_t(vs[c]) + r] - x0[r];
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double id = 1.0 / det;
    auto gg = [&](int d, int c) { return (J[0][d] * J[0][c] + J[1][d] * J[1][c] + J[2][d] * J[2][c]) * id; };
    g00 = gg(0, 0); g01 = gg(0, 1); g02 = gg(0, 2); g11 = gg(1, 1); g12 = gg(1, 2); g22 = gg(2, 2);
    if (f) {
      const double f0 = f[e * 3], f1 = f[e * 3 + 1], f2 = f[e * 3 + 2];
#pragma unroll
      for (int d = 0; d < 3; ++d) jtf[d] = J[0][d] * f0 + J[1][d] * f1 + J[2][d] * f2;
    } else {
      jtf[0] = jtf[1] = jtf[2] = 0.0;
    }
    al = need_matrix ? alpha[e] : 0.0;
    bd = need_matrix ? beta[e] / det : 0.0;
    ess = 0;
#pragma unroll
    for (int fc = 0; fc < 6; ++fc)
      if (mp.elem_face[e * 6 + fc] < 0) ess |= 1u << fc;
  }
  // from the edge vectors J[r][c] (row-major) and the element's data
  __device__ __forceinline__ void from(const double* Jr, double alpha, double beta, const double* f, unsigned ess_) {
    double J[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) J[r][c] = Jr[3 * r + c];
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double id = 1.0 / det;
    auto gg = [&](int d, int c) { return (J[0][d] * J[0][c] + J[1][d] * J[1][c] + J[2][d] * J[2][c]) * id; };
    g00 = gg(0, 0); g01 = gg(0, 1); g02 = gg(0, 2); g11 = gg(1, 1); g12 = gg(1, 2); g22 = gg(2, 2);
    if (f) {
#pragma unroll
      for (int d = 0; d < 3; ++d) jtf[d] = J[0][d] * f[0] + J[1][d] * f[1] + J[2][d] * f[2];
    } else {
      jtf[0] = jtf[1] = jtf[2] = 0.0;
    }
    al = alpha;
    bd = beta / det;
    ess = ess_;
  }
  __device__ __forceinline__ bool ess_dof(int i) const { return i >= 12 && ((ess >> ((i - 12) >> 2)) & 1u); }
  // alpha G[c][0..2] for a lane-varying component c, blended with exact 0/1
  // weights (a select chain over an array would become scratch memory)
  __device__ __forceinline__ void arow(int c, double (&ag)[3]) const {
    const double w0 = c == 0 ? 1.0 : 0.0, w1 = c == 1 ? 1.0 : 0.0, w2 = c == 2 ? 1.0 : 0.0;
    ag[0] = al * (w0 * g00 + w1 * g01 + w2 * g02);
    ag[1] = al * (w0 * g01 + w1 * g11 + w2 * g12);
    ag[2] = al * (w0 * g02 + w1 * g12 + w2 * g22);
  }
  __device__ __forceinline__ double jsel(int c) const {
    const double w0 = c == 0 ? 1.0 : 0.0, w1 = c == 1 ? 1.0 : 0.0, w2 = c == 2 ? 1.0 : 0.0;
    return w0 * jtf[0] + w1 * jtf[1] + w2 * jtf[2];
  }
};

// Unscaled right-hand side entry of local dof i: the load term (J^T f)_d s_i
// minus the boundary correction sum_j M_ij g_j over boundary dofs j, or g_i
// on a boundary dof.  The setup kernel accumulates the same terms in the same
// order, so both paths agree bitwise.
__device__ __forceinline__ double rhs_entry(const Elem& el, const DeviceMaps& mp, int i, const double* gb) {
  const double2* TD = reinterpret_cast<const double2*>(mp.tab_ref);
  const double* sr = mp.tab_ref + 2 * N * N;
  if (el.ess_dof(i)) return gb ? gb[i - 12] : 0.0;
  double corr = 0.0;
  if (gb && el.ess) {
    double ag[3];
    el.arow(comp(i), ag);
#pragma unroll
    for (int j = 12; j < 36; ++j) {
      const double2 td = TD[j * N + i];
      const double v = fma(ag[comp(j)], td.x, el.bd * td.y);
      corr = fma(el.ess_dof(j) ? v : 0.0, gb[j - 12], corr);
    }
  }
  return el.jsel(comp(i)) * sr[i] - corr;
}

// Power-of-two scale 2^-floor(E/2) for a diagonal entry d = m 2^E, so that
// the scaled diagonal lies in [0.5, 2).
__device__ __forceinline__ double pow2_scale(double d) {
  if (!(d > 0.0) || !isfinite(d)) return 1.0;
  int E;
  (void)frexp(d, &E);
  return ldexp(1.0, -(E >> 1));
}

// LDS strides put the element slots of a wave in different banks: 370 and 36
// doubles are 4 and 8 dwords apart modulo 32 banks.
constexpr int SSTRIDE = 370;   // staging of up to 366 outputs per element

constexpr int SETUP_WAVES = 4;   // waves per setup workgroup (16 elements)

// Per-wave LDS of the setup kernel.
// Per-element inputs of a wave's 4 elements, as one 1 KB block of dwords:
// [0, 72) edge vectors J (18 per element), [72, 216) K1Meta (36 per element),
// [216, 224) alpha, [224, 232) beta, [232, 256) f (6 per element).
constexpr int IN_GEO = 0, IN_META = 72, IN_ALPHA = 216, IN_BETA = 224, IN_F = 232, IN_DWORDS = 256;

struct SetupWaveLds {
  double stage[SETUP_EPW][SSTRIDE];      // outputs on their way to HBM
  alignas(16) uint32_t in[IN_DWORDS];    // inputs of the wave's elements
};

// Direct-to-LDS copy of the inputs of elements e0 .. e0 + 3 (indices past the
// last element are clamped to it).  Completion is awaited with vmcnt.
__device__ __forceinline__ void load_inputs(uint32_t* in, const DeviceMaps& mp, const double* alpha,
                                            const double* beta, const double* f, int64_t e0, int64_t ne, int lane) {
#pragma unroll
  for (int q = 0; q < IN_DWORDS / 64; ++q) {
    const int w = 64 * q + lane;
    const uint32_t* base;
    int per, rel;
    if (w < IN_META) {
      base = reinterpret_cast<const uint32_t*>(mp.k1_geo), per = 18, rel = w - IN_GEO;
    } else if (w < IN_ALPHA) {
      base = reinterpret_cast<const uint32_t*>(mp.k1_meta), per = 36, rel = w - IN_META;
    } else if (w < IN_BETA) {
      base = reinterpret_cast<const uint32_t*>(alpha), per = 2, rel = w - IN_ALPHA;
    } else if (w < IN_F) {
      base = reinterpret_cast<const uint32_t*>(beta), per = 2, rel = w - IN_BETA;
    } else {
      base = reinterpret_cast<const uint32_t*>(f ? f : alpha), per = f ? 6 : 2, rel = f ? w - IN_F : 0;
    }
    const int k = rel / per;
    int64_t el = e0 + k;
    el = el < ne ? el : ne - 1;
    __builtin_amdgcn_global_load_lds(base + el * per + (rel - k * per), (__attribute__((address_space(3))) void*)(in + 64 * q),
                                     4, 0, 0);
  }
}
struct alignas(16) SetupLds {
  double2 td[N * N];   // reference integrals {T_ij, Dv_ij}, shared by the workgroup
  double sr[N];
  SetupWaveLds w[SETUP_WAVES];
};

// Order the LDS accesses of the lanes of one wave (a wave executes its LDS
// instructions in order, so no wait is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Copy the first len doubles of each element slot's staging area to the
// records of elements e0 .. e0 + EPW - 1 at offset off, as coalesced 16-byte
// stores.
template <int EPW>
__device__ __forceinline__ void write_records(double* factor, const double (*stage)[SSTRIDE], int64_t e0, int64_t ne,
                                              int off, int len) {
  const int h2 = len / 2;
  for (int c = threadIdx.x & 63; c < EPW * h2; c += 64) {
    const int tm = c / h2, p = c - tm * h2;
    if (e0 + tm < ne)
      *reinterpret_cast<double2*>(factor + (e0 + tm) * REC + off + 2 * p) =
          *reinterpret_cast<const double2*>(&stage[tm][2 * p]);
  }
}

// Pivot data of one Gauss-Jordan step: 1/d and d - 1 (the value the pivot
// entry takes in the update).  A pivot that is not positive is recorded in
// bad and replaced by 1.
struct Pivot {
  double inv, pc;
};
__device__ __forceinline__ Pivot make_pivot(double d, unsigned& bad) {
  const bool ok = d > 0.0;
  bad |= ok ? 0u : 1u;
  d = ok ? d : 1.0;
  return {1.0 / d, d - 1.0};
}

// Pivot S of the sweep as seen by every lane of the element's row: interior
// pivot S (S < 12) is R[S] of lane S, face pivot K = S - 12 is column S of the
// face row K, i.e. A of lane K (K < 12) or B of lane K - 12.
template <int S>
__device__ __forceinline__ double pivot_value(const double (&R)[37], const double (&A)[37], const double (&B)[37]) {
  if constexpr (S < 12) return row_bcast<S>(R[S]);
  else if constexpr (S < 24) return row_bcast<S - 12>(A[S]);
  else return row_bcast<S - 24>(B[S]);
}

// Step S of the sweep (S < 12: interior pivot S over all three rows; S >= 12:
// face pivot S - 12 over the face rows, face columns and rhs).  Column S + 1
// holds the next pivot: it is updated first, so that the next division
// overlaps the rest of this step.
template <int S>
__device__ __forceinline__ Pivot sweep_step(double (&R)[37], double (&A)[37], double (&B)[37], int t, Pivot pv,
                                            unsigned& bad) {
  constexpr bool INT = S < 12;
  constexpr int L = S < 12 ? S : (S - 12) % 12;   // lane holding the pivot row
  const bool own = t == L;
  double mi = 0.0, ma, mb;
  if constexpr (INT) {
    mi = own ? 1.0 - pv.inv : R[S] * pv.inv;
    ma = A[S] * pv.inv;
    mb = B[S] * pv.inv;
  } else {
    ma = (S < 24 && own) ? 1.0 - pv.inv : A[S] * pv.inv;
    mb = (S >= 24 && own) ? 1.0 - pv.inv : B[S] * pv.inv;
  }
  auto col = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    double p;
    if constexpr (j == S) p = pv.pc;
    else if constexpr (INT) p = row_bcast<L>(R[j]);
    else if constexpr (S < 24) p = row_bcast<L>(A[j]);
    else p = row_bcast<L>(B[j]);
    if constexpr (j > S || (!INT && j >= 12)) {
      // face rows: interior columns still to be pivoted, face columns, rhs
      A[j] = fma(-ma, p, A[j]);
      B[j] = fma(-mb, p, B[j]);
      // (the updates must not sink towards their first use)
      __asm__ volatile("" : "+v"(A[j]), "+v"(B[j]));
    }
    if constexpr (INT) {
      R[j] = fma(-mi, p, R[j]);
      __asm__ volatile("" : "+v"(R[j]));
    }
  };
  constexpr int J0 = INT ? 0 : 12;
  Pivot next{1.0, 0.0};
  if constexpr (S + 1 < 36) {
    col(std::integral_constant<int, S + 1>{});
    next = make_pivot(pivot_value<S + 1>(R, A, B), bad);
  }
  static_for<J0, 37>([&](auto jc) {
    if constexpr (decltype(jc)::value != S + 1 || S + 1 == 36) col(jc);
  });
  return next;
}

template <int S0, int S1>
__device__ __forceinline__ Pivot sweep(double (&R)[37], double (&A)[37], double (&B)[37], int t, Pivot pv,
                                       unsigned& bad) {
  if constexpr (S0 < S1) {
    const Pivot nx = sweep_step<S0>(R, A, B, t, pv, bad);
    return sweep<S0 + 1, S1>(R, A, B, t, nx, bad);
  } else {
    return pv;
  }
}

struct FinalArgs {
  int64_t nfaces;
  const int64_t* rowbase;
  const int32_t* nslots;
  const int32_t* selfslot;
  double* Hval;     // null: leave H alone
  double* r;        // null: leave r alone
  const double* side;
};

__global__ __launch_bounds__(64 * SETUP_WAVES) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_setup_k1(
    SetupArgs a, double* side, int64_t nf) {
  __shared__ SetupLds L;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tau = lane >> 4, t16 = lane & 15;
  const int t = t16 < 12 ? t16 : 0;   // lanes 12..15 shadow lane 0
  const int64_t e0 = (xcd_block() * SETUP_WAVES + wave) * SETUP_EPW;   // first element of this wave
  const int64_t e = e0 + tau;
  const bool valid = e < a.ne;
  const bool live = valid && t16 < 12;
  const int64_t es = valid ? e : 0;
  const DeviceMaps& mp = a.mp;
  const bool rhs = (a.mode & MODE_RHS) != 0;
  const double* gb = (rhs && a.g) ? a.g + es * NB : nullptr;
  SetupWaveLds& W = L.w[wave];

  // inputs of the wave's elements and the reference integrals into LDS
  load_inputs(W.in, mp, a.alpha, a.beta, rhs ? a.f : nullptr, e0 < a.ne ? e0 : a.ne - 1, a.ne, lane);
  {
    const double2* src = reinterpret_cast<const double2*>(mp.tab_ref);
    double2* dst = L.td;
    for (int p = threadIdx.x; p < N * N + N / 2; p += 64 * SETUP_WAVES) dst[p] = src[p];
  }
  __builtin_amdgcn_s_waitcnt(0);   // the direct-to-LDS copies have landed
  __syncthreads();
  const K1Meta& hm = *reinterpret_cast<const K1Meta*>(&W.in[IN_META + 36 * tau]);
  Elem el;
  {
    const double* in = reinterpret_cast<const double*>(W.in);
    unsigned ess = 0;
#pragma unroll
    for (int fc = 0; fc < 6; ++fc)
      if (hm.fid[fc] < 0) ess |= 1u << fc;
    el.from(in + (IN_GEO / 2) + 9 * tau, in[IN_ALPHA / 2 + tau], in[IN_BETA / 2 + tau],
            rhs ? in + IN_F / 2 + 3 * tau : nullptr, ess);
  }
  if (live && t == 0 && !(el.det > 0.0)) report_error(a.status, HYB_E_JACOBIAN, e);

  const double2* TD = L.td;
  const double* sr = L.sr;
  const int ia = 12 + t, ib = 24 + t;   // local dofs of the two face rows
  const int ci = t >> 2, ca = t >> 3, cb = (12 + t) >> 3;
  double agi[3], aga[3], agb[3];
  el.arow(ci, agi);
  el.arow(ca, aga);
  el.arow(cb, agb);

  // ---- scales of the three rows, from their diagonal entries ----
  // (same operations as the corresponding entries of the assembled rows)
  auto diag_of = [&](int i, const double (&ag)[3], int c) {
    const double2 td = TD[i * N + i];
    const double w0 = c == 0 ? 1.0 : 0.0, w1 = c == 1 ? 1.0 : 0.0, w2 = c == 2 ? 1.0 : 0.0;
    return fma(w0 * ag[0] + w1 * ag[1] + w2 * ag[2], td.x, el.bd * td.y);
  };
  const double si = pow2_scale(diag_of(t, agi, ci));
  const double sa = el.ess_dof(ia) ? 1.0 : pow2_scale(diag_of(ia, aga, ca));
  const double sb = el.ess_dof(ib) ? 1.0 : pow2_scale(diag_of(ib, agb, cb));
  // scale of local dof j, from the lane that holds its row
  auto sig = [&](auto jc) -> double {
    constexpr int j = decltype(jc)::value;
    if constexpr (j < 12) return row_bcast<j>(si);
    else if constexpr (j < 24) return row_bcast<j - 12>(sa);
    else return row_bcast<j - 24>(sb);
  };

  // ---- assembly of the three scaled rows ----
  // The boundary correction of the right-hand side is accumulated from the
  // unscaled entries in the order rhs_entry uses.
  auto gval = [&](int j) { return gb ? gb[j - 12] : 0.0; };
  double R[37], A[37], B[37];
  double cri = 0.0, cra = 0.0, crb = 0.0;
  const bool ei = false, ea = el.ess_dof(ia), eb = el.ess_dof(ib);
  auto entry = [&](int i, int j, bool erow, const double (&ag)[3], double& cr) {
    const double2 td = TD[j * N + i];
    const double v = fma(ag[comp(j)], td.x, el.bd * td.y);
    const bool ej = el.ess_dof(j);
    if (j >= 12 && rhs) cr = fma(ej ? v : 0.0, gval(j), cr);
    return (erow || ej) ? (i == j ? 1.0 : 0.0) : v;
  };
  static_for<0, 36>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const double sj = sig(jc);
    R[j] = entry(t, j, ei, agi, cri) * (si * sj);
    A[j] = entry(ia, j, ea, aga, cra) * (sa * sj);
    B[j] = entry(ib, j, eb, agb, crb) * (sb * sj);
    __asm__ volatile("" : "+v"(R[j]), "+v"(A[j]), "+v"(B[j]));   // keep the entries computed here
  });
  R[36] = rhs ? si * (el.jsel(ci) * sr[t] - cri) : 0.0;
  A[36] = rhs ? sa * (ea ? gval(ia) : el.jsel(ca) * sr[ia] - cra) : 0.0;
  B[36] = rhs ? sb * (eb ? gval(ib) : el.jsel(cb) * sr[ib] - crb) : 0.0;

  // ---- sweep of the interior pivots over all rows ----
  unsigned bad = 0;
  Pivot pv = make_pivot(pivot_value<0>(R, A, B), bad);
  pv = sweep<0, 12>(R, A, B, t, pv, bad);

  // ---- interior outputs: A_ii^{-1} row t, E row t, y_i ----
  // A_ii^{-1}[t][j] = -s_t s_j (R[j] - 2 delta_tj), E[t][b] = s_t / s_b R[12 + b]
  {
    double* st = W.stage[tau];
    static_for<0, 12>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const double v = -(R[j] - (j == t ? 2.0 : 0.0)) * (si * sig(jc));
      if (t16 < 12 && j <= t) st[t * (t + 1) / 2 + j] = v;
    });
    static_for<12, 36>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const double v = R[j] * (si / sig(jc));
      if (t16 < 12) st[OFF_E + 24 * t + (j - 12)] = v;
    });
  }
  if (live && rhs) a.y[e * N + t] = R[36] * si;
  wave_sync();
  write_records<SETUP_EPW>(a.factor, W.stage, e0, a.ne, 0, OFF_SI);

  // ---- sweep of the face pivots over the face rows ----
  sweep<12, 36>(R, A, B, t, pv, bad);
  if (live && t == 0 && bad) report_error(a.status, HYB_E_NOT_SPD, e);

  // ---- face outputs: S^{-1} rows, y_b, r_T; then the record and H_T ----
  // S^{-1}[a][b] = -s_a s_b (S[a][b] - 2 delta_ab), lower triangle staged by rows
  wave_sync();   // the record copy above has read the staging area
  auto face_out = [&](const double (&S)[37], int arow, double s_a) {
    double* st = W.stage[tau];
    static_for<12, 36>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr int b = j - 12;
      const double v = -(S[j] - (b == arow ? 2.0 : 0.0)) * (s_a * sig(jc));
      if (t16 < 12 && b <= arow) st[arow * (arow + 1) / 2 + b] = v;
    });
    if (!live || !rhs) return;
    const double z = S[36] * s_a;
    a.y[e * N + 12 + arow] = z;
    const int fa = arow >> 2;
    const int Fa = hm.fid[fa];
    if (Fa < 0) return;
    const int ja = own_idx(hm.pi[fa], arow & 3);
    const double v = (fa & 1) ? z : -z;
    if ((hm.own >> fa) & 1) a.r[int64_t(Fa) * 4 + ja] = v;
    else side[nf * 16 + int64_t(Fa) * 4 + ja] = v;
  };
  face_out(A, t, sa);
  face_out(B, 12 + t, sb);
  wave_sync();
  write_records<SETUP_EPW>(a.factor, W.stage, e0, a.ne, OFF_SI, 300);
  // H_T = D S^{-1} D into the CSR rows: every 4-entry row segment (one face
  // row against the 4 dofs of one face) is written as two 16-byte halves by
  // two adjacent lanes.  A same-face block goes in place from the face's
  // owner and to the side buffer from its neighbour.
  for (int c = lane; c < SETUP_EPW * 288; c += 64) {
    const int tm = c / 288, rem = c - tm * 288;
    const int arow = rem / 12, fb = (rem >> 1) % 6, half = rem & 1;
    if (e0 + tm >= a.ne) continue;
    const K1Meta& hq = *reinterpret_cast<const K1Meta*>(&W.in[IN_META + 36 * tm]);
    const int fa = arow >> 2;
    const int Fa = hq.fid[fa], Fb = hq.fid[fb];
    if (Fa < 0 || Fb < 0) continue;
    const int ja = own_idx(hq.pi[fa], arow & 3);
    // element-frame dofs of the owner-frame positions 2 half and 2 half + 1
    const int pb = hq.pi[fb];
    int i2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int p0 = q, p1 = half;
      if (pb & 2) p0 = 1 - p0;
      if (pb & 4) p1 = 1 - p1;
      if (pb & 1) {
        const int tq = p0;
        p0 = p1;
        p1 = tq;
      }
      i2[q] = p0 + 2 * p1;
    }
    const double sg = ((fa ^ fb) & 1) ? -1.0 : 1.0;   // eps_a eps_b
    const double* st = W.stage[tm];
    const double2 v = make_double2(sg * st[spk(arow, 4 * fb + i2[0])], sg * st[spk(arow, 4 * fb + i2[1])]);
    double* dst;
    if (fb == fa && !((hq.own >> fa) & 1)) dst = side + int64_t(Fa) * 16 + ja * 4 + 2 * half;
    else dst = a.Hval + hq.rb[fa] + int64_t(ja) * hq.ns[fa] * 4 + int64_t(hq.slot[fa * 6 + fb]) * 4 + 2 * half;
    *reinterpret_cast<double2*>(dst) = v;
  }
}

// Add the neighbours' terms of the same-face blocks of H (16 per face, owner
// frame, row-major) and of r (4 per face) from the side buffer.
// One thread per face row (4 per face): its 4-entry same-face segment of H
// (two 16-byte halves) and its entry of r.
__global__ __launch_bounds__(256) void k_finalize_k1(FinalArgs a) {
  const int64_t nrows = a.nfaces * 4;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nrows; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t F = i >> 2;
    const int ja = int(i & 3);
    if (a.Hval) {
      double2* h = reinterpret_cast<double2*>(a.Hval + a.rowbase[F] + int64_t(ja) * a.nslots[F] * 4 +
                                              int64_t(a.selfslot[F]) * 4);
      const double2* sd = reinterpret_cast<const double2*>(a.side + 4 * i);
      double2 h0 = h[0], h1 = h[1];
      const double2 s0 = sd[0], s1 = sd[1];
      h0.x += s0.x;
      h0.y += s0.y;
      h1.x += s1.x;
      h1.y += s1.y;
      h[0] = h0;
      h[1] = h1;
    }
    if (a.r) a.r[i] += a.side[a.nfaces * 16 + i];
  }
}

// ---------------------------------------------------------------------------
// Right-hand side on stored factors, and recovery.  The wave stages the
// records of its five elements (contiguous in HBM) in LDS with coalesced
// 16-byte loads, then each team works on its element.
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
  double* side;     // neighbour terms of r (4 per face after 16 per face of H)
  int64_t nfaces;
};

// Records of the SOLVE_EPW elements of a wave, copied HBM -> LDS by the
// direct-to-LDS loads of gfx950 (1 KB per instruction, no registers), each
// into a 6 KB + 16 B slot: the slots are 4 dwords apart modulo the LDS banks
// and hold the overhang of the last, partial chunk of a record.
constexpr int REC_CHUNKS = (REC * 8 + 1023) / 1024;   // 6
constexpr int RSLOT = REC_CHUNKS * 128 + 2;           // doubles per slot
// the recovery reads only E and S^{-1} (doubles OFF_E .. OFF_SI + 300)
constexpr int REC_CHUNKS_R = ((OFF_SI + 300 - OFF_E) * 8 + 1023) / 1024;   // 5
constexpr int RSLOT_R = REC_CHUNKS_R * 128 + 2;
static_assert((OFF_E * 8) % 16 == 0, "16-byte aligned copy start");

template <int SLOT>
struct alignas(16) SolveLdsT {
  double rec[SOLVE_EPW * SLOT];
  double v[SOLVE_EPW + 1][49];   // per-team exchange vectors
};
using SolveLds = SolveLdsT<RSLOT>;

// Recovery: the exchange vector of a team lives in its slot's tail (past the
// 588 doubles of E and S^{-1}, written once the copies have landed), so the
// wave needs 26 KB of LDS and six waves fit on a CU.
constexpr int RTAIL = OFF_SI + 300 - OFF_E;   // 588
static_assert(RSLOT_R - RTAIL >= 49, "exchange vector fits in the slot tail");
struct alignas(16) RecoverLds {
  double rec[SOLVE_EPW * RSLOT_R];
  double vspare[49];             // the wave's idle lanes
};

// Record of element min(e0 + k, ne - 1) into slot k; lane i of chunk q moves
// bytes q KB + 16 i of the record, clamped to its last 16 bytes.
// Copy doubles FIRST .. of each of the wave's SOLVE_EPW element records into
// LDS slots of SLOT doubles, CHUNKS x 1 KB per record (the last chunk's
// lanes past the record's end re-read its last 16 bytes).
template <int FIRST, int CHUNKS, int SLOT>
__device__ __forceinline__ void stage_records(double* dst, const double* factor, int64_t e0, int64_t ne) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < SOLVE_EPW; ++k) {
    int64_t el = e0 + k;
    el = el < ne ? el : ne - 1;
    const char* base = reinterpret_cast<const char*>(factor + el * REC);
#pragma unroll
    for (int q = 0; q < CHUNKS; ++q) {
      int off = FIRST * 8 + q * 1024 + 16 * lane;
      off = off < REC * 8 - 16 ? off : REC * 8 - 16;
      __builtin_amdgcn_global_load_lds(base + off,
                                       (__attribute__((address_space(3))) void*)(dst + k * SLOT + 128 * q), 16, 0, 0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);   // all counters: the LDS copies have landed
}

__global__ __launch_bounds__(64) void k_rhs_k1(SimtArgs a) {
  __shared__ SolveLds L;
  const int lane = threadIdx.x, tau = lane / TEAM, t = lane - tau * TEAM;
  const int64_t e0 = xcd_block() * SOLVE_EPW;
  const int64_t e = e0 + tau;
  const bool live = tau < SOLVE_EPW && e < a.ne;
  const int64_t es = live ? e : 0;
  const DeviceMaps& mp = a.mp;
  stage_records<0, REC_CHUNKS, RSLOT>(L.rec, a.factor, e0, a.ne);
  const double* gb = a.g ? a.g + es * NB : nullptr;
  Elem el;
  el.load(mp, es, a.alpha, a.beta, a.f, gb != nullptr);
  const double fi = rhs_entry(el, mp, t, gb);
  const double fa = rhs_entry(el, mp, 12 + t, gb);
  const double fb = rhs_entry(el, mp, 24 + t, gb);
  double* v = L.v[tau];
  v[t] = fi;
  __syncthreads();
  const double* rec = L.rec + (live ? tau : 0) * RSLOT;
  // y_i = A_ii^{-1} f_i; t_b = f_b - E^T f_i
  double yi = 0.0, ta = fa, tb = fb;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double fc = v[c];
    yi = fma(rec[spk(t, c)], fc, yi);
    ta = fma(-rec[OFF_E + 24 * c + t], fc, ta);
    tb = fma(-rec[OFF_E + 24 * c + 12 + t], fc, tb);
  }
  v[12 + t] = ta;
  v[24 + t] = tb;
  __syncthreads();
  // z = S^{-1} t_b
  double za = 0.0, zb = 0.0;
#pragma unroll
  for (int b = 0; b < 24; ++b) {
    const double tv = v[12 + b];
    za = fma(rec[OFF_SI + spk(t, b)], tv, za);
    zb = fma(rec[OFF_SI + spk(12 + t, b)], tv, zb);
  }
  if (!live) return;
  a.y[e * N + t] = yi;
  a.y[e * N + 12 + t] = za;
  a.y[e * N + 24 + t] = zb;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int arow = 12 * h + t;
    const int fc = arow >> 2;
    const int F = mp.elem_face[e * 6 + fc];
    if (F < 0) continue;
    const int ja = own_idx(mp.elem_pi[e * 8 + fc], arow & 3);
    const double z = h ? zb : za;
    const double v = (fc & 1) ? z : -z;
    if (mp.face_owner[F] == e) a.r[int64_t(F) * 4 + ja] = v;
    else a.side[a.nfaces * 16 + int64_t(F) * 4 + ja] = v;
  }
}

__global__ __launch_bounds__(64) void k_recover_k1(SimtArgs a) {
  __shared__ RecoverLds L;
  const int lane = threadIdx.x, tau = lane / TEAM, t = lane - tau * TEAM;
  const int64_t e0 = xcd_block() * SOLVE_EPW;
  const int64_t e = e0 + tau;
  const bool live = tau < SOLVE_EPW && e < a.ne;
  const int64_t es = live ? e : 0;
  const DeviceMaps& mp = a.mp;
  // D lambda on the two face rows of this lane and y, loaded before the
  // record copies are issued so that both are in flight together
  double lam2[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int arow = 12 * h + t;
    const int fc = arow >> 2;
    const int F = mp.elem_face[es * 6 + fc];
    double x = 0.0;
    if (F >= 0) {
      x = a.lambda[int64_t(F) * 4 + own_idx(mp.elem_pi[es * 8 + fc], arow & 3)];
      if (!(fc & 1)) x = -x;
    }
    lam2[h] = x;
  }
  const double yi = a.y[es * N + t], ya = a.y[es * N + 12 + t], yb = a.y[es * N + 24 + t];
  stage_records<OFF_E, REC_CHUNKS_R, RSLOT_R>(L.rec, a.factor, e0, a.ne);
  double* v = tau < SOLVE_EPW ? L.rec + tau * RSLOT_R + RTAIL : L.vspare;
  v[t] = lam2[0];
  v[12 + t] = lam2[1];
  __syncthreads();
  // the slot starts at E (record offset OFF_E); S^{-1} follows at OFF_SI - OFF_E
  const double* slot = L.rec + (live ? tau : 0) * RSLOT_R;
  const double* Si = slot + (OFF_SI - OFF_E);
  // u_b = y_b - S^{-1} D lambda
  double ua = ya, ub = yb;
#pragma unroll
  for (int b = 0; b < 24; ++b) {
    const double tl = v[b];
    ua = fma(-Si[spk(t, b)], tl, ua);
    ub = fma(-Si[spk(12 + t, b)], tl, ub);
  }
  v[24 + t] = ua;
  v[36 + t] = ub;
  __syncthreads();
  // u_i = y_i - E u_b
  double ui = yi;
#pragma unroll
  for (int b = 0; b < 24; ++b) ui = fma(-slot[24 * t + b], v[24 + b], ui);
  if (!live) return;
  a.u[e * N + t] = ui;
  a.u[e * N + 12 + t] = ua;
  a.u[e * N + 24 + t] = ub;
}

}  // namespace k1
}  // namespace hyb
