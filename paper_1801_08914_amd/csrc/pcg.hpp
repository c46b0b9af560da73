// Jacobi-preconditioned CG on the CSR matrix H:
//   SpMV j:    beta_{j-1} = rz_j / rz_{j-1};  p_j = z_j + beta_{j-1} p_{j-1};
//              q_j = H p_j;  partials of p_j . q_j
//   update j:  alpha_j = rz_j / (p_j . q_j);  x += alpha_j p_j;
//              r -= alpha_j q_j;  z = D^{-1} r;  partials of r.z and r.r
// Reductions are deterministic: every block reduces a fixed contiguous range
// of rows in a fixed tree order, and the per-block partials are summed in
// index order by one routine (sum_partials).  Who sums them depends on size:
// * in-kernel (small systems, launch-bound): every block of the consuming
//   kernel sums the producing kernel's partials itself, so all blocks hold
//   the same scalar bit for bit; two launches per iteration;
// * separate (large systems, where every block reading every partial would
//   cost more L2 traffic than two more launches): a one-block kernel after
//   each of the two forms the scalar.
// Both give the same bits.  (A "last block sums" handshake would need an
// agent-scope release per block, which writes back the XCD's L2 every time.)
// The update partials alternate between two slots by iteration parity (U_j
// in slot j & 1, the initial ones in slot 1), and p between two buffers.
#pragma once

#include "kernels_common.hpp"

namespace hyb {

constexpr int kPcgThreads = 256;

// Scalars for the host: rr of the current iterate (after a k_pcg_rr launch)
// and rr0; rz_j of each update kernel, by parity (written by its block 0).
struct PcgScalars {
  double rr;
  double rr0;
  double rz[2];
  double alpha;    // separate reductions: alpha_j for update j
  double beta;     // separate reductions: beta_{j-1} for SpMV j
  double pad[2];
};

// Face-panel SpMV.  The K2 = (k+1)^2 rows of an interior face are
// consecutive, have the same columns (the K2 dofs of each neighbouring face)
// and are stored one after the other, so they form a dense row-major K2 x w
// panel at row_ptr[F K2].  L lanes per face take the panel's columns
// c = lane + L j: one column index and one vector entry per column serve all
// K2 rows.  CPL columns per lane are loaded before the first product (rows
// wider than L CPL finish in a loop); each lane group takes two faces.
struct SpmvShape {
  int lanes, faces_per_block;
};

inline SpmvShape spmv_shape(int k) {
  const int lanes = k == 0 ? 4 : k == 1 ? 16 : k == 2 ? 32 : 64;
  return {lanes, 2 * kPcgThreads / lanes};
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  // fixed-order tree over the block
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kPcgThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// Sum of part[stride i + c] over i < n in index order: contiguous runs per
// thread, then the fixed tree; the same value in every block.
__device__ __forceinline__ double sum_partials(const double* part, int n, int stride, int c, double* red) {
  const int per = (n + kPcgThreads - 1) / kPcgThreads;
  const int i0 = threadIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += part[stride * i + c];
  return block_sum(s, red);
}

// Logical block of this workgroup: consecutive logical blocks (consecutive
// rows) go to the same XCD, whose L2 then holds the vector entries that the
// rows of that XCD gather.
__device__ __forceinline__ int pcg_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned q = nb / 8, rem = nb % 8, x = b % 8, i = b / 8;
  return int(x * q + (x < rem ? x : rem) + i);
}

// Rows [lo, hi) of logical block lb: contiguous chunks, so partial sums are fixed.
__device__ __forceinline__ void chunk(int64_t m, int nblk, int lb, int64_t& lo, int64_t& hi) {
  const int64_t per = (m + nblk - 1) / nblk;
  lo = int64_t(lb) * per;
  hi = lo + per < m ? lo + per : m;
}

// dinv = 1 / diag(H); x = 0; r = b; z = dinv r; p_prev = 0; partials of
// r.z, r.r into update slot 1.  LPR lanes per row look for the diagonal entry.
template <int LPR>
__global__ __launch_bounds__(kPcgThreads) void k_pcg_init(int64_t m, const int64_t* rp, const int32_t* ci,
                                                       const double* val, const double* b, double* x,
                                                       double* r, double* z, double* p0, double* dinv,
                                                       double* part_u, int nblk) {
  __shared__ double red[kPcgThreads];
  constexpr int G = kPcgThreads / LPR;
  const int lb = pcg_block();
  int64_t lo, hi;
  chunk(m, nblk, lb, lo, hi);
  const int sub = threadIdx.x % LPR, grp = threadIdx.x / LPR;
  double srz = 0.0, srr = 0.0;
  for (int64_t i = lo + grp; i < hi; i += G) {
    double d = 0.0;
    for (int64_t q = rp[i] + sub; q < rp[i + 1]; q += LPR)
      if (ci[q] == i) d = val[q];
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) d += __shfl_xor(d, off, LPR);   // one nonzero term
    if (sub == 0) {
      const double di = d != 0.0 ? 1.0 / d : 0.0;
      dinv[i] = di;
      x[i] = 0.0;
      p0[i] = 0.0;
      const double ri = b[i];
      r[i] = ri;
      const double zi = di * ri;
      z[i] = zi;
      srz += ri * zi;
      srr += ri * ri;
    }
  }
  srz = block_sum(srz, red);
  srr = block_sum(srr, red);
  if (threadIdx.x == 0) {
    double* u = part_u + 2 * size_t(nblk);   // slot 1
    u[2 * lb] = srz;
    u[2 * lb + 1] = srr;
  }
}

// beta_{it-1} = rz_it / rz_{it-1}: rz_it from the partials of update it - 1
// (slot (it - 1) & 1), rz_{it-1} as update it - 1 recorded it.
__device__ __forceinline__ double pcg_beta(const double* part_u, int nblk_u, const PcgScalars* sc, int it,
                                           double* red) {
  const double rz = sum_partials(part_u + 2 * size_t(nblk_u) * ((it - 1) & 1), nblk_u, 2, 0, red);
  const double rz_prev = sc->rz[(it - 1) & 1];
  return rz_prev != 0.0 ? rz / rz_prev : 0.0;
}

// alpha_it = rz_it / (p.q) from the SpMV partials and those of update it - 1
// (or of the initialisation), slot (it + 1) & 1; rz_it is returned too.
__device__ __forceinline__ double pcg_alpha(const double* part_s, int nblk_s, const double* part_u, int nblk_u,
                                            int it, double* red, double& rz) {
  const double pq = sum_partials(part_s, nblk_s, 1, 0, red);
  rz = sum_partials(part_u + 2 * size_t(nblk_u) * ((it + 1) & 1), nblk_u, 2, 0, red);
  return pq != 0.0 ? rz / pq : 0.0;
}

// New search direction of entry j: z + beta p_prev (one expression, so every
// block that needs entry j forms the same value).
__device__ __forceinline__ double direction(const double* z, const double* pp, double be, int64_t j) {
  return __builtin_fma(be, pp[j], z[j]);
}

// SpMV of iteration it over face panels, gathering z + beta p_prev for the
// panel columns; p_it for the own rows into the other p buffer; partials of
// p.q.  Matrix entries are streamed once (non-temporal loads), the vectors
// stay in cache.  Each row's sum runs over the panel columns in a fixed
// order: per lane in column order, then a fixed butterfly over the L lanes.
template <int K2, int L, int CPL, bool FUSED>
__global__ __launch_bounds__(kPcgThreads) void k_pcg_spmv(int64_t nfb, const int64_t* rp, const int32_t* ci,
                                                       const double* val, const double* z, const double* pp,
                                                       double* p, double* q, const double* part_u, int nblk_u,
                                                       const PcgScalars* sc, int it, double* part_s, int nblk) {
  static_assert(L >= K2 && (L & (L - 1)) == 0, "one lane per panel row for the output");
  __shared__ double red[kPcgThreads];
  constexpr int G = kPcgThreads / L;
  double be = 0.0;
  if (!FUSED) {
    be = it > 0 ? sc->beta : 0.0;
  } else if (it > 0) {
    be = pcg_beta(part_u, nblk_u, sc, it, red);
  }
  const int lb = pcg_block();
  int64_t lo, hi;
  chunk(nfb, nblk, lb, lo, hi);
  const int sub = threadIdx.x % L, grp = threadIdx.x / L;
  double s = 0.0;
  for (int64_t F = lo + grp; F < hi; F += G) {
    const int64_t r0 = F * K2;
    const int64_t base = rp[r0];
    const int w = int(rp[r0 + 1] - base);
    // past the panel's width: weight 0 on the face's own first row (a valid
    // index), so that every load is issued without a branch
    double v[CPL][K2], x[CPL];
    int32_t c[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int col = sub + j * L;
      const bool ok = col < w;
      c[j] = ok ? __builtin_nontemporal_load(ci + base + col) : int32_t(r0);
#pragma unroll
      for (int a = 0; a < K2; ++a)
        v[j][a] = ok ? __builtin_nontemporal_load(val + base + int64_t(a) * w + col) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) x[j] = direction(z, pp, be, c[j]);
    double acc[K2];
#pragma unroll
    for (int a = 0; a < K2; ++a) {
      acc[a] = 0.0;
#pragma unroll
      for (int j = 0; j < CPL; ++j) acc[a] += v[j][a] * x[j];
    }
    for (int col = sub + CPL * L; col < w; col += L) {
      const double xc = direction(z, pp, be, __builtin_nontemporal_load(ci + base + col));
#pragma unroll
      for (int a = 0; a < K2; ++a) acc[a] += __builtin_nontemporal_load(val + base + int64_t(a) * w + col) * xc;
    }
#pragma unroll
    for (int a = 0; a < K2; ++a) {
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) acc[a] += __shfl_xor(acc[a], off, L);
    }
#pragma unroll
    for (int a = 0; a < K2; ++a) {
      if (sub == a) {
        const double pi = direction(z, pp, be, r0 + a);
        p[r0 + a] = pi;
        q[r0 + a] = acc[a];
        s += pi * acc[a];
      }
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part_s[lb] = s;
}

// Update of iteration it: alpha = rz_it / (p.q) from the SpMV partials and
// the partials of update it - 1 (or of the initialisation); x += alpha p;
// r -= alpha q; z = dinv r; partials of r.z, r.r into slot it & 1.  Block 0
// records rz_it for the next SpMV.
template <bool FUSED>
__global__ __launch_bounds__(kPcgThreads) void k_pcg_update(int64_t m, const double* __restrict__ p,
                                                         const double* __restrict__ q,
                                                         const double* __restrict__ dinv, double* __restrict__ x,
                                                         double* __restrict__ r, double* __restrict__ z,
                                                         const double* part_s, int nblk_s, double* part_u,
                                                         PcgScalars* sc, int it, int nblk) {
  __shared__ double red[kPcgThreads];
  double al;
  if (FUSED) {
    double rz;
    al = pcg_alpha(part_s, nblk_s, part_u, nblk, it, red, rz);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->rz[it & 1] = rz;
  } else {
    al = sc->alpha;
  }
  const int lb = pcg_block();
  int64_t lo, hi;
  chunk(m, nblk, lb, lo, hi);
  double srz = 0.0, srr = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPcgThreads) {
    x[i] += al * p[i];
    const double ri = r[i] - al * q[i];
    r[i] = ri;
    const double zi = dinv[i] * ri;
    z[i] = zi;
    srz += ri * zi;
    srr += ri * ri;
  }
  srz = block_sum(srz, red);
  srr = block_sum(srr, red);
  if (threadIdx.x == 0) {
    double* u = part_u + 2 * size_t(nblk) * (it & 1);
    u[2 * lb] = srz;
    u[2 * lb + 1] = srr;
  }
}

// Separate reductions, one block: which = 0: alpha_it (and rz_it recorded
// as the in-kernel form records it) after SpMV it; 1: beta_it for SpMV it + 1
// after update it.
__global__ __launch_bounds__(kPcgThreads) void k_pcg_scalar(const double* part_s, int nblk_s,
                                                         const double* part_u, int nblk_u, PcgScalars* sc, int it,
                                                         int which) {
  __shared__ double red[kPcgThreads];
  if (which == 0) {
    double rz;
    const double al = pcg_alpha(part_s, nblk_s, part_u, nblk_u, it, red, rz);
    if (threadIdx.x == 0) {
      sc->alpha = al;
      sc->rz[it & 1] = rz;
    }
  } else {
    const double be = pcg_beta(part_u, nblk_u, sc, it + 1, red);
    if (threadIdx.x == 0) sc->beta = be;
  }
}

// One block: rr of the update partials in slot `slot` for the host's
// convergence test (and rr0 when first).
__global__ __launch_bounds__(kPcgThreads) void k_pcg_rr(const double* part_u, int nblk, int slot, PcgScalars* sc,
                                                     int first) {
  __shared__ double red[kPcgThreads];
  const double rr = sum_partials(part_u + 2 * size_t(nblk) * slot, nblk, 2, 1, red);
  if (threadIdx.x == 0) {
    sc->rr = rr;
    if (first) sc->rr0 = rr;
  }
}

__global__ void k_fill(double* x, int64_t n, double v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    x[i] = v;
}

// Zero the same-face (diagonal) blocks of H, the only entries that receive
// two element terms (added atomically by the setup kernels).
__global__ void k_zero_diag_blocks(int64_t nfaces, int K2, const int64_t* rowbase, const int32_t* nslots,
                                   const int32_t* selfslot, double* val) {
  const int64_t tot = nfaces * K2 * K2;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < tot; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t F = i / (K2 * K2);
    const int rem = int(i - F * K2 * K2), j = rem / K2, jj = rem % K2;
    val[rowbase[F] + int64_t(j) * nslots[F] * K2 + selfslot[F] * K2 + jj] = 0.0;
  }
}

__global__ void k_fill_i32(int32_t* x, int64_t n, int32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    x[i] = v;
}

}  // namespace hyb
