// Jacobi-preconditioned CG on the CSR matrix H with deterministic reductions:
// every block reduces a fixed contiguous range of rows in a fixed tree order,
// and a one-block kernel sums the per-block partials in index order.  (A
// "last block sums" handshake inside the producing kernel would need an
// agent-scope release per block, which writes back the XCD's L2 each time.)
// Per iteration: SpMV with the direction update folded in (p double-buffered),
// sum -> alpha, vector update, sum -> beta.
#pragma once

#include "kernels_common.hpp"

namespace hyb {

constexpr int kPcgThreads = 256;

// Scalars kept on the device between kernels.
struct PcgScalars {
  double rz;       // r . z of the current iterate
  double pq;       // p . H p
  double rr;       // r . r
  double rr0;
  double alpha;
  double beta;     // direction update of the next SpMV (0 before the first)
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

// dinv = 1 / diag(H); x = 0; r = b; z = dinv r; p_prev = 0; partial r.z, r.r.
// LPR lanes per row look for the diagonal entry.
template <int LPR>
__global__ __launch_bounds__(kPcgThreads) void k_pcg_init(int64_t m, const int64_t* rp, const int32_t* ci,
                                                       const double* val, const double* b, double* x,
                                                       double* r, double* z, double* p0, double* dinv,
                                                       double* part, int nblk) {
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
    part[2 * lb] = srz;
    part[2 * lb + 1] = srr;
  }
}

// New search direction of entry j: z + beta p_prev (one expression, so every
// block that needs entry j forms the same value).
__device__ __forceinline__ double direction(const double* z, const double* pp, double be, int64_t j) {
  return __builtin_fma(be, pp[j], z[j]);
}

// p = z + beta p_prev (own rows, into the other p buffer) and q = H p over
// face panels, gathering z + beta p_prev for the panel columns; partial p.q.
// Matrix entries are streamed once (non-temporal loads), the vectors stay in
// cache.  Each row's sum runs over the panel columns in a fixed order: per
// lane in column order, then a fixed butterfly over the L lanes.
template <int K2, int L, int CPL>
__global__ __launch_bounds__(kPcgThreads) void k_pcg_spmv(int64_t nfb, const int64_t* rp, const int32_t* ci,
                                                       const double* val, const double* z, const double* pp,
                                                       double* p, double* q, const PcgScalars* sc, double* part,
                                                       int nblk) {
  static_assert(L >= K2 && (L & (L - 1)) == 0, "one lane per panel row for the output");
  __shared__ double red[kPcgThreads];
  constexpr int G = kPcgThreads / L;
  const int lb = pcg_block();
  int64_t lo, hi;
  chunk(nfb, nblk, lb, lo, hi);
  const double be = sc->beta;
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
  if (threadIdx.x == 0) part[lb] = s;
}

// One block: sums of the partials in index order (contiguous runs per thread,
// then the fixed tree).  stride 1: part[i] (p.q); stride 2: part[2i], part[2i+1]
// (r.z, r.r).  which = 0: init (rz, rr, rr0, beta = 0); 1: alpha = rz / pq;
// 2: beta = rz_new / rz, rz = rz_new, rr.
__global__ __launch_bounds__(kPcgThreads) void k_pcg_reduce(const double* part, int nblk, PcgScalars* sc,
                                                         int which) {
  __shared__ double red[kPcgThreads];
  const int stride = which == 1 ? 1 : 2;
  double s0 = 0.0, s1 = 0.0;
  const int per = (nblk + kPcgThreads - 1) / kPcgThreads;
  for (int i = threadIdx.x * per; i < (threadIdx.x + 1) * per && i < nblk; ++i) {
    s0 += part[stride * i];
    if (stride == 2) s1 += part[2 * i + 1];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    if (which == 0) {
      sc->rz = s0;
      sc->rr = s1;
      sc->rr0 = s1;
      sc->beta = 0.0;
    } else if (which == 1) {
      sc->pq = s0;
      sc->alpha = s0 != 0.0 ? sc->rz / s0 : 0.0;
    } else {
      sc->beta = sc->rz != 0.0 ? s0 / sc->rz : 0.0;
      sc->rz = s0;
      sc->rr = s1;
    }
  }
}

// x += alpha p; r -= alpha q; z = dinv r; partial r.z, r.r
__global__ __launch_bounds__(kPcgThreads) void k_pcg_update(int64_t m, const PcgScalars* sc, const double* p,
                                                         const double* q, const double* dinv, double* x,
                                                         double* r, double* z, double* part, int nblk) {
  __shared__ double red[kPcgThreads];
  const int lb = pcg_block();
  int64_t lo, hi;
  chunk(m, nblk, lb, lo, hi);
  const double al = sc->alpha;
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
    part[2 * lb] = srz;
    part[2 * lb + 1] = srr;
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
