// Jacobi-preconditioned CG on the CSR matrix H with deterministic reductions:
// every block reduces a fixed contiguous range in a fixed tree order, and one
// block sums the per-block partials in index order.
#pragma once

#include "kernels_common.hpp"

namespace hyb {

constexpr int kPcgThreads = 256;

// Scalars kept on the device between kernels.
struct PcgScalars {
  double rz;       // r . z
  double rz_new;
  double pq;       // p . H p
  double rr;       // r . r
  double rr0;
  double alpha;
  double beta;
  double pad;
};

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

// Rows [lo, hi) of each block: a contiguous chunk so partial sums are fixed.
__device__ __forceinline__ void chunk(int64_t m, int nblk, int64_t& lo, int64_t& hi) {
  const int64_t per = (m + nblk - 1) / nblk;
  lo = int64_t(blockIdx.x) * per;
  hi = lo + per < m ? lo + per : m;
}

// dinv = 1 / diag(H); x = 0; r = b; z = dinv r; p = z; partial r.z and r.r
__global__ __launch_bounds__(kPcgThreads) void k_pcg_init(int64_t m, const int64_t* rp, const int32_t* ci,
                                                       const double* val, const double* b, double* x,
                                                       double* r, double* z, double* p, double* dinv,
                                                       double* part, int nblk) {
  __shared__ double red[kPcgThreads];
  int64_t lo, hi;
  chunk(m, nblk, lo, hi);
  double srz = 0.0, srr = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPcgThreads) {
    double d = 0.0;
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
      if (ci[q] == i) d = val[q];
    const double di = d != 0.0 ? 1.0 / d : 0.0;
    dinv[i] = di;
    x[i] = 0.0;
    const double ri = b[i];
    r[i] = ri;
    const double zi = di * ri;
    z[i] = zi;
    p[i] = zi;
    srz += ri * zi;
    srr += ri * ri;
  }
  srz = block_sum(srz, red);
  srr = block_sum(srr, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = srz;
    part[2 * blockIdx.x + 1] = srr;
  }
}

// q = H p, partial p.q
__global__ __launch_bounds__(kPcgThreads) void k_pcg_spmv(int64_t m, const int64_t* rp, const int32_t* ci,
                                                       const double* val, const double* p, double* q,
                                                       double* part, int nblk) {
  __shared__ double red[kPcgThreads];
  int64_t lo, hi;
  chunk(m, nblk, lo, hi);
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPcgThreads) {
    double acc = 0.0;
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) acc += val[t] * p[ci[t]];
    q[i] = acc;
    s += p[i] * acc;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[2 * blockIdx.x] = s;
}

// Single-block sum of the partials in index order.
// which = 0: init (rz, rr0, rr); 1: alpha = rz / pq; 2: beta = rz_new / rz.
__global__ __launch_bounds__(kPcgThreads) void k_pcg_reduce(const double* part, int nblk, PcgScalars* sc,
                                                         int which) {
  __shared__ double red[kPcgThreads];
  double s0 = 0.0, s1 = 0.0;
  // each thread sums a contiguous run, then the fixed tree
  const int per = (nblk + kPcgThreads - 1) / kPcgThreads;
  for (int i = threadIdx.x * per; i < (threadIdx.x + 1) * per && i < nblk; ++i) {
    s0 += part[2 * i];
    s1 += part[2 * i + 1];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    if (which == 0) {
      sc->rz = s0;
      sc->rr = s1;
      sc->rr0 = s1;
    } else if (which == 1) {
      sc->pq = s0;
      sc->alpha = s0 != 0.0 ? sc->rz / s0 : 0.0;
    } else {
      sc->rz_new = s0;
      sc->rr = s1;
      sc->beta = sc->rz != 0.0 ? s0 / sc->rz : 0.0;
      sc->rz = s0;
    }
  }
}

// x += alpha p; r -= alpha q; z = dinv r; partial r.z, r.r
__global__ __launch_bounds__(kPcgThreads) void k_pcg_update(int64_t m, const PcgScalars* sc, const double* p,
                                                         const double* q, const double* dinv, double* x,
                                                         double* r, double* z, double* part, int nblk) {
  __shared__ double red[kPcgThreads];
  int64_t lo, hi;
  chunk(m, nblk, lo, hi);
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
    part[2 * blockIdx.x] = srz;
    part[2 * blockIdx.x + 1] = srr;
  }
}

// p = z + beta p
__global__ __launch_bounds__(kPcgThreads) void k_pcg_direction(int64_t m, const PcgScalars* sc, const double* z,
                                                            double* p) {
  const double be = sc->beta;
  for (int64_t i = int64_t(blockIdx.x) * kPcgThreads + threadIdx.x; i < m; i += int64_t(gridDim.x) * kPcgThreads)
    p[i] = z[i] + be * p[i];
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
