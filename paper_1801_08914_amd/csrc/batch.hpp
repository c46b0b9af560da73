// Batches of independent problems of mixed order.  FP64 problems: a kernel
// per order and phase (each gets the register allocation, and so the
// occupancy, of the single-plan kernel of that order), launched for up to
// eight problems at a time with their descriptors in the kernel arguments.
// Mixed-precision problems: one persistent launch per phase over a list of
// work items.
#pragma once

#include "kernels_common.hpp"
#include "mixed.hpp"
#include "setup_generic.hpp"
#include "setup_k3.hpp"

namespace hyb {

struct BatchProb {
  SetupArgs s;       // matrix (and optional right-hand side) of the problem
  RecoverArgs r;     // recovery of the problem
  int32_t k;
  int32_t K2;        // (k+1)^2
  int32_t mixed;     // HYB_MIXED problem (the mixed element routines)
  int32_t sweeps;    // its refinement sweeps (< 0: adaptive)
  int64_t nfaces;
  int64_t m;
};

struct BatchItem {
  int32_t prob;
  int32_t nblk;      // element blocks in this item
  int64_t blk0;      // first element block (blocks of the order's EPB elements)
};

// Element blocks of the mixed-precision problems per order (512-thread
// workgroups): 8 x 64, 4 x 128, then one element per block (RT3: its FP64
// element matrix in the workgroup's scratch slot).  The per-element
// arithmetic does not depend on the number of elements per workgroup, so a
// batch gives the single plans' bits.
__host__ __device__ constexpr int batch_epb_mixed(int k) { return k == 0 ? 8 : (k == 1 ? 4 : 1); }
constexpr int kBatchThreads = 512;
constexpr int kBatchThreadsK3 = 512;

// A pointer read from a descriptor in memory is generic (flat) to the
// compiler, and flat accesses count on the LDS wait counter too, so every
// wait for an LDS result would also wait for the memory accesses in flight.
// Every buffer of a problem is in device memory: the batch kernels pass each
// pointer through the global address space, and the element routines
// compile to global loads and stores.
// (The pointers are wave-uniform: rebuilt from scalar registers as global
// pointers, a form the compiler does not fold back to the generic one.)
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
  using G = __attribute__((address_space(1))) T*;
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint64_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
  const uint64_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
  return (T*)reinterpret_cast<G>(lo | (hi << 32));
}

__device__ __forceinline__ DeviceMaps global_maps(DeviceMaps m) {
  m.e2v = as_global(m.e2v);
  m.xyz = as_global(m.xyz);
  m.elem_face = as_global(m.elem_face);
  m.elem_pi = as_global(m.elem_pi);
  m.elem_slot = as_global(m.elem_slot);
  m.face_rowbase = as_global(m.face_rowbase);
  m.face_nslots = as_global(m.face_nslots);
  m.tab_s = as_global(m.tab_s);
  m.tab_d = as_global(m.tab_d);
  m.tab_w = as_global(m.tab_w);
  m.tab_ref = as_global(m.tab_ref);
  m.gauss_x = as_global(m.gauss_x);
  m.face_selfslot = as_global(m.face_selfslot);
  m.face_owner = as_global(m.face_owner);
  m.k1_geo = as_global(m.k1_geo);
  m.k1_meta = as_global(m.k1_meta);
  m.face_w = as_global(m.face_w);
  m.tab1d = as_global(m.tab1d);
  return m;
}

__device__ __forceinline__ SetupArgs global_args(const SetupArgs& s) {
  SetupArgs a = s;
  a.mp = global_maps(s.mp);
  a.alpha = as_global(s.alpha);
  a.beta = as_global(s.beta);
  a.f = as_global(s.f);
  a.g = as_global(s.g);
  a.factor = as_global(s.factor);
  a.y = as_global(s.y);
  a.Hval = as_global(s.Hval);
  a.r = as_global(s.r);
  a.status = as_global(s.status);
  return a;
}

__device__ __forceinline__ RecoverArgs global_args(const RecoverArgs& s) {
  RecoverArgs a = s;
  a.mp = global_maps(s.mp);
  a.factor = as_global(s.factor);
  a.y = as_global(s.y);
  a.lambda = as_global(s.lambda);
  a.u = as_global(s.u);
  return a;
}

// The mixed-precision element routines as separate functions: inlined into
// one persistent kernel, the four bodies share one register allocation (and
// spill); called, each keeps its own.  A call per element block.
template <int K, int TEAM, int EPB>
__device__ __attribute__((noinline)) void batch_setup_mx(const SetupArgs& a, double* smem, int64_t blk, int sweeps,
                                                         double* scratch) {
  setup_mixed_body<K, TEAM, EPB>(global_args(a), smem, blk, sweeps, scratch);
}

// The next work item of a persistent workgroup from the launch's queue
// counter (cleared by a kernel before the launch): thread 0 takes it, the
// workgroup reads it after a barrier.  Items are sorted by cost, so the
// most expensive ones are taken first.
__device__ __forceinline__ int64_t next_item(int32_t* queue, int64_t* slot) {
  __syncthreads();   // every thread has read the previous item
  if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
  __syncthreads();
  return *slot;
}

// Zero the same-face blocks of H (and r) of every problem: blockIdx.y is the
// problem.
__global__ __launch_bounds__(256) void k_batch_zero(const BatchProb* probs) {
  const BatchProb& P = probs[blockIdx.y];
  const int K2 = P.K2;
  const int64_t nd = P.nfaces * K2 * K2;
  const int64_t nr = (P.s.mode & MODE_RHS) ? P.m : 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nd + nr; i += int64_t(gridDim.x) * blockDim.x) {
    if (i < nd) {
      const int64_t F = i / (K2 * K2);
      const int rem = int(i - F * K2 * K2), j = rem / K2, jj = rem % K2;
      P.s.Hval[P.s.mp.face_rowbase[F] + int64_t(j) * P.s.mp.face_nslots[F] * K2 + P.s.mp.face_selfslot[F] * K2 + jj] =
          0.0;
    } else {
      P.s.r[i - nd] = 0.0;
    }
  }
  // the mixed form's count of elements solved in FP64 restarts with the setup
  if (P.mixed && blockIdx.x == 0 && threadIdx.x == 0) P.s.status[2] = 0;
}

// The FP64 problems: per order, launches of up to kMultiProbs problems with
// their descriptors in the kernel arguments, each problem's element blocks a
// consecutive range of the grid (the hardware hands out the workgroups as
// CUs free up), in the single-plan kernels' teams (and so their bits).  The
// body then compiles as in the single-plan kernels: descriptor fields are
// loaded from the argument segment where they are used, while a persistent
// loop over work items keeps them live across the body and spills (RT2
// inlined in such a loop: 1040 bytes of spills against 276 here, 63 against
// 44 us per element and CU; RT3 called from it: 400 bytes and 177 against
// 156 us; RT1 10.7 against 9.7 us).
constexpr int kMultiProbs = 8;
template <class Args>
struct MultiT {
  Args p[kMultiProbs];
  int64_t start[kMultiProbs + 1];   // first workgroup of each problem; start[np] = grid
  int32_t np;
};
using MultiArgs = MultiT<SetupArgs>;
using MultiRecArgs = MultiT<RecoverArgs>;

// The problem of workgroup g (wave-uniform).
template <class Args>
__device__ __forceinline__ int multi_problem(const MultiT<Args>& m, int64_t g) {
  int pi = 0;
#pragma unroll
  for (int q = 1; q < kMultiProbs; ++q) pi += (q < m.np && g >= m.start[q]) ? 1 : 0;
  return __builtin_amdgcn_readfirstlane(pi);
}

// Setup teams (lanes per element) and elements per workgroup of order k:
// those of the single-plan kernels.
__host__ __device__ constexpr int setup_team(int k) { return k == 0 ? 16 : (k == 1 ? 64 : 512); }
__host__ __device__ constexpr int setup_teams(int k) { return k == 0 ? 16 : (k == 1 ? 4 : 1); }

template <int K>
__global__ __launch_bounds__(setup_team(K) * setup_teams(K), K == 2 ? 4 : (K == 3 ? 1 : 2)) void k_setup_multi(
    MultiArgs m) {
  extern __shared__ double smem[];
  const int64_t g = blockIdx.x;
  const int pi = multi_problem(m, g);
  const SetupArgs& a = m.p[pi];
  if constexpr (K <= 2) setup_generic_body<K, setup_team(K), setup_teams(K)>(a, smem, g - m.start[pi]);
  else setup_k3_body<kBatchThreadsK3>(a, smem, g - m.start[pi]);
}

template <int K>
__global__ __launch_bounds__(recover_team(K) * recover_teams(K)) void k_recover_multi(MultiRecArgs m) {
  extern __shared__ double smem[];
  const int64_t g = blockIdx.x;
  const int pi = multi_problem(m, g);
  recover_generic_body<K, recover_team(K), recover_teams(K)>(m.p[pi], smem, g - m.start[pi]);
}

// The mixed-precision problems: one persistent launch per phase walks a
// cost-sorted list of work items (problem, run of element blocks) taken from
// an atomic work queue, whatever their orders (the mixed element routines are
// called, each with its own register allocation).
__global__ __launch_bounds__(kBatchThreads) void k_setup_batch_mixed(const BatchProb* probs, const BatchItem* items,
                                                                     int64_t nitems, double* scratch,
                                                                     int32_t* queue) {
  extern __shared__ double smem[];
  __shared__ int64_t item;
  // workgroup b owns scratch slot b (k = 3; the grid has at most kMixedSlots workgroups)
  double* slot = scratch ? scratch + int64_t(blockIdx.x) * MixedLayout<3, 512, 1>::slot : nullptr;
  for (int64_t w = next_item(queue, &item); w < nitems; w = next_item(queue, &item)) {
    const BatchItem it = items[w];
    const BatchProb& P = probs[it.prob];
    for (int b = 0; b < it.nblk; ++b) {
      const int64_t blk = it.blk0 + b;
      switch (P.k) {
        case 0: batch_setup_mx<0, 64, 8>(P.s, smem, blk, P.sweeps, nullptr); break;
        case 1: batch_setup_mx<1, 128, 4>(P.s, smem, blk, P.sweeps, nullptr); break;
        case 2: batch_setup_mx<2, 512, 1>(P.s, smem, blk, P.sweeps, nullptr); break;
        default: batch_setup_mx<3, 512, 1>(P.s, smem, blk, P.sweeps, slot); break;
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kBatchThreads) void k_recover_batch_mixed(const BatchProb* probs,
                                                                       const BatchItem* items, int64_t nitems,
                                                                       int32_t* queue) {
  extern __shared__ double smem[];
  __shared__ int64_t item;
  for (int64_t w = next_item(queue, &item); w < nitems; w = next_item(queue, &item)) {
    const BatchItem it = items[w];
    const BatchProb& P = probs[it.prob];
    const RecoverArgs a = global_args(P.r);
    for (int b = 0; b < it.nblk; ++b) {
      const int64_t blk = it.blk0 + b;
      switch (P.k) {
        case 0: recover_mixed_body<0, 64, 8>(a, smem, blk); break;
        case 1: recover_mixed_body<1, 128, 4>(a, smem, blk); break;
        case 2: recover_mixed_body<2, 512, 1>(a, smem, blk); break;
        default: recover_mixed_body<3, 512, 1>(a, smem, blk); break;
      }
      __syncthreads();
    }
  }
}

// LDS bytes of one block of the batch kernels for order k.
inline size_t batch_setup_lds(int k) {
  switch (k) {
    case 0: return 8 * size_t(setup_teams(0)) * size_t(GenericLayout<0, setup_team(0), setup_teams(0)>::per);
    case 1: return 8 * size_t(setup_teams(1)) * size_t(GenericLayout<1, setup_team(1), setup_teams(1)>::per);
    case 2: return 8 * size_t(GenericLayout<2, setup_team(2), setup_teams(2)>::per);
    default: return 8 * size_t(K3Layout::per);
  }
}
inline size_t batch_recover_lds(int k) {
  switch (k) {
    case 0: return 8 * size_t(recover_teams(0)) * size_t(recover_per<0>());
    case 1: return 8 * size_t(recover_teams(1)) * size_t(recover_per<1>());
    case 2: return 8 * size_t(recover_teams(2)) * size_t(recover_per<2>());
    default: return 8 * size_t(recover_teams(3)) * size_t(recover_per<3>());
  }
}

inline size_t batch_setup_lds_mixed(int k) {
  switch (k) {
    case 0: return 8 * 8 * size_t(MixedLayout<0, 64, 8>::per);
    case 1: return 8 * 4 * size_t(MixedLayout<1, 128, 4>::per);
    case 2: return 8 * size_t(MixedLayout<2, 512, 1>::per);
    default: return 8 * size_t(MixedLayout<3, 512, 1>::per);
  }
}
inline size_t batch_recover_lds_mixed(int k) {
  switch (k) {
    case 0: return 8 * 8 * size_t(RT<0>::nb);
    case 1: return 8 * 4 * size_t(RT<1>::nb);
    case 2: return 8 * size_t(RT<2>::nb);
    default: return 8 * size_t(RT<3>::nb);
  }
}

}  // namespace hyb
