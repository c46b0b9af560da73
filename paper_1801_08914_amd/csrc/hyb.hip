// C ABI of the hybridization library: plan, bind, setup, rhs, solve,
// recover, status.  Kernels are in setup_generic.hpp and pcg.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/hyb.h"
#include "pcg.hpp"
#include "plan.hpp"
#include "k1_fast.hpp"
#include "setup_generic.hpp"
#include "mixed.hpp"
#include "setup_k3.hpp"
#include "batch.hpp"

#include <algorithm>

struct hyb_plan {
  hyb::Plan P;
};

namespace {

thread_local int64_t g_last_detail = -1;

inline hipStream_t stream_of(const hyb::Plan& P) { return reinterpret_cast<hipStream_t>(P.opts.stream); }

hyb::DeviceMaps device_maps(const hyb::Plan& P) {
  const auto* base = static_cast<const uint8_t*>(P.buf.maps);
  const auto& L = P.lay;
  hyb::DeviceMaps m;
  m.e2v = reinterpret_cast<const int32_t*>(base + L.e2v);
  m.xyz = reinterpret_cast<const double*>(base + L.xyz);
  m.elem_face = reinterpret_cast<const int32_t*>(base + L.elem_face);
  m.elem_pi = base + L.elem_pi;
  m.elem_slot = base + L.elem_slot;
  m.face_rowbase = reinterpret_cast<const int64_t*>(base + L.face_rowbase);
  m.face_nslots = reinterpret_cast<const int32_t*>(base + L.face_nslots);
  m.tab_s = reinterpret_cast<const double*>(base + L.tab_s);
  m.tab_d = reinterpret_cast<const double*>(base + L.tab_d);
  m.tab_w = reinterpret_cast<const double*>(base + L.tab_w);
  m.tab_ref = reinterpret_cast<const double*>(base + L.tab_ref);
  m.gauss_x = reinterpret_cast<const double*>(base + L.tab_x);
  m.tab1d = reinterpret_cast<const double*>(base + L.tab_1d);
  m.face_selfslot = reinterpret_cast<const int32_t*>(base + L.face_selfslot);
  m.face_owner = reinterpret_cast<const int32_t*>(base + L.face_owner);
  m.k1_geo = reinterpret_cast<const double*>(base + L.k1_geo);
  m.k1_meta = base + L.k1_meta;
  m.face_w = reinterpret_cast<const double*>(base + L.face_w);
  return m;
}

int hip_fail(hipError_t err) {
  g_last_detail = int64_t(err);
  return HYB_E_HIP;
}

#define HYB_HIP(call)                              \
  do {                                             \
    hipError_t err_ = (call);                      \
    if (err_ != hipSuccess) return hip_fail(err_); \
  } while (0)

int fill(hipStream_t s, double* x, int64_t n, double v) {
  if (n <= 0) return HYB_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(hyb::k_fill, dim3(unsigned(blocks)), dim3(256), 0, s, x, n, v);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

template <int K, int TEAM, int EPB>
int launch_setup(const hyb::SetupArgs& a, hipStream_t s) {
  if (a.ne == 0) return HYB_OK;
  const int64_t blocks = (a.ne + EPB - 1) / EPB;
  hipLaunchKernelGGL((hyb::k_setup_generic<K, TEAM, EPB>), dim3(unsigned(blocks)), dim3(TEAM * EPB), 0, s, a);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

template <int K, int TEAM, int EPB>
int launch_recover(const hyb::RecoverArgs& a, hipStream_t s) {
  if (a.ne == 0) return HYB_OK;
  const int64_t blocks = (a.ne + EPB - 1) / EPB;
  hipLaunchKernelGGL((hyb::k_recover_generic<K, TEAM, EPB>), dim3(unsigned(blocks)), dim3(TEAM * EPB), 0, s, a);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

int dispatch_setup(int k, const hyb::SetupArgs& a, hipStream_t s) {
  switch (k) {
    case 0: return launch_setup<0, 16, 16>(a, s);
    case 1: return launch_setup<1, 64, 4>(a, s);
    case 2: return launch_setup<2, 512, 1>(a, s);
    case 3:
      if (a.ne > 0) {
        hipLaunchKernelGGL(hyb::k_setup_k3<512>, dim3(unsigned(a.ne)), dim3(512), 0, s, a);
        HYB_HIP(hipGetLastError());
      }
      return HYB_OK;
    default: return HYB_E_ARG;
  }
}

int dispatch_recover(int k, const hyb::RecoverArgs& a, hipStream_t s) {
  switch (k) {
    case 0: return launch_recover<0, 16, 16>(a, s);
    case 1: return launch_recover<1, 64, 4>(a, s);
    case 2: return launch_recover<2, hyb::recover_team(2), 1>(a, s);
    case 3: return launch_recover<3, hyb::recover_team(3), hyb::recover_teams(3)>(a, s);
    default: return HYB_E_ARG;
  }
}

int64_t mixed_record_len(int k) {
  switch (k) {
    case 0: return hyb::MixedRec<0>::len;
    case 1: return hyb::MixedRec<1>::len;
    case 2: return hyb::MixedRec<2>::len;
    default: return hyb::MixedRec<3>::len;
  }
}

template <int K, int TEAM, int EPB>
int launch_setup_mixed(const hyb::SetupArgs& a, int sweeps, hipStream_t s) {
  if (a.ne == 0) return HYB_OK;
  const int64_t blocks = (a.ne + EPB - 1) / EPB;
  hipLaunchKernelGGL((hyb::k_setup_mixed<K, TEAM, EPB>), dim3(unsigned(blocks)), dim3(TEAM * EPB), 0, s, a, sweeps);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

// k = 3: a persistent grid of at most kMixedSlots workgroups, each with its
// scratch slot (FP64 element matrix, FP32 work columns) in the work buffer.
int launch_setup_mixed3(const hyb::SetupArgs& a, int sweeps, double* scratch, hipStream_t s) {
  if (a.ne == 0) return HYB_OK;
  const int64_t grid = std::min<int64_t>(a.ne, hyb::kMixedSlots);
  hipLaunchKernelGGL((hyb::k_setup_mixed_slots<3, 512>), dim3(unsigned(grid)), dim3(512), 0, s, a, sweeps, scratch);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

// Bytes of the k = 3 mixed scratch slots.
int64_t mixed_scratch_bytes(int k) {
  return k == 3 ? int64_t(8) * hyb::kMixedSlots * hyb::MixedLayout<3, 512, 1>::slot : 0;
}

template <int K, int TEAM, int EPB>
int launch_recover_mixed(const hyb::RecoverArgs& a, hipStream_t s) {
  if (a.ne == 0) return HYB_OK;
  const int64_t blocks = (a.ne + EPB - 1) / EPB;
  hipLaunchKernelGGL((hyb::k_recover_mixed<K, TEAM, EPB>), dim3(unsigned(blocks)), dim3(TEAM * EPB), 0, s, a);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

int dispatch_setup_mixed(int k, const hyb::SetupArgs& a, int sweeps, double* scratch, hipStream_t s) {
  // the count of elements solved in FP64 restarts with every call
  hipLaunchKernelGGL(hyb::k_fill_i32, dim3(1), dim3(64), 0, s, a.status + 2, int64_t(1), 0);
  HYB_HIP(hipGetLastError());
  switch (k) {
    case 0: return launch_setup_mixed<0, 64, 4>(a, sweeps, s);
    case 1: return launch_setup_mixed<1, 128, 2>(a, sweeps, s);
    case 2: return launch_setup_mixed<2, 512, 1>(a, sweeps, s);
    case 3: return launch_setup_mixed3(a, sweeps, scratch, s);
    default: return HYB_E_ARG;
  }
}

int dispatch_recover_mixed(int k, const hyb::RecoverArgs& a, hipStream_t s) {
  switch (k) {
    case 0: return launch_recover_mixed<0, 16, 16>(a, s);
    case 1: return launch_recover_mixed<1, 64, 4>(a, s);
    case 2: return launch_recover_mixed<2, 128, 1>(a, s);
    case 3: return launch_recover_mixed<3, 256, 1>(a, s);
    default: return HYB_E_ARG;
  }
}

hipEvent_t take_event(hyb::Plan& P) {
  if (!P.ev_pool.empty()) {
    void* e = P.ev_pool.back();
    P.ev_pool.pop_back();
    return reinterpret_cast<hipEvent_t>(e);
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Record an event on the plan's stream into list (start or stop of a pair).
void mark(hyb::Plan& P, std::vector<void*>& list) {
  if (!P.timing) return;
  hipEvent_t e = take_event(P);
  if (!e) return;
  (void)hipEventRecord(e, stream_of(P));
  list.push_back(e);
}

int zero_diag(const hyb::Plan& P, hipStream_t s) {
  const int64_t tot = P.nfaces * P.ord.K2 * P.ord.K2;
  if (tot == 0) return HYB_OK;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  const hyb::DeviceMaps m = device_maps(P);
  hipLaunchKernelGGL(hyb::k_zero_diag_blocks, dim3(unsigned(blocks)), dim3(256), 0, s, P.nfaces, P.ord.K2,
                     m.face_rowbase, m.face_nslots, m.face_selfslot, P.buf.val);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

hyb::k1::SimtArgs simt_args(const hyb::Plan& P) {
  hyb::k1::SimtArgs a{};
  a.mp = device_maps(P);
  a.ne = P.ne;
  a.alpha = P.alpha_d;
  a.beta = P.beta_d;
  a.factor = P.buf.factor;
  a.y = P.buf.y;
  a.r = P.buf.r;
  a.side = P.buf.work;
  a.nfaces = P.nfaces;
  return a;
}

// Add the neighbour terms of the same-face blocks of H and of r.
int finalize_k1(const hyb::Plan& P, hipStream_t s, bool matrix, bool rhs) {
  const int64_t tot = (matrix || rhs) ? P.nfaces * 4 : 0;
  if (tot == 0) return HYB_OK;
  const hyb::DeviceMaps m = device_maps(P);
  hyb::k1::FinalArgs f{};
  f.nfaces = P.nfaces;
  f.rowbase = m.face_rowbase;
  f.nslots = m.face_nslots;
  f.selfslot = m.face_selfslot;
  f.Hval = matrix ? P.buf.val : nullptr;
  f.r = rhs ? P.buf.r : nullptr;
  f.side = P.buf.work;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(hyb::k1::k_finalize_k1, dim3(unsigned(blocks)), dim3(256), 0, s, f);
  HYB_HIP(hipGetLastError());
  return HYB_OK;
}

// PCG vectors and partial sums; the RT_1 setup also uses the buffer for the
// neighbour terms of the same-face blocks of H and of r (20 per face).
// PCG work: r, z, p (two buffers), q, dinv; SpMV partials (1 per block),
// update partials (2 per block, two slots), scalars.
int64_t work_bytes(int64_t m, int nblk, int nblk_spmv, int64_t nfaces) {
  const int64_t pcg = 8 * (6 * m + int64_t(nblk_spmv) + 4 * int64_t(nblk)) + 512;
  const int64_t side = 8 * 20 * nfaces;
  return pcg > side ? pcg : side;
}

}  // namespace

extern "C" {

int64_t hyb_last_detail(void) { return g_last_detail; }

const char* hyb_strerror(int code) {
  switch (code) {
    case HYB_OK: return "ok";
    case HYB_E_ARG: return "invalid argument";
    case HYB_E_MESH: return "invalid mesh connectivity";
    case HYB_E_JACOBIAN: return "non-positive Jacobian determinant";
    case HYB_E_NOT_SPD: return "element matrix not positive definite";
    case HYB_E_STATE: return "call out of order";
    case HYB_E_NOMEM: return "missing device buffer";
    case HYB_E_NOCONV: return "PCG did not converge";
    case HYB_E_HIP: return "HIP runtime error";
    case HYB_E_INTERNAL: return "internal invariant broken";
    case HYB_E_REFINE: return "mixed-precision refinement did not converge";
    default: return "unknown status";
  }
}

int hyb_plan_create(const hyb_mesh* mesh, int k, const hyb_opts* opt, hyb_plan_t** out, hyb_sizes* sizes) {
  g_last_detail = -1;
  if (!out) return HYB_E_ARG;
  *out = nullptr;
  if (opt && ((opt->precision != HYB_FP64 && opt->precision != HYB_MIXED) || opt->pcg_reduce < 0 ||
              opt->pcg_reduce > 2 || opt->refine_sweeps > 16 ||
              (opt->system != HYB_HYBRID && opt->system != HYB_STATIC) ||
              (opt->system == HYB_STATIC && opt->precision != HYB_FP64) ||
              (opt->weighted_c && opt->system == HYB_STATIC) ||
              (opt->quad_q != 0 && opt->quad_q != k + 2)))
    return HYB_E_ARG;
  hyb_plan* p = new (std::nothrow) hyb_plan;
  if (!p) return HYB_E_NOMEM;
  int64_t detail = -1;
  int rc = hyb::build_plan(mesh, k, p->P, detail);
  if (rc != HYB_OK) {
    g_last_detail = detail;
    delete p;
    return rc;
  }
  if (opt) p->P.opts = *opt;
  hyb::Plan& P = p->P;
  P.mixed = P.opts.precision == HYB_MIXED;
  P.stat = P.opts.system == HYB_STATIC;
  P.sweeps = P.opts.refine_sweeps < 0 ? -1 : P.opts.refine_sweeps;
  if (P.stat && P.has_natural) {
    // static condensation keeps one global dof per face dof and numbers them
    // like the multipliers, which natural boundary faces do not have
    delete p;
    return HYB_E_ARG;
  }
  P.fast_k1 = k == 1 && P.all_affine && P.opts.kernel_variant == 0 && !P.mixed && !P.stat && !P.opts.weighted_c &&
              !P.has_natural;
  if (P.opts.weighted_c) {
    // M_s of the weighted constraint: the face dofs' tangential nodes are the
    // k+1 Gauss-Legendre points, so the face mass matrix of their Lagrange
    // basis is diagonal, w_a0 w_a1 at position a0 + (k+1) a1
    std::vector<double> x, w;
    hyb::gauss_legendre_01(k + 1, x, w);
    for (int a1 = 0; a1 <= k; ++a1)
      for (int a0 = 0; a0 <= k; ++a0) P.face_w[size_t(a0 + (k + 1) * a1)] = w[size_t(a0)] * w[size_t(a1)];
  }
  if (P.fast_k1) P.factor_len = hyb::k1::REC;
  if (P.mixed) P.factor_len = mixed_record_len(k);
  // PCG grids, multiples of the 8 XCDs: vector kernels about one row per
  // thread, the SpMV two rows per lane group
  auto grid_for = [](int64_t rows, int64_t per, int64_t cap) {
    int64_t n = (rows + per - 1) / per;
    n = (n + 7) / 8 * 8;
    return int(n < 8 ? 8 : (n > cap ? cap : n));
  };
  const int64_t K2 = int64_t(k + 1) * (k + 1);
  P.max_row = 0;
  for (int64_t i = 0; i < P.m; ++i) P.max_row = std::max(P.max_row, P.row_ptr[i + 1] - P.row_ptr[i]);
  // the face-panel SpMV relies on the pattern built by the plan: the K2 rows
  // of a face have equal length, the same columns, and follow each other
  bool panels = P.m % K2 == 0;
  for (int64_t F = 0; panels && F < P.m / K2; ++F) {
    const int64_t b = P.row_ptr[F * K2], w = P.row_ptr[F * K2 + 1] - b;
    for (int64_t a = 1; panels && a < K2; ++a) {
      panels = P.row_ptr[F * K2 + a] == b + a * w && P.row_ptr[F * K2 + a + 1] == b + (a + 1) * w;
      for (int64_t c = 0; panels && c < w; ++c) panels = P.col[b + a * w + c] == P.col[b + c];
    }
  }
  if (!panels) {
    g_last_detail = 0;
    delete p;
    return HYB_E_INTERNAL;
  }
  P.work_blocks = grid_for(P.m, hyb::kPcgThreads, 16384);
  P.spmv_blocks = grid_for(P.m / K2, hyb::spmv_shape(k).faces_per_block, 65536);
  if (sizes) {
    sizes->ne = P.ne;
    sizes->k = k;
    sizes->n_local = P.ord.n;
    sizes->n_interior = P.ord.ni;
    sizes->n_face_dofs = P.ord.K2;
    sizes->n_faces = P.nfaces;
    sizes->n_boundary_faces = P.nbfaces;
    sizes->m = P.m;
    sizes->nnz = P.nnz;
    sizes->factor_len = P.factor_len;
    sizes->bytes_maps = int64_t(P.lay.total);
    sizes->bytes_factor = 8 * P.ne * P.factor_len;
    sizes->bytes_y = 8 * P.ne * P.ord.n;
    sizes->bytes_work = std::max(work_bytes(P.m, P.work_blocks, P.spmv_blocks, P.nfaces),
                                 P.mixed ? mixed_scratch_bytes(k) : int64_t(0));
  }
  *out = p;
  return HYB_OK;
}

int hyb_plan_topology(const hyb_plan_t* plan, int32_t* elem_face, uint8_t* elem_pi, int32_t* face_owner,
                      int32_t* face_nbr, int64_t* row_ptr, int32_t* col) {
  if (!plan) return HYB_E_ARG;
  const hyb::Plan& P = plan->P;
  if (elem_face) std::memcpy(elem_face, P.elem_face.data(), sizeof(int32_t) * P.elem_face.size());
  if (elem_pi)
    for (int64_t e = 0; e < P.ne; ++e)
      for (int f = 0; f < 6; ++f) elem_pi[6 * e + f] = P.elem_pi[size_t(8 * e + f)];
  if (face_owner) std::memcpy(face_owner, P.face_owner.data(), sizeof(int32_t) * P.face_owner.size());
  if (face_nbr) std::memcpy(face_nbr, P.face_nbr.data(), sizeof(int32_t) * P.face_nbr.size());
  if (row_ptr) std::memcpy(row_ptr, P.row_ptr.data(), sizeof(int64_t) * P.row_ptr.size());
  if (col) std::memcpy(col, P.col.data(), sizeof(int32_t) * P.col.size());
  return HYB_OK;
}

int hyb_bind(hyb_plan_t* plan, const hyb_buffers* buf) {
  if (!plan || !buf) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  if (!buf->maps || !buf->factor || !buf->y || !buf->val || !buf->r || !buf->work || !buf->status ||
      (P.m > 0 && (!buf->row_ptr || !buf->col)))
    return HYB_E_NOMEM;
  P.buf = *buf;
  hipStream_t s = stream_of(P);
  std::vector<uint8_t> host(P.lay.total, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(host.data() + off, src, bytes);
  };
  const auto& L = P.lay;
  put(L.e2v, P.e2v.data(), 4 * P.e2v.size());
  put(L.xyz, P.xyz.data(), 8 * P.xyz.size());
  put(L.elem_face, P.elem_face.data(), 4 * P.elem_face.size());
  put(L.elem_pi, P.elem_pi.data(), P.elem_pi.size());
  put(L.elem_slot, P.elem_slot.data(), P.elem_slot.size());
  put(L.face_rowbase, P.face_rowbase.data(), 8 * P.face_rowbase.size());
  put(L.face_nslots, P.face_nslots.data(), 4 * P.face_nslots.size());
  put(L.tab_s, P.tab_s.data(), 8 * P.tab_s.size());
  put(L.tab_d, P.tab_d.data(), 8 * P.tab_d.size());
  put(L.tab_w, P.tab_w.data(), 8 * P.tab_w.size());
  put(L.tab_ref, P.tab_ref.data(), 8 * P.tab_ref.size());
  put(L.tab_x, P.tab_x.data(), 8 * P.tab_x.size());
  put(L.tab_1d, P.tab_1d.data(), 8 * P.tab_1d.size());
  put(L.face_selfslot, P.face_selfslot.data(), 4 * P.face_selfslot.size());
  {
    std::vector<int32_t> owner_elem(size_t(P.nfaces));
    for (int64_t F = 0; F < P.nfaces; ++F) owner_elem[size_t(F)] = P.face_owner[size_t(2 * F)];
    put(L.face_owner, owner_elem.data(), 4 * owner_elem.size());
  }
  put(L.k1_geo, P.k1_geo.data(), 8 * P.k1_geo.size());
  put(L.k1_meta, P.k1_meta.data(), P.k1_meta.size());
  put(L.face_w, P.face_w.data(), 8 * P.face_w.size());
  HYB_HIP(hipMemcpyAsync(buf->maps, host.data(), host.size(), hipMemcpyHostToDevice, s));
  if (P.m > 0) {
    HYB_HIP(hipMemcpyAsync(buf->row_ptr, P.row_ptr.data(), 8 * P.row_ptr.size(), hipMemcpyHostToDevice, s));
    HYB_HIP(hipMemcpyAsync(buf->col, P.col.data(), 4 * P.col.size(), hipMemcpyHostToDevice, s));
  }
  hipLaunchKernelGGL(hyb::k_fill_i32, dim3(1), dim3(64), 0, s, buf->status, int64_t(4), 0);
  HYB_HIP(hipGetLastError());
  HYB_HIP(hipStreamSynchronize(s));  // host staging goes out of scope
  P.bound = true;
  P.have_setup = P.have_rhs = false;
  return HYB_OK;
}

int hyb_setup(hyb_plan_t* plan, const double* alpha, const double* beta, const double* f, const double* g) {
  if (!plan || !alpha || !beta) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  if (!P.bound) return HYB_E_STATE;
  hipStream_t s = stream_of(P);
  hyb::SetupArgs a{};
  a.mp = device_maps(P);
  a.ne = P.ne;
  a.alpha = alpha;
  a.beta = beta;
  a.f = f;
  a.g = f ? g : nullptr;
  a.factor = P.buf.factor;
  a.y = P.buf.y;
  a.Hval = P.buf.val;
  a.r = P.buf.r;
  a.status = P.buf.status;
  a.mode = hyb::MODE_MATRIX | (f ? hyb::MODE_RHS : 0);
  a.stat = P.stat ? 1 : 0;
  mark(P, P.ev_setup);
  int rc = HYB_OK;
  if (P.fast_k1) {
    if (P.ne > 0) {
      constexpr int per_block = hyb::k1::SETUP_EPW * hyb::k1::SETUP_WAVES;
      const unsigned blocks = unsigned((P.ne + per_block - 1) / per_block);
      hipLaunchKernelGGL(hyb::k1::k_setup_k1, dim3(blocks), dim3(64 * hyb::k1::SETUP_WAVES), 0, s, a, P.buf.work,
                         P.nfaces);
      HYB_HIP(hipGetLastError());
      rc = finalize_k1(P, s, true, f != nullptr);
    }
  } else {
    rc = zero_diag(P, s);
    if (!rc && f) rc = fill(s, P.buf.r, P.m, 0.0);
    if (!rc) rc = P.mixed ? dispatch_setup_mixed(P.ord.k, a, P.sweeps, P.buf.work, s) : dispatch_setup(P.ord.k, a, s);
  }
  mark(P, P.ev_setup);
  if (rc) return rc;
  P.have_setup = true;
  P.have_rhs = f != nullptr;
  P.alpha_d = alpha;
  P.beta_d = beta;
  return HYB_OK;
}

int hyb_rhs(hyb_plan_t* plan, const double* f, const double* g) {
  if (!plan || !f) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  if (!P.have_setup) return HYB_E_STATE;
  hipStream_t s = stream_of(P);
  int rc = HYB_OK;
  if (P.fast_k1) {
    hyb::k1::SimtArgs b = simt_args(P);
    b.f = f;
    b.g = g;
    if (P.ne > 0) {
      const unsigned blocks = unsigned((P.ne + hyb::k1::SOLVE_EPW - 1) / hyb::k1::SOLVE_EPW);
      hipLaunchKernelGGL(hyb::k1::k_rhs_k1, dim3(blocks), dim3(64), 0, s, b);
      HYB_HIP(hipGetLastError());
      rc = finalize_k1(P, s, false, true);
    }
  } else {
    rc = fill(s, P.buf.r, P.m, 0.0);
    if (rc) return rc;
    hyb::SetupArgs a{};
    a.mp = device_maps(P);
    a.ne = P.ne;
    // the boundary correction -M_re g_e reassembles M_T from setup's coefficients
    a.alpha = P.alpha_d;
    a.beta = P.beta_d;
    a.f = f;
    a.g = g;
    a.factor = P.buf.factor;
    a.y = P.buf.y;
    a.Hval = P.buf.val;
    a.r = P.buf.r;
    a.status = P.buf.status;
    a.mode = hyb::MODE_RHS;
    a.stat = P.stat ? 1 : 0;
    rc = P.mixed ? dispatch_setup_mixed(P.ord.k, a, P.sweeps, P.buf.work, s) : dispatch_setup(P.ord.k, a, s);
  }
  if (rc) return rc;
  P.have_rhs = true;
  return HYB_OK;
}

}  // extern "C"

namespace {

// Bytes of PCG work (vectors, partial sums, the scalars) of a plan.
size_t pcg_work_bytes(const hyb::Plan& P) {
  return ((8 * (6 * size_t(P.m) + P.spmv_blocks + 4 * size_t(P.work_blocks)) + 63) & ~size_t(63)) +
         sizeof(hyb::PcgScalars);
}

// The Jacobi-PCG of hyb_pcg with its work vectors at w.
int pcg_run(hyb::Plan& P, double rtol, int maxit, double* lambda, hyb_solve_info* info, double* w) {
  hipStream_t s = stream_of(P);
  const int64_t m = P.m;
  const int nblk = P.work_blocks, nspmv = P.spmv_blocks;
  double* r = w;
  double* z = r + m;
  double* pb[2] = {z + m, z + 2 * m};
  double* q = z + 3 * m;
  double* dinv = q + m;
  double* part_s = dinv + m;           // SpMV partials
  double* part_u = part_s + nspmv;     // update partials, two slots
  auto* sc = reinterpret_cast<hyb::PcgScalars*>(
      reinterpret_cast<uint8_t*>(w) + ((8 * (6 * size_t(m) + nspmv + 4 * size_t(nblk)) + 63) & ~size_t(63)));
  if (info) *info = hyb_solve_info{0, 0, 0.0};
  if (m == 0) {
    if (info) info->converged = 1;
    return HYB_OK;
  }
  const int k = P.ord.k;
  const int64_t nfb = m / ((k + 1) * (k + 1));   // faces with multipliers
  const dim3 grid{unsigned(nblk), 1, 1}, grid_s{unsigned(nspmv), 1, 1};
  const dim3 blk{unsigned(hyb::kPcgThreads), 1, 1};
  // lanes per row of the diagonal search; panel shapes (K2, lanes, columns
  // per lane) cover the widest panels, 11 faces: 11, 44, 99, 176 columns
  auto init = P.max_row <= 16 ? hyb::k_pcg_init<4> : P.max_row <= 48 ? hyb::k_pcg_init<8>
            : P.max_row <= 112 ? hyb::k_pcg_init<16> : hyb::k_pcg_init<32>;
  // partial sums in the consuming kernels unless every block reading every
  // partial would move more than about 8 MB through L2 per iteration
  const double sum_bytes = 8.0 * (double(nspmv) * nblk + 2.0 * double(nblk) * nspmv);
  const bool fused = P.opts.pcg_reduce == 1 || (P.opts.pcg_reduce == 0 && sum_bytes <= 8.0 * (1 << 20));
  auto spmv = fused ? (k == 0 ? hyb::k_pcg_spmv<1, 4, 3, true> : k == 1 ? hyb::k_pcg_spmv<4, 16, 3, true>
                       : k == 2 ? hyb::k_pcg_spmv<9, 32, 4, true> : hyb::k_pcg_spmv<16, 64, 3, true>)
                    : (k == 0 ? hyb::k_pcg_spmv<1, 4, 3, false> : k == 1 ? hyb::k_pcg_spmv<4, 16, 3, false>
                       : k == 2 ? hyb::k_pcg_spmv<9, 32, 4, false> : hyb::k_pcg_spmv<16, 64, 3, false>);
  auto update = fused ? hyb::k_pcg_update<true> : hyb::k_pcg_update<false>;
  hipLaunchKernelGGL(init, grid, blk, 0, s, m, P.buf.row_ptr, P.buf.col, P.buf.val, P.buf.r, lambda, r, z, pb[0],
                     dinv, part_u, nblk);
  hipLaunchKernelGGL(hyb::k_pcg_rr, dim3(1), blk, 0, s, part_u, nblk, 1, sc, 1);
  HYB_HIP(hipGetLastError());
  hyb::PcgScalars hs{};
  HYB_HIP(hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
  HYB_HIP(hipStreamSynchronize(s));
  const double rr0 = hs.rr0;
  const double tol2 = rtol * rtol * rr0;
  int it = 0;
  bool conv = rr0 <= tol2 || rr0 == 0.0;
  double rr = rr0;
  const int check = 8;
  while (!conv && it < maxit) {
    const int batch = (maxit - it) < check ? (maxit - it) : check;
    for (int b = 0; b < batch; ++b) {
      // iteration j: p_{j-1} = pb[j & 1], p_j into the other buffer
      const int j = it + b;
      const double* pp = pb[j & 1];
      double* pn = pb[(j + 1) & 1];
      if (!fused && j > 0)
        hipLaunchKernelGGL(hyb::k_pcg_scalar, dim3(1), blk, 0, s, part_s, nspmv, part_u, nblk, sc, j - 1, 1);
      hipLaunchKernelGGL(spmv, grid_s, blk, 0, s, nfb, P.buf.row_ptr, P.buf.col, P.buf.val, z, pp, pn, q, part_u,
                         nblk, sc, j, part_s, nspmv);
      if (!fused) hipLaunchKernelGGL(hyb::k_pcg_scalar, dim3(1), blk, 0, s, part_s, nspmv, part_u, nblk, sc, j, 0);
      hipLaunchKernelGGL(update, grid, blk, 0, s, m, pn, q, dinv, lambda, r, z, part_s, nspmv, part_u, sc, j, nblk);
    }
    it += batch;
    hipLaunchKernelGGL(hyb::k_pcg_rr, dim3(1), blk, 0, s, part_u, nblk, (it - 1) & 1, sc, 0);
    HYB_HIP(hipGetLastError());
    HYB_HIP(hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
    HYB_HIP(hipStreamSynchronize(s));
    rr = hs.rr;
    conv = rr <= tol2;
  }
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->rel_res = rr0 > 0.0 ? std::sqrt(rr / rr0) : 0.0;
  }
  return conv ? HYB_OK : HYB_E_NOCONV;
}

}  // namespace

extern "C" {

int hyb_pcg(hyb_plan_t* plan, double rtol, int maxit, double* lambda, hyb_solve_info* info) {
  if (!plan || !lambda || maxit < 0) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  if (!P.have_rhs) return HYB_E_STATE;
  return pcg_run(P, rtol, maxit, lambda, info, P.buf.work);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// hyb_pcg_noalloc: the same PCG with its work vectors, partial sums and
// scalars in a file-scope device array instead of the bound work buffer.
// Host code never passes the array's name to a kernel (that is a host-side
// stand-in): each device's address comes from hipGetSymbolAddress, taken
// once per device with that device current.
namespace {
constexpr size_t kNoAllocBytes = size_t(48) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(double** out) {
  int dev = 0;
  HYB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HYB_E_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HYB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HYB_E_INTERNAL;
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return HYB_OK;
}
}  // namespace

extern "C" {

int hyb_pcg_noalloc(hyb_plan_t* plan, double rtol, int maxit, double* lambda, hyb_solve_info* info) {
  if (!plan || !lambda || maxit < 0) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  const size_t need = pcg_work_bytes(P);
  if (need > kNoAllocBytes) {
    g_last_detail = int64_t(need);
    return HYB_E_ARG;
  }
  if (!P.have_rhs) return HYB_E_STATE;
  double* w = nullptr;
  const int rc = scratch_of_current_device(&w);
  if (rc) return rc;
  return pcg_run(P, rtol, maxit, lambda, info, w);
}

int hyb_recover(hyb_plan_t* plan, const double* lambda, double* u) {
  if (!plan || !lambda || !u) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  if (!P.have_rhs) return HYB_E_STATE;
  hyb::RecoverArgs a{};
  a.mp = device_maps(P);
  a.ne = P.ne;
  a.factor = P.buf.factor;
  a.y = P.buf.y;
  a.lambda = lambda;
  a.u = u;
  a.stat = P.stat ? 1 : 0;
  mark(P, P.ev_recover);
  int rc = HYB_OK;
  if (P.fast_k1) {
    hyb::k1::SimtArgs b = simt_args(P);
    b.lambda = lambda;
    b.u = u;
    if (P.ne > 0) {
      hipLaunchKernelGGL(hyb::k1::k_recover_k1, dim3(unsigned((P.ne + hyb::k1::SOLVE_EPW - 1) / hyb::k1::SOLVE_EPW)), dim3(64), 0, stream_of(P), b);
      HYB_HIP(hipGetLastError());
    }
  } else {
    rc = P.mixed ? dispatch_recover_mixed(P.ord.k, a, stream_of(P)) : dispatch_recover(P.ord.k, a, stream_of(P));
  }
  mark(P, P.ev_recover);
  return rc;
}

int hyb_solve(hyb_plan_t* plan, const double* f, const double* g, double rtol, int maxit, double* lambda,
              double* u, hyb_solve_info* info) {
  if (!plan || !f || !lambda || !u || maxit < 0) return HYB_E_ARG;
  if (!plan->P.have_setup) return HYB_E_STATE;
  int rc = hyb_rhs(plan, f, g);
  if (rc) return rc;
  const int rc_pcg = hyb_pcg(plan, rtol, maxit, lambda, info);
  if (rc_pcg != HYB_OK && rc_pcg != HYB_E_NOCONV) return rc_pcg;
  rc = hyb_recover(plan, lambda, u);
  return rc ? rc : rc_pcg;
}

int hyb_fallback_count(hyb_plan_t* plan, int64_t* count) {
  if (!plan || !count) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  if (!P.bound) return HYB_E_STATE;
  hipStream_t s = stream_of(P);
  int32_t st[4] = {0, 0, 0, 0};
  HYB_HIP(hipMemcpyAsync(st, P.buf.status, sizeof(st), hipMemcpyDeviceToHost, s));
  HYB_HIP(hipStreamSynchronize(s));
  *count = P.mixed ? int64_t(st[2]) : 0;
  return HYB_OK;
}

int hyb_get_csr(const hyb_plan_t* plan, const int64_t** row_ptr, const int32_t** col, const double** val,
                int64_t* m, int64_t* nnz) {
  if (!plan) return HYB_E_ARG;
  const hyb::Plan& P = plan->P;
  if (!P.bound) return HYB_E_STATE;
  if (row_ptr) *row_ptr = P.buf.row_ptr;
  if (col) *col = P.buf.col;
  if (val) *val = P.buf.val;
  if (m) *m = P.m;
  if (nnz) *nnz = P.nnz;
  return HYB_OK;
}

int hyb_timing_enable(hyb_plan_t* plan, int on) {
  if (!plan) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  for (void* e : P.ev_setup) P.ev_pool.push_back(e);
  for (void* e : P.ev_recover) P.ev_pool.push_back(e);
  P.ev_setup.clear();
  P.ev_recover.clear();
  P.timing = on != 0;
  return HYB_OK;
}

int hyb_timing_read(hyb_plan_t* plan, double* ms_setup, int* n_setup, double* ms_recover, int* n_recover) {
  if (!plan) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  HYB_HIP(hipStreamSynchronize(stream_of(P)));
  auto sum = [&](std::vector<void*>& L, double* ms, int* cnt) -> int {
    double tot = 0.0;
    int c = 0;
    for (size_t i = 0; i + 1 < L.size(); i += 2) {
      float t = 0.0f;
      hipError_t err = hipEventElapsedTime(&t, reinterpret_cast<hipEvent_t>(L[i]), reinterpret_cast<hipEvent_t>(L[i + 1]));
      if (err != hipSuccess) return hip_fail(err);
      tot += t;
      ++c;
    }
    for (void* e : L) P.ev_pool.push_back(e);
    L.clear();
    if (ms) *ms = tot;
    if (cnt) *cnt = c;
    return HYB_OK;
  };
  int rc = sum(P.ev_setup, ms_setup, n_setup);
  if (rc) return rc;
  return sum(P.ev_recover, ms_recover, n_recover);
}

int hyb_set_stream(hyb_plan_t* plan, void* stream) {
  if (!plan) return HYB_E_ARG;
  plan->P.opts.stream = stream;
  return HYB_OK;
}

int hyb_status(hyb_plan_t* plan, int64_t* detail) {
  if (!plan) return HYB_E_ARG;
  hyb::Plan& P = plan->P;
  if (!P.bound) return HYB_E_STATE;
  hipStream_t s = stream_of(P);
  int32_t st[4] = {0, 0, 0, 0};
  HYB_HIP(hipMemcpyAsync(st, P.buf.status, sizeof(st), hipMemcpyDeviceToHost, s));
  HYB_HIP(hipStreamSynchronize(s));
  if (detail) *detail = st[0] ? int64_t(st[1]) : -1;
  return st[0];
}

void hyb_destroy(hyb_plan_t* plan) {
  if (!plan) return;
  hyb::Plan& P = plan->P;
  for (auto* L : {&P.ev_setup, &P.ev_recover, &P.ev_pool})
    for (void* e : *L) (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(e));
  delete plan;
}

// ---------------------------------------------------------------------------
// Batches: many independent plans, one persistent launch per phase.

}  // extern "C"

struct hyb_batch {
  std::vector<hyb_plan_t*> plans;
  hipStream_t stream = nullptr;
  int cus = 0;
  hyb_batch_tiles tiles{0, 0};
  std::vector<hyb::BatchProb> probs;       // host copy of the descriptors
  std::vector<hyb::BatchItem> items;       // cost-sorted work list of the mixed problems
  size_t n_mx = 0;                         // its length
  hyb::BatchProb* d_probs = nullptr;
  hyb::BatchItem* d_items = nullptr;
  size_t cap_items = 0;
  size_t lds_setup_mx = 0, lds_recover_mx = 0;
  bool dirty = true;                       // descriptors or items changed since upload
  bool use_graph = false;
  hipGraphExec_t g_setup = nullptr, g_recover = nullptr;
  hipStream_t gstream = nullptr;           // capture/replay stream (graphs need a non-null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  double* scratch = nullptr;               // k = 3 mixed: a slot per workgroup of the mixed launch
  int32_t* d_queue = nullptr;              // work-queue counters of the mixed launches (kQueues)
  // optional HIP-event timing of each phase (start/stop pairs, launch order)
  bool timing = false;
  std::vector<hipEvent_t> ev_setup, ev_recover, ev_pool;
};

namespace {

// queue counters: mixed setup, mixed recovery
constexpr int kQueues = 2;
// the multi-problem descriptors travel as kernel arguments (at most 4 KB)
static_assert(sizeof(hyb::MultiArgs) <= 4096 && sizeof(hyb::MultiRecArgs) <= 4096, "kernel-argument size");

int batch_epb_of(const hyb::Plan& P) { return hyb::batch_epb_mixed(P.ord.k); }

// Relative cost of one element block of a plan (flops of assembly and
// factorization of the batch kernels, per block of its elements).
double batch_block_cost(const hyb::Plan& P) {
  const int k = P.ord.k;
  const double n = 3.0 * (k + 1) * (k + 1) * (k + 2), Q = double((k + 2) * (k + 2) * (k + 2));
  return batch_epb_of(P) * (2.0 * n * n * Q / 2 + n * n * n / 3);
}

int batch_tiles_effective(const hyb_batch* b, int& bpc, int& ipb) {
  bpc = b->tiles.blocks_per_cu > 0 ? b->tiles.blocks_per_cu : 2;
  ipb = b->tiles.items_per_block > 0 ? b->tiles.items_per_block : 1;
  return HYB_OK;
}

void batch_build_items(hyb_batch* b) {
  int bpc, ipb;
  batch_tiles_effective(b, bpc, ipb);
  b->items.clear();
  for (size_t p = 0; p < b->plans.size(); ++p) {
    const hyb::Plan& P = b->plans[p]->P;
    if (!P.mixed) continue;   // FP64 problems: k_setup_multi, k_recover_multi
    const int epb = batch_epb_of(P);
    const int64_t nblk = (P.ne + epb - 1) / epb;
    for (int64_t q = 0; q < nblk; q += ipb) {
      hyb::BatchItem it{};
      it.prob = int32_t(p);
      it.blk0 = q;
      it.nblk = int32_t(std::min<int64_t>(ipb, nblk - q));
      b->items.push_back(it);
    }
  }
  // most expensive first, stable: deterministic order
  std::stable_sort(b->items.begin(), b->items.end(), [&](const hyb::BatchItem& x, const hyb::BatchItem& y) {
    const hyb::Plan &px = b->plans[x.prob]->P, &py = b->plans[y.prob]->P;
    return batch_block_cost(px) * x.nblk > batch_block_cost(py) * y.nblk;
  });
  b->n_mx = b->items.size();
  b->dirty = true;
}

int batch_upload(hyb_batch* b) {
  if (!b->dirty) return HYB_OK;
  if (b->items.size() > b->cap_items) {
    if (b->d_items) HYB_HIP(hipFree(b->d_items));
    b->d_items = nullptr;
    HYB_HIP(hipMalloc(&b->d_items, sizeof(hyb::BatchItem) * std::max<size_t>(b->items.size(), 1)));
    b->cap_items = b->items.size();
  }
  if (!b->items.empty())
    HYB_HIP(hipMemcpyAsync(b->d_items, b->items.data(), sizeof(hyb::BatchItem) * b->items.size(),
                           hipMemcpyHostToDevice, b->stream));
  HYB_HIP(hipMemcpyAsync(b->d_probs, b->probs.data(), sizeof(hyb::BatchProb) * b->probs.size(),
                         hipMemcpyHostToDevice, b->stream));
  HYB_HIP(hipStreamSynchronize(b->stream));
  b->dirty = false;
  for (hipGraphExec_t* g : {&b->g_setup, &b->g_recover})
    if (*g) {
      (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
  return HYB_OK;
}

unsigned batch_grid(const hyb_batch* b, size_t nitems) {
  int bpc, ipb;
  batch_tiles_effective(b, bpc, ipb);
  const int64_t want = int64_t(bpc) * b->cus;
  return unsigned(std::max<int64_t>(1, std::min(want, int64_t(nitems))));
}

int batch_launch_setup(hyb_batch* b, hipStream_t st) {
  int64_t zmax = 1;
  for (const auto& pr : b->probs) zmax = std::max<int64_t>(zmax, pr.nfaces * pr.K2 * pr.K2 + pr.m);
  const unsigned zx = unsigned(std::min<int64_t>((zmax + 255) / 256, 1024));
  hipLaunchKernelGGL(hyb::k_batch_zero, dim3(zx, unsigned(b->probs.size())), dim3(256), 0, st, b->d_probs);
  HYB_HIP(hipGetLastError());
  const size_t nmx = b->n_mx;
  // the queue counters start at zero (a kernel, not a memset: graph replays)
  if (nmx) {   // the queue counter starts at zero (a kernel, not a memset: graph replays)
    hipLaunchKernelGGL(hyb::k_fill_i32, dim3(1), dim3(64), 0, st, b->d_queue, int64_t(1), 0);
    HYB_HIP(hipGetLastError());
  }
  // the FP64 problems by order, most expensive order first, kMultiProbs
  // problems per launch with their descriptors in the kernel arguments
  for (int k = 3; k >= 0; --k) {
    const int per = hyb::setup_teams(k);
    const auto kern = k == 3 ? hyb::k_setup_multi<3>
                      : k == 2 ? hyb::k_setup_multi<2>
                      : k == 1 ? hyb::k_setup_multi<1>
                               : hyb::k_setup_multi<0>;
    hyb::MultiArgs m{};
    for (size_t p = 0; p <= b->probs.size(); ++p) {
      const bool take = p < b->probs.size() && !b->probs[p].mixed && b->probs[p].k == k && b->probs[p].s.ne > 0;
      if (take) {
        m.start[m.np + 1] = m.start[m.np] + (b->probs[p].s.ne + per - 1) / per;
        m.p[m.np++] = b->probs[p].s;
      }
      if (m.np == hyb::kMultiProbs || (p == b->probs.size() && m.np > 0)) {
        if (m.start[m.np] > int64_t(INT32_MAX)) return HYB_E_ARG;   // grid beyond the x-dimension limit
        hipLaunchKernelGGL(kern, dim3(unsigned(m.start[m.np])), dim3(hyb::setup_team(k) * per),
                           hyb::batch_setup_lds(k), st, m);
        HYB_HIP(hipGetLastError());
        m = hyb::MultiArgs{};
      }
    }
  }
  if (nmx) {
    const unsigned gm = std::min<unsigned>(batch_grid(b, nmx), unsigned(hyb::kMixedSlots));
    hipLaunchKernelGGL(hyb::k_setup_batch_mixed, dim3(gm), dim3(hyb::kBatchThreads), b->lds_setup_mx, st,
                       b->d_probs, b->d_items, int64_t(nmx), b->scratch, b->d_queue);
    HYB_HIP(hipGetLastError());
  }
  return HYB_OK;
}

int batch_launch_recover(hyb_batch* b, hipStream_t st) {
  const size_t nmx = b->n_mx;
  if (nmx) {
    hipLaunchKernelGGL(hyb::k_fill_i32, dim3(1), dim3(64), 0, st, b->d_queue + 1, int64_t(1), 0);
    HYB_HIP(hipGetLastError());
  }
  for (int k = 3; k >= 0; --k) {
    const int per = hyb::recover_teams(k);
    const auto kern = k == 3 ? hyb::k_recover_multi<3>
                      : k == 2 ? hyb::k_recover_multi<2>
                      : k == 1 ? hyb::k_recover_multi<1>
                               : hyb::k_recover_multi<0>;
    hyb::MultiRecArgs m{};
    for (size_t p = 0; p <= b->probs.size(); ++p) {
      const bool take = p < b->probs.size() && !b->probs[p].mixed && b->probs[p].k == k && b->probs[p].r.ne > 0;
      if (take) {
        m.start[m.np + 1] = m.start[m.np] + (b->probs[p].r.ne + per - 1) / per;
        m.p[m.np++] = b->probs[p].r;
      }
      if (m.np == hyb::kMultiProbs || (p == b->probs.size() && m.np > 0)) {
        if (m.start[m.np] > int64_t(INT32_MAX)) return HYB_E_ARG;   // grid beyond the x-dimension limit
        hipLaunchKernelGGL(kern, dim3(unsigned(m.start[m.np])), dim3(hyb::recover_team(k) * per),
                           hyb::batch_recover_lds(k), st, m);
        HYB_HIP(hipGetLastError());
        m = hyb::MultiRecArgs{};
      }
    }
  }
  if (nmx) {
    hipLaunchKernelGGL(hyb::k_recover_batch_mixed, dim3(batch_grid(b, nmx)), dim3(hyb::kBatchThreads),
                       b->lds_recover_mx, st, b->d_probs, b->d_items, int64_t(nmx), b->d_queue + 1);
    HYB_HIP(hipGetLastError());
  }
  return HYB_OK;
}

// A timing event recorded on st (from the batch's pool), appended to list.
int batch_mark(hyb_batch* b, std::vector<hipEvent_t>& list, hipStream_t st) {
  if (!b->timing) return HYB_OK;
  hipEvent_t e = nullptr;
  if (!b->ev_pool.empty()) {
    e = b->ev_pool.back();
    b->ev_pool.pop_back();
  } else {
    HYB_HIP(hipEventCreate(&e));
  }
  list.push_back(e);
  HYB_HIP(hipEventRecord(e, st));
  return HYB_OK;
}

// Run fn on the stream, or replay its captured graph; with timing on, the
// phase is bracketed by events on the stream it runs on.
template <class Fn>
int batch_run(hyb_batch* b, hipGraphExec_t& g, std::vector<hipEvent_t>& evs, Fn&& fn) {
  int rc = batch_upload(b);
  if (rc) return rc;
  if (!b->use_graph) {
    if ((rc = batch_mark(b, evs, b->stream))) return rc;
    if ((rc = fn(b, b->stream))) return rc;
    return batch_mark(b, evs, b->stream);
  }
  // graphs are captured and replayed on the batch's own stream, ordered
  // after and before the plans' stream by events
  if (!g) {
    hipGraph_t graph = nullptr;
    HYB_HIP(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
    rc = fn(b, b->gstream);
    hipError_t e2 = hipStreamEndCapture(b->gstream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    HYB_HIP(e2);
    hipError_t e3 = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HYB_HIP(e3);
  }
  HYB_HIP(hipEventRecord(b->ev_in, b->stream));
  HYB_HIP(hipStreamWaitEvent(b->gstream, b->ev_in, 0));
  if ((rc = batch_mark(b, evs, b->gstream))) return rc;
  HYB_HIP(hipGraphLaunch(g, b->gstream));
  if ((rc = batch_mark(b, evs, b->gstream))) return rc;
  HYB_HIP(hipEventRecord(b->ev_out, b->gstream));
  HYB_HIP(hipStreamWaitEvent(b->stream, b->ev_out, 0));
  return HYB_OK;
}

}  // namespace

extern "C" {

int hyb_batch_create(hyb_plan_t* const* plans, int32_t count, hyb_batch_t** out) {
  if (!out || count <= 0 || !plans) return HYB_E_ARG;
  *out = nullptr;
  for (int32_t i = 0; i < count; ++i)
    if (!plans[i]) return HYB_E_ARG;
  for (int32_t i = 0; i < count; ++i)
    if (!plans[i]->P.bound) return HYB_E_STATE;
  hyb_batch* b = new (std::nothrow) hyb_batch;
  if (!b) return HYB_E_NOMEM;
  b->plans.assign(plans, plans + count);
  b->stream = stream_of(plans[0]->P);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->cus <= 0)
    b->cus = 256;
  b->probs.resize(size_t(count));
  for (int32_t i = 0; i < count; ++i) {
    hyb::Plan& P = plans[i]->P;
    // the batch kernels use the generic element routines and record layout;
    // factors and y left by the affine RT_1 kernels are in that kernel's own
    // layout, so a plan switched here must be set up again (by the batch or
    // hyb_setup) before hyb_rhs or hyb_recover
    if (P.fast_k1) P.have_setup = P.have_rhs = false;
    P.fast_k1 = false;
    hyb::BatchProb& pr = b->probs[size_t(i)];
    pr = hyb::BatchProb{};
    pr.k = P.ord.k;
    pr.K2 = P.ord.K2;
    pr.mixed = P.mixed ? 1 : 0;
    pr.sweeps = P.sweeps;
    pr.nfaces = P.nfaces;
    pr.m = P.m;
    pr.s.mp = device_maps(P);
    pr.s.ne = P.ne;
    pr.s.factor = P.buf.factor;
    pr.s.y = P.buf.y;
    pr.s.Hval = P.buf.val;
    pr.s.r = P.buf.r;
    pr.s.status = P.buf.status;
    pr.s.mode = hyb::MODE_MATRIX;
    pr.s.stat = P.stat ? 1 : 0;   // static condensation: S and its load, u_b = sigma x
    pr.r.mp = pr.s.mp;
    pr.r.ne = P.ne;
    pr.r.factor = P.buf.factor;
    pr.r.y = P.buf.y;
    pr.r.stat = pr.s.stat;
    if (P.mixed) {
      b->lds_setup_mx = std::max(b->lds_setup_mx, hyb::batch_setup_lds_mixed(P.ord.k));
      b->lds_recover_mx = std::max(b->lds_recover_mx, hyb::batch_recover_lds_mixed(P.ord.k));
    }
  }
  bool mixed3 = false;
  for (int32_t i = 0; i < count; ++i) mixed3 |= plans[i]->P.mixed && plans[i]->P.ord.k == 3;
  hipError_t e1 = hipMalloc(&b->d_probs, sizeof(hyb::BatchProb) * b->probs.size());
  if (e1 == hipSuccess) e1 = hipMalloc(&b->d_queue, kQueues * sizeof(int32_t));
  if (e1 == hipSuccess && mixed3) e1 = hipMalloc(&b->scratch, size_t(mixed_scratch_bytes(3)));
  if (e1 == hipSuccess) e1 = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
  if (e1 == hipSuccess) e1 = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e1 == hipSuccess) e1 = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  {
    const void* ks[4] = {reinterpret_cast<const void*>(hyb::k_setup_multi<0>),
                         reinterpret_cast<const void*>(hyb::k_setup_multi<1>),
                         reinterpret_cast<const void*>(hyb::k_setup_multi<2>),
                         reinterpret_cast<const void*>(hyb::k_setup_multi<3>)};
    const void* kr[4] = {reinterpret_cast<const void*>(hyb::k_recover_multi<0>),
                         reinterpret_cast<const void*>(hyb::k_recover_multi<1>),
                         reinterpret_cast<const void*>(hyb::k_recover_multi<2>),
                         reinterpret_cast<const void*>(hyb::k_recover_multi<3>)};
    for (int k = 0; k < 4 && e1 == hipSuccess; ++k) {
      e1 = hipFuncSetAttribute(ks[k], hipFuncAttributeMaxDynamicSharedMemorySize, int(hyb::batch_setup_lds(k)));
      if (e1 == hipSuccess)
        e1 = hipFuncSetAttribute(kr[k], hipFuncAttributeMaxDynamicSharedMemorySize, int(hyb::batch_recover_lds(k)));
    }
  }
  if (e1 == hipSuccess && b->lds_setup_mx)
    e1 = hipFuncSetAttribute(reinterpret_cast<const void*>(hyb::k_setup_batch_mixed),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(b->lds_setup_mx));
  if (e1 == hipSuccess && b->lds_recover_mx)
    e1 = hipFuncSetAttribute(reinterpret_cast<const void*>(hyb::k_recover_batch_mixed),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(b->lds_recover_mx));
  if (e1 != hipSuccess) {
    hyb_batch_destroy(b);
    return hip_fail(e1);
  }
  batch_build_items(b);
  *out = b;
  return HYB_OK;
}

int hyb_batch_set(hyb_batch_t* b, int32_t p, const double* alpha, const double* beta, const double* f,
                  const double* g, const double* lambda, double* u) {
  if (!b || p < 0 || p >= int32_t(b->plans.size())) return HYB_E_ARG;
  hyb::BatchProb& pr = b->probs[size_t(p)];
  pr.s.alpha = alpha;
  pr.s.beta = beta;
  pr.s.f = f;
  pr.s.g = f ? g : nullptr;
  pr.s.mode = hyb::MODE_MATRIX | (f ? hyb::MODE_RHS : 0);
  pr.r.lambda = lambda;
  pr.r.u = u;
  b->dirty = true;
  return HYB_OK;
}

int hyb_batch_set_tiles(hyb_batch_t* b, const hyb_batch_tiles* tiles) {
  if (!b || !tiles || tiles->blocks_per_cu < 0 || tiles->items_per_block < 0 || tiles->blocks_per_cu > 64 ||
      tiles->items_per_block > 1024)
    return HYB_E_ARG;
  b->tiles = *tiles;
  batch_build_items(b);
  return HYB_OK;
}

int hyb_batch_get_tiles(const hyb_batch_t* b, hyb_batch_tiles* tiles) {
  if (!b || !tiles) return HYB_E_ARG;
  int bpc, ipb;
  batch_tiles_effective(b, bpc, ipb);
  tiles->blocks_per_cu = bpc;
  tiles->items_per_block = ipb;
  return HYB_OK;
}

int hyb_batch_graph(hyb_batch_t* b, int enable) {
  if (!b) return HYB_E_ARG;
  b->use_graph = enable != 0;
  return HYB_OK;
}

int hyb_batch_setup(hyb_batch_t* b) {
  if (!b) return HYB_E_ARG;
  for (const auto& pr : b->probs)
    if (!pr.s.alpha || !pr.s.beta) return HYB_E_STATE;
  int rc = batch_run(b, b->g_setup, b->ev_setup, batch_launch_setup);
  if (rc) return rc;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    hyb::Plan& P = b->plans[i]->P;
    P.have_setup = true;
    P.have_rhs = b->probs[i].s.f != nullptr;
    P.alpha_d = b->probs[i].s.alpha;
    P.beta_d = b->probs[i].s.beta;
  }
  return HYB_OK;
}

int hyb_batch_recover(hyb_batch_t* b) {
  if (!b) return HYB_E_ARG;
  for (size_t i = 0; i < b->plans.size(); ++i)
    if (!b->plans[i]->P.have_rhs || !b->probs[i].r.lambda || !b->probs[i].r.u) return HYB_E_STATE;
  return batch_run(b, b->g_recover, b->ev_recover, batch_launch_recover);
}

int hyb_batch_autotune(hyb_batch_t* b, int reps, hyb_batch_tiles* best) {
  if (!b || reps <= 0) return HYB_E_ARG;
  for (const auto& pr : b->probs)
    if (!pr.s.alpha || !pr.s.beta || !pr.r.lambda || !pr.r.u) return HYB_E_STATE;
  bool any_mixed = false;
  for (const auto& pr : b->probs) any_mixed |= pr.mixed != 0;
  if (!any_mixed) {   // the tiles shape only the mixed problems' launch
    const hyb_batch_tiles t{2, 1};
    const int rc = hyb_batch_set_tiles(b, &t);
    if (!rc && best) *best = t;
    return rc;
  }
  const bool graph = b->use_graph, timing = b->timing;
  b->use_graph = false;
  b->timing = false;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  HYB_HIP(hipEventCreate(&t0));
  HYB_HIP(hipEventCreate(&t1));
  const int bpcs[] = {1, 2, 4, 8};
  const int ipbs[] = {1, 2, 4, 8};
  hyb_batch_tiles win{2, 1};
  float wbest = -1.0f;
  int rc = HYB_OK;
  for (int bpc : bpcs) {
    for (int ipb : ipbs) {
      hyb_batch_tiles t{bpc, ipb};
      if ((rc = hyb_batch_set_tiles(b, &t))) break;
      // one untimed pass, then reps timed passes of setup + recovery
      if ((rc = hyb_batch_setup(b)) || (rc = hyb_batch_recover(b))) break;
      if (hipEventRecord(t0, b->stream) != hipSuccess) { rc = HYB_E_HIP; break; }
      for (int r = 0; r < reps && !rc; ++r) {
        rc = hyb_batch_setup(b);
        if (!rc) rc = hyb_batch_recover(b);
      }
      if (rc) break;
      if (hipEventRecord(t1, b->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess) {
        rc = HYB_E_HIP;
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, t0, t1);
      if (wbest < 0.0f || ms < wbest) {
        wbest = ms;
        win = t;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  b->use_graph = graph;
  b->timing = timing;
  if (rc) return rc;
  rc = hyb_batch_set_tiles(b, &win);
  if (rc) return rc;
  if (best) *best = win;
  return HYB_OK;
}

int hyb_batch_timing_enable(hyb_batch_t* b, int on) {
  if (!b) return HYB_E_ARG;
  for (auto* L : {&b->ev_setup, &b->ev_recover}) {
    for (hipEvent_t e : *L) b->ev_pool.push_back(e);
    L->clear();
  }
  b->timing = on != 0;
  return HYB_OK;
}

int hyb_batch_timing_read(hyb_batch_t* b, double* ms_setup, int* n_setup, double* ms_recover, int* n_recover) {
  if (!b) return HYB_E_ARG;
  HYB_HIP(hipStreamSynchronize(b->stream));
  if (b->gstream) HYB_HIP(hipStreamSynchronize(b->gstream));
  auto sum = [&](std::vector<hipEvent_t>& L, double* ms, int* cnt) -> int {
    double tot = 0.0;
    int c = 0;
    for (size_t i = 0; i + 1 < L.size(); i += 2) {
      float t = 0.0f;
      hipError_t err = hipEventElapsedTime(&t, L[i], L[i + 1]);
      if (err != hipSuccess) return hip_fail(err);
      tot += t;
      ++c;
    }
    for (hipEvent_t e : L) b->ev_pool.push_back(e);
    L.clear();
    if (ms) *ms = tot;
    if (cnt) *cnt = c;
    return HYB_OK;
  };
  int rc = sum(b->ev_setup, ms_setup, n_setup);
  if (rc) return rc;
  return sum(b->ev_recover, ms_recover, n_recover);
}

void hyb_batch_destroy(hyb_batch_t* b) {
  if (!b) return;
  if (b->gstream) (void)hipStreamSynchronize(b->gstream);
  for (auto* L : {&b->ev_setup, &b->ev_recover, &b->ev_pool})
    for (hipEvent_t e : *L) (void)hipEventDestroy(e);
  for (hipGraphExec_t g : {b->g_setup, b->g_recover})
    if (g) (void)hipGraphExecDestroy(g);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_probs) (void)hipFree(b->d_probs);
  if (b->scratch) (void)hipFree(b->scratch);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  delete b;
}

}  // extern "C"
