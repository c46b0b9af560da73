// Host-side plan of the hybridization library: mesh copy, topology of the
// constraint matrix C (faces, owners, neighbour frame codes, multiplier ids),
// the CSR pattern of H with per-element scatter slots, reference basis tables
// at the quadrature points, and the layout of the caller-owned device buffers.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hyb.h"

namespace hyb {

// Per-order constants of RT_k on hexahedra.
struct Order {
  int k = 0;
  int K1 = 1;     // k + 1 open (Gauss-Legendre) points per tangential axis
  int K2 = 1;     // (k+1)^2 dofs per face
  int n = 6;      // 3 (k+1)^2 (k+2) broken dofs per element
  int ni = 0;     // 3 k (k+1)^2 interior dofs
  int nb = 6;     // 6 (k+1)^2 face dofs
  int q1 = 2;     // Gauss points per direction (k + 2)
  int Q = 8;      // q1^3
  explicit Order(int k_ = 0);
};

// Face data of one element for the RT_1 scatter into H (copied to the
// device as raw bytes).
struct K1Meta {
  static constexpr int kBytes = 144;
  int64_t rb[6];     // first CSR entry of the face's row block
  int32_t fid[6];    // face index, -1 on the boundary
  int32_t ns[6];     // column blocks per row of the face
  uint8_t slot[36];  // slot of face fb in the rows of face fa
  uint8_t pi[6];     // frame code
  uint8_t own;       // bit f: this element owns face f
  uint8_t pad[5];
};
static_assert(sizeof(K1Meta) == K1Meta::kBytes, "K1Meta layout");

// Byte offsets of every array inside the device "maps" buffer.
struct MapLayout {
  size_t e2v = 0, xyz = 0, elem_face = 0, elem_pi = 0, elem_slot = 0,
         face_rowbase = 0, face_nslots = 0, tab_s = 0, tab_d = 0, tab_w = 0,
         tab_ref = 0, tab_x = 0, tab_1d = 0, face_selfslot = 0, face_owner = 0, k1_geo = 0, k1_meta = 0, face_w = 0,
         total = 0;
};

struct Plan {
  Order ord;
  int64_t ne = 0, nv = 0;
  std::vector<double> xyz;          // nv x 3
  std::vector<int32_t> e2v;         // ne x 8
  // topology
  int64_t nfaces = 0, nbfaces = 0;  // interior / boundary faces
  std::vector<int32_t> elem_face;   // ne x 6, interior face id or -1
  std::vector<uint8_t> elem_pi;     // ne x 8: neighbour frame code per face (0..5),
                                    // byte 6: bit f set = face f is a natural boundary face
  bool has_natural = false;         // some boundary face is natural
  std::vector<int32_t> face_owner;  // nfaces x 2 (element, local face)
  std::vector<int32_t> face_nbr;    // nfaces x 2
  // CSR of H and scatter slots
  int64_t m = 0, nnz = 0;
  std::vector<int64_t> row_ptr;     // m + 1
  std::vector<int32_t> col;         // nnz
  std::vector<int64_t> face_rowbase;  // nfaces: row_ptr of the face's first row
  std::vector<int32_t> face_nslots;   // nfaces: faces in the face's rows
  std::vector<uint8_t> elem_slot;     // ne x 36: slot of face b in face a's rows
  std::vector<int32_t> face_selfslot; // nfaces: slot of the face in its own rows
  bool all_affine = false;            // every element is a parallelepiped
  bool fast_k1 = false;               // RT_1 affine kernels (own factor record layout)
  bool mixed = false;                 // HYB_MIXED element kernels (own factor record layout)
  bool stat = false;                  // HYB_STATIC: static condensation S instead of H
  int sweeps = 0;                     // HYB_MIXED refinement sweeps
  // reference tables at the Gauss points (axis 0 fastest)
  std::vector<double> tab_s;        // Q x n: basis value (its only nonzero component)
  std::vector<double> tab_d;        // Q x n: reference divergence
  std::vector<double> tab_w;        // Q: weights
  std::vector<double> tab_ref;      // affine reference integrals (see plan.cpp)
  std::vector<double> tab_x;        // q1 Gauss points on [0,1]
  std::vector<double> tab_1d;       // 1D tables [basis][point]: closed values (k+2), their
                                    // derivatives (k+2), open values (k+1)
  // RT_1 affine kernels: per-element edge vectors J (9 doubles, row-major,
  // J[r][c] = x_{v_c}[r] - x_0[r] for vertices v = 1, 2, 4) and the element's
  // face data for the scatter into H (K1Meta, 144 bytes)
  std::vector<double> k1_geo;
  // multiplier weights per face-dof position (K2): the diagonal of the face
  // mass matrix M_s of the weighted constraint C = M_s C_0, or all ones
  std::vector<double> face_w;
  std::vector<uint8_t> k1_meta;
  MapLayout lay;
  int64_t factor_len = 0;
  // device state
  hyb_opts opts{};
  hyb_buffers buf{};
  bool bound = false, have_setup = false, have_rhs = false;
  const double* alpha_d = nullptr;  // coefficients of the last setup (caller-owned)
  const double* beta_d = nullptr;
  int work_blocks = 0;                // PCG vector kernels (init, update)
  int spmv_blocks = 0;                // PCG SpMV
  int64_t max_row = 0;                // longest row of H
  // optional HIP-event timing of the main kernels (hipEvent_t kept as void*)
  bool timing = false;
  std::vector<void*> ev_setup, ev_recover;  // start/stop pairs, in launch order
  std::vector<void*> ev_pool;
};

int build_plan(const hyb_mesh* mesh, int k, Plan& P, int64_t& detail);

// 1D rules written for this library (Newton on Legendre polynomials).
void gauss_legendre_01(int q, std::vector<double>& x, std::vector<double>& w);
void gauss_lobatto_01(int npts, std::vector<double>& x);

}  // namespace hyb
