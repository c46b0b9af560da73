// Device helpers shared by the hybridization kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hyb {

// Per-order compile-time constants of RT_k on hexahedra.
template <int K>
struct RT {
  static constexpr int K1 = K + 1;
  static constexpr int K2 = K1 * K1;
  static constexpr int n = 3 * K2 * (K + 2);     // broken dofs per element
  static constexpr int ni = 3 * K * K2;          // interior dofs
  static constexpr int nb = 6 * K2;              // face dofs
  static constexpr int q1 = K + 2;               // Gauss points per direction
  static constexpr int Q = q1 * q1 * q1;
  static constexpr int npk = n * (n + 1) / 2;    // packed lower triangle
  static constexpr int nbpk = nb * (nb + 1) / 2;
  // component (axis) of the local dof i
  __device__ __host__ __forceinline__ static constexpr int comp(int i) {
    return i < ni ? i / (K * K2 > 0 ? K * K2 : 1) : ((i - ni) / K2) >> 1;
  }
};

// Packed row-major lower triangle index, j <= i.
__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }

// Inverse of pk: linear index t -> (i, j) with j <= i (an FP32 estimate,
// exact after the correction steps for t < 2^24).
__device__ __forceinline__ void unpk(int t, int& i, int& j) {
  int r = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  i = r;
  j = t - r * (r + 1) / 2;
}

// Advance a packed lower-triangle position (i, j) by d entries (row i holds
// i + 1 entries): the incremental form of unpk for strided loops.
__device__ __forceinline__ void pk_advance(int& i, int& j, int d) {
  j += d;
  while (j > i) {
    j -= i + 1;
    ++i;
  }
}

// Neighbour frame -> owner frame on face dof indices (j0, j1) in 0..K:
// swap (bit 0), mirror j0 (bit 1), mirror j1 (bit 2).
__device__ __forceinline__ void frame_map(int pi, int K, int& p0, int& p1) {
  if (pi & 1) { int t = p0; p0 = p1; p1 = t; }
  if (pi & 2) p0 = K - p0;
  if (pi & 4) p1 = K - p1;
}

struct DeviceMaps {
  const int32_t* e2v;
  const double* xyz;
  const int32_t* elem_face;
  const uint8_t* elem_pi;      // 8 bytes per element: frame code per face, byte 6 natural-face bits
  const uint8_t* elem_slot;    // 36 bytes per element
  const int64_t* face_rowbase;
  const int32_t* face_nslots;
  const double* tab_s;         // Q x n
  const double* tab_d;         // Q x n
  const double* tab_w;         // Q
  const double* tab_ref;       // 2 n^2 + n
  const double* gauss_x;       // q1 points on [0,1]
  const int32_t* face_selfslot;
  const int32_t* face_owner;   // owner element of every interior face
  const double* k1_geo;        // RT_1 affine: per-element edge vectors (9)
  const uint8_t* k1_meta;      // RT_1 affine: per-element face data (144 B)
  const double* face_w;        // multiplier weight per face-dof position (K2)
  const double* tab1d;         // 1D tables [basis][point]: closed values, derivatives, open values
};

// Sticky device error: the first (code, element) pair wins.
__device__ __forceinline__ void report_error(int32_t* status, int code, int64_t elem) {
  if (atomicCAS(reinterpret_cast<int*>(status), 0, code) == 0) status[1] = int32_t(elem);
}

}  // namespace hyb
