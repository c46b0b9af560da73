// Host planning under AddressSanitizer and UndefinedBehaviorSanitizer: builds
// plans for seeded structured, jittered and rotated hex meshes of every order
// (with random natural-face masks), checks the topology and CSR invariants,
// and drives every error path of the planner.  Prints "ok" and exits 0 on
// success.  Built and run by tests/test_host_sanitizers.py.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "../../paper_1801_08914_amd/csrc/plan.hpp"

namespace {

uint64_t g_state = 0x9e3779b97f4a7c15ull;
uint64_t next_u64() {   // splitmix64
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
double uniform() { return double(next_u64() >> 11) * 0x1p-53; }

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                      \
    }                                                                    \
  } while (0)

struct Mesh {
  std::vector<double> xyz;
  std::vector<int32_t> e2v;
  int64_t nv = 0, ne = 0;
};

// Structured N^3 mesh of the unit cube, interior vertices jittered by up to
// jit h, each element's vertex order turned by a random one of the symmetries
// that keep det J > 0 (a cyclic permutation of the axes, then two axes
// mirrored or none).
Mesh structured(int N, double jit, bool rotate) {
  Mesh m;
  const int V = N + 1;
  m.nv = int64_t(V) * V * V;
  m.ne = int64_t(N) * N * N;
  for (int l = 0; l < V; ++l)
    for (int j = 0; j < V; ++j)
      for (int i = 0; i < V; ++i) {
        const int c[3] = {i, j, l};
        for (int d = 0; d < 3; ++d) {
          double x = double(c[d]) / N;
          const bool inner = i > 0 && i < N && j > 0 && j < N && l > 0 && l < N;
          if (inner) x += jit * (2.0 * uniform() - 1.0) / N;
          m.xyz.push_back(x);
        }
      }
  for (int l = 0; l < N; ++l)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        int32_t v[8];
        for (int c = 0; c < 8; ++c) {
          const int a = c & 1, b = (c >> 1) & 1, cc = c >> 2;
          v[c] = int32_t((i + a) + V * ((j + b) + V * (l + cc)));
        }
        if (rotate) {
          const int shift = int(next_u64() % 3), mir = int(next_u64() % 4);
          int32_t w[8];
          for (int c = 0; c < 8; ++c) {
            int bits[3] = {c & 1, (c >> 1) & 1, c >> 2};
            int r[3];
            for (int d = 0; d < 3; ++d) r[(d + shift) % 3] = bits[d];
            if (mir == 1) { r[0] ^= 1; r[1] ^= 1; }
            if (mir == 2) { r[1] ^= 1; r[2] ^= 1; }
            if (mir == 3) { r[0] ^= 1; r[2] ^= 1; }
            w[c] = v[r[0] + 2 * r[1] + 4 * r[2]];
          }
          for (int c = 0; c < 8; ++c) v[c] = w[c];
        }
        for (int c = 0; c < 8; ++c) m.e2v.push_back(v[c]);
      }
  return m;
}

void check_plan(const Mesh& m, int k, int N, const uint8_t* ess) {
  hyb_mesh hm{m.nv, m.ne, m.xyz.data(), m.e2v.data(), ess};
  hyb::Plan P;
  int64_t detail = -1;
  const int rc = hyb::build_plan(&hm, k, P, detail);
  CHECK(rc == HYB_OK);
  const int64_t K2 = int64_t(k + 1) * (k + 1);
  CHECK(P.nfaces == 3 * int64_t(N) * N * (N - 1));
  CHECK(P.nbfaces == 6 * int64_t(N) * N);
  CHECK(P.m == P.nfaces * K2);
  CHECK(int64_t(P.row_ptr.size()) == P.m + 1 && P.row_ptr[0] == 0 && P.row_ptr[size_t(P.m)] == P.nnz);
  for (int64_t i = 0; i < P.m; ++i) {
    CHECK(P.row_ptr[size_t(i + 1)] > P.row_ptr[size_t(i)]);
    for (int64_t q = P.row_ptr[size_t(i)]; q < P.row_ptr[size_t(i + 1)]; ++q) {
      CHECK(P.col[size_t(q)] >= 0 && P.col[size_t(q)] < P.m);
      if (q > P.row_ptr[size_t(i)]) CHECK(P.col[size_t(q)] > P.col[size_t(q - 1)]);
    }
  }
  std::vector<int> seen(size_t(P.nfaces), 0);
  for (int64_t e = 0; e < m.ne; ++e) {
    std::set<int32_t> faces;
    for (int f = 0; f < 6; ++f) {
      const int32_t F = P.elem_face[size_t(6 * e + f)];
      CHECK(F >= -1 && F < P.nfaces);
      if (F < 0) continue;
      CHECK(faces.insert(F).second);
      ++seen[size_t(F)];
      CHECK(P.elem_pi[size_t(8 * e + f)] < 8);
      for (int g = 0; g < 6; ++g)
        if (P.elem_face[size_t(6 * e + g)] >= 0) CHECK(P.elem_slot[size_t(36 * e + 6 * f + g)] < P.face_nslots[size_t(F)]);
    }
    const uint8_t nat = P.elem_pi[size_t(8 * e + 6)];
    for (int f = 0; f < 6; ++f) {
      const bool boundary = P.elem_face[size_t(6 * e + f)] < 0;
      const bool natural = ess && boundary && ess[6 * e + f] == 0;
      CHECK(((nat >> f) & 1) == (natural ? 1 : 0));
    }
  }
  for (int64_t F = 0; F < P.nfaces; ++F) {
    CHECK(seen[size_t(F)] == 2);
    CHECK(P.face_owner[size_t(2 * F)] < P.face_nbr[size_t(2 * F)]);
    CHECK(P.face_nslots[size_t(F)] >= 1 && P.face_nslots[size_t(F)] <= 11);
  }
  CHECK(int64_t(P.tab_s.size()) == int64_t(P.ord.Q) * P.ord.n);
  CHECK(P.lay.total > 0);
}

int expect_error(const hyb_mesh* hm, int k, int code) {
  hyb::Plan P;
  int64_t detail = -1;
  const int rc = hyb::build_plan(hm, k, P, detail);
  CHECK(rc == code);
  return int(detail);
}

}  // namespace

int main() {
  for (int N = 1; N <= 4; ++N)
    for (int k = 0; k <= 3; ++k)
      for (int variant = 0; variant < 3; ++variant) {
        const Mesh m = structured(N, variant ? 0.2 : 0.0, variant == 2);
        std::vector<uint8_t> ess(size_t(6 * m.ne));
        for (auto& x : ess) x = uint8_t(next_u64() & 1);
        check_plan(m, k, N, nullptr);
        check_plan(m, k, N, ess.data());
      }
  // error paths
  Mesh m = structured(2, 0.0, false);
  hyb_mesh hm{m.nv, m.ne, m.xyz.data(), m.e2v.data(), nullptr};
  expect_error(nullptr, 1, HYB_E_ARG);
  expect_error(&hm, 4, HYB_E_ARG);
  expect_error(&hm, -1, HYB_E_ARG);
  {
    Mesh bad = m;
    bad.e2v[3 * 8 + 5] = int32_t(bad.nv + 7);
    hyb_mesh hb{bad.nv, bad.ne, bad.xyz.data(), bad.e2v.data(), nullptr};
    CHECK(expect_error(&hb, 1, HYB_E_MESH) == 3);
  }
  {
    Mesh inv = m;
    const int perm[8] = {1, 0, 3, 2, 5, 4, 7, 6};   // mirrored element: det J < 0
    int32_t w[8];
    for (int c = 0; c < 8; ++c) w[c] = inv.e2v[size_t(5 * 8 + perm[c])];
    for (int c = 0; c < 8; ++c) inv.e2v[size_t(5 * 8 + c)] = w[c];
    hyb_mesh hi{inv.nv, inv.ne, inv.xyz.data(), inv.e2v.data(), nullptr};
    CHECK(expect_error(&hi, 1, HYB_E_JACOBIAN) == 5);
  }
  {
    std::vector<int32_t> tri;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 8; ++c) tri.push_back(m.e2v[size_t(c)]);
    hyb_mesh ht{m.nv, 3, m.xyz.data(), tri.data(), nullptr};
    expect_error(&ht, 0, HYB_E_MESH);
  }
  {
    hyb_mesh he{0, 0, nullptr, nullptr, nullptr};
    hyb::Plan P;
    int64_t detail = -1;
    CHECK(hyb::build_plan(&he, 2, P, detail) == HYB_OK && P.m == 0 && P.nnz == 0);
  }
  std::printf("ok\n");
  return 0;
}
