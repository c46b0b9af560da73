// Host planning: topology of the multiplier space, CSR pattern of H,
// scatter slots and reference tables.  No GPU calls here, so a plan can be
// built and inspected on a machine without a GPU.
#include "plan.hpp"

#include <cstring>

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

namespace hyb {

Order::Order(int k_) : k(k_) {
  K1 = k + 1;
  K2 = K1 * K1;
  n = 3 * K2 * (k + 2);
  ni = 3 * k * K2;
  nb = 6 * K2;
  q1 = k + 2;
  Q = q1 * q1 * q1;
}

namespace {

constexpr double kPi = 3.14159265358979323846;

// Legendre P_N and P'_N at x in [-1,1] by the three-term recurrence.
void legendre(int N, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (N == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 1; j < N; ++j) {
    double p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = N * (x * p1 - p0) / (x * x - 1.0);
}

// Local vertex of face f at face corner a + 2b.
int face_corner(int f, int c) {
  int d = f >> 1, s = f & 1;
  int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
  int a = c & 1, b = c >> 1;
  return (s << d) | (a << t0) | (b << t1);
}

// Neighbour frame (p0, p1) -> owner frame: swap (bit 0), then mirror p0
// (bit 1), then mirror p1 (bit 2), with indices in 0..K.
inline void frame_map(int pi, int K, int& p0, int& p1) {
  if (pi & 1) std::swap(p0, p1);
  if (pi & 2) p0 = K - p0;
  if (pi & 4) p1 = K - p1;
}

std::vector<double> lagrange_at(const std::vector<double>& z, double x) {
  std::vector<double> v(z.size(), 1.0);
  for (size_t i = 0; i < z.size(); ++i)
    for (size_t j = 0; j < z.size(); ++j)
      if (j != i) v[i] *= (x - z[j]) / (z[i] - z[j]);
  return v;
}

std::vector<double> lagrange_deriv_at(const std::vector<double>& z, double x) {
  std::vector<double> v(z.size(), 0.0);
  for (size_t i = 0; i < z.size(); ++i)
    for (size_t m = 0; m < z.size(); ++m) {
      if (m == i) continue;
      double t = 1.0 / (z[i] - z[m]);
      for (size_t j = 0; j < z.size(); ++j)
        if (j != i && j != m) t *= (x - z[j]) / (z[i] - z[j]);
      v[i] += t;
    }
  return v;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

void gauss_legendre_01(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double t = std::cos(kPi * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(q, t, p, dp);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    double p, dp;
    legendre(q, t, p, dp);
    // map to [0,1] ascending: t descends with i
    x[q - 1 - i] = 0.5 * (t + 1.0);
    w[q - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // (2/((1-t^2) P'^2)) / 2
  }
}

void gauss_lobatto_01(int npts, std::vector<double>& x) {
  int N = npts - 1;  // roots of P'_N plus the two ends
  x.assign(npts, 0.0);
  x[0] = 0.0;
  x[npts - 1] = 1.0;
  for (int i = 1; i < N; ++i) {
    double t = -std::cos(kPi * i / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(N, t, p, dp);
      double d2p = (2.0 * t * dp - N * (N + 1) * p) / (1.0 - t * t);
      double dt = dp / d2p;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    x[i] = 0.5 * (t + 1.0);
  }
  std::sort(x.begin(), x.end());
}

int build_plan(const hyb_mesh* mesh, int k, Plan& P, int64_t& detail) {
  detail = -1;
  if (!mesh || k < 0 || k > 3 || mesh->ne < 0 || mesh->nv < 0) return HYB_E_ARG;
  if ((mesh->ne > 0 && !mesh->e2v) || (mesh->nv > 0 && !mesh->xyz)) return HYB_E_ARG;
  if (mesh->ne > (int64_t(1) << 31) - 2) return HYB_E_ARG;
  P.ord = Order(k);
  const Order& o = P.ord;
  P.ne = mesh->ne;
  P.nv = mesh->nv;
  P.xyz.assign(mesh->xyz, mesh->xyz + 3 * mesh->nv);
  P.e2v.assign(mesh->e2v, mesh->e2v + 8 * mesh->ne);
  const int64_t ne = P.ne;
  for (int64_t i = 0; i < 8 * ne; ++i)
    if (P.e2v[i] < 0 || P.e2v[i] >= P.nv) { detail = i / 8; return HYB_E_MESH; }

  // det J > 0 at the eight corners (edge vectors from each corner).
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t* ev = &P.e2v[8 * e];
    for (int v = 0; v < 8; ++v) {
      double J[3][3];
      for (int d = 0; d < 3; ++d) {
        int v1 = v | (1 << d), v0 = v & ~(1 << d);
        for (int r = 0; r < 3; ++r) J[r][d] = P.xyz[3 * ev[v1] + r] - P.xyz[3 * ev[v0] + r];
      }
      double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                   J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                   J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (!(det > 0.0)) { detail = e; return HYB_E_JACOBIAN; }
    }
  }

  // Parallelepipeds: x_v = x_0 + a E_0 + b E_1 + c E_2 at every vertex, up
  // to rounding of the coordinates themselves.
  P.all_affine = true;
  for (int64_t e = 0; e < ne && P.all_affine; ++e) {
    const int32_t* ev = &P.e2v[8 * e];
    double E[3][3], scale = 0.0;
    for (int d = 0; d < 3; ++d)
      for (int r = 0; r < 3; ++r) {
        E[d][r] = P.xyz[3 * ev[1 << d] + r] - P.xyz[3 * ev[0] + r];
        scale = std::max(scale, std::fabs(P.xyz[3 * ev[1 << d] + r]) + std::fabs(P.xyz[3 * ev[0] + r]));
      }
    for (int v = 3; v < 8 && P.all_affine; ++v) {
      for (int r = 0; r < 3; ++r) {
        double pred = P.xyz[3 * ev[0] + r];
        for (int d = 0; d < 3; ++d)
          if ((v >> d) & 1) pred += E[d][r];
        if (std::fabs(P.xyz[3 * ev[v] + r] - pred) > 1e-13 * (scale + 1e-300)) P.all_affine = false;
      }
    }
  }

  // Faces: sort (sorted vertex quadruple, element, local face) records.
  struct Rec { std::array<int32_t, 4> key; int32_t e; int32_t f; };
  std::vector<Rec> recs(size_t(6 * ne));
  for (int64_t e = 0; e < ne; ++e)
    for (int f = 0; f < 6; ++f) {
      Rec& r = recs[size_t(6 * e + f)];
      for (int c = 0; c < 4; ++c) r.key[c] = P.e2v[8 * e + face_corner(f, c)];
      std::sort(r.key.begin(), r.key.end());
      r.e = int32_t(e);
      r.f = f;
    }
  std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
    if (a.key != b.key) return a.key < b.key;
    if (a.e != b.e) return a.e < b.e;
    return a.f < b.f;
  });
  std::vector<int64_t> partner(size_t(6 * ne), -1);  // (e*6+f) of the other copy
  P.nbfaces = 0;
  for (size_t i = 0; i < recs.size();) {
    size_t j = i + 1;
    while (j < recs.size() && recs[j].key == recs[i].key) ++j;
    if (j - i > 2) { detail = recs[i].e; return HYB_E_MESH; }
    if (j - i == 2) {
      if (recs[i].e == recs[i + 1].e) { detail = recs[i].e; return HYB_E_MESH; }
      int64_t a = int64_t(recs[i].e) * 6 + recs[i].f, b = int64_t(recs[i + 1].e) * 6 + recs[i + 1].f;
      partner[size_t(a)] = b;
      partner[size_t(b)] = a;
    } else {
      ++P.nbfaces;
    }
    i = j;
  }
  // Number interior faces by (owner, owner's local face).
  P.elem_face.assign(size_t(6 * ne), -1);
  P.elem_pi.assign(size_t(8 * ne), 0);
  P.face_owner.clear();
  P.face_nbr.clear();
  int64_t nf = 0;
  for (int64_t e = 0; e < ne; ++e)
    for (int f = 0; f < 6; ++f) {
      int64_t pr = partner[size_t(6 * e + f)];
      if (pr < 0 || pr / 6 < e) continue;
      int64_t en = pr / 6;
      int fn = int(pr % 6);
      P.elem_face[size_t(6 * e + f)] = int32_t(nf);
      P.elem_face[size_t(6 * en + fn)] = int32_t(nf);
      P.face_owner.push_back(int32_t(e));
      P.face_owner.push_back(f);
      P.face_nbr.push_back(int32_t(en));
      P.face_nbr.push_back(fn);
      int vo[4], vn[4];
      for (int c = 0; c < 4; ++c) {
        vo[c] = P.e2v[8 * e + face_corner(f, c)];
        vn[c] = P.e2v[8 * en + face_corner(fn, c)];
      }
      int found = -1;
      for (int pi = 0; pi < 8 && found < 0; ++pi) {
        bool ok = true;
        for (int c = 0; c < 4 && ok; ++c) {
          int a = c & 1, b = c >> 1;
          frame_map(pi, 1, a, b);
          ok = vo[a + 2 * b] == vn[c];
        }
        if (ok) found = pi;
      }
      if (found < 0) { detail = en; return HYB_E_MESH; }
      P.elem_pi[size_t(8 * en + fn)] = uint8_t(found);
      ++nf;
    }
  P.nfaces = nf;
  // natural boundary faces (Sec. 5: only faces with prescribed normal flux
  // are eliminated): bit f of byte 6 of the element's frame record
  P.has_natural = false;
  if (mesh->ess) {
    for (int64_t e = 0; e < ne; ++e)
      for (int f = 0; f < 6; ++f)
        if (P.elem_face[size_t(6 * e + f)] < 0 && mesh->ess[6 * e + f] == 0) {
          P.elem_pi[size_t(8 * e + 6)] |= uint8_t(1u << f);
          P.has_natural = true;
        }
  }
  P.m = nf * o.K2;
  if (P.m > (int64_t(1) << 31) - 1) return HYB_E_ARG;

  // Row pattern of each face: the interior faces of its two elements.
  P.face_rowbase.assign(size_t(nf), 0);
  P.face_nslots.assign(size_t(nf), 0);
  std::vector<std::array<int32_t, 11>> slots(static_cast<size_t>(nf));
  int64_t base = 0;
  for (int64_t F = 0; F < nf; ++F) {
    int32_t lst[12];
    int cnt = 0;
    for (int side = 0; side < 2; ++side) {
      int64_t e = side == 0 ? P.face_owner[size_t(2 * F)] : P.face_nbr[size_t(2 * F)];
      for (int f = 0; f < 6; ++f) {
        int32_t G = P.elem_face[size_t(6 * e + f)];
        if (G >= 0) lst[cnt++] = G;
      }
    }
    std::sort(lst, lst + cnt);
    cnt = int(std::unique(lst, lst + cnt) - lst);
    if (cnt > 11) { detail = P.face_owner[size_t(2 * F)]; return HYB_E_MESH; }
    for (int s = 0; s < cnt; ++s) slots[size_t(F)][size_t(s)] = lst[s];
    P.face_nslots[size_t(F)] = cnt;
    P.face_rowbase[size_t(F)] = base;
    base += int64_t(o.K2) * cnt * o.K2;
  }
  P.nnz = base;
  P.row_ptr.assign(size_t(P.m + 1), 0);
  P.col.assign(size_t(P.nnz), 0);
  for (int64_t F = 0; F < nf; ++F) {
    int cnt = P.face_nslots[size_t(F)];
    for (int j = 0; j < o.K2; ++j) {
      int64_t row = F * o.K2 + j;
      int64_t start = P.face_rowbase[size_t(F)] + int64_t(j) * cnt * o.K2;
      P.row_ptr[size_t(row)] = start;
      for (int s = 0; s < cnt; ++s)
        for (int jj = 0; jj < o.K2; ++jj)
          P.col[size_t(start + s * o.K2 + jj)] = int32_t(int64_t(slots[size_t(F)][size_t(s)]) * o.K2 + jj);
    }
  }
  P.row_ptr[size_t(P.m)] = P.nnz;
  P.face_selfslot.assign(size_t(nf), 0);
  for (int64_t F = 0; F < nf; ++F) {
    const auto& L = slots[size_t(F)];
    int cnt = P.face_nslots[size_t(F)];
    P.face_selfslot[size_t(F)] = int32_t(std::lower_bound(L.begin(), L.begin() + cnt, int32_t(F)) - L.begin());
  }
  P.elem_slot.assign(size_t(36 * ne), 255);
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < 6; ++a) {
      int32_t Fa = P.elem_face[size_t(6 * e + a)];
      if (Fa < 0) continue;
      for (int b = 0; b < 6; ++b) {
        int32_t Fb = P.elem_face[size_t(6 * e + b)];
        if (Fb < 0) continue;
        const auto& L = slots[size_t(Fa)];
        int cnt = P.face_nslots[size_t(Fa)];
        int s = int(std::lower_bound(L.begin(), L.begin() + cnt, Fb) - L.begin());
        P.elem_slot[size_t(36 * e + 6 * a + b)] = uint8_t(s);
      }
    }

  // Reference tables at the tensor Gauss points.
  std::vector<double> xq, wq, zo, wo, zc;
  gauss_legendre_01(o.q1, xq, wq);
  gauss_legendre_01(o.K1, zo, wo);
  gauss_lobatto_01(k + 2, zc);
  P.tab_x = xq;
  std::vector<std::vector<double>> Lc(o.q1), dLc(o.q1), Lo(o.q1);
  for (int a = 0; a < o.q1; ++a) {
    Lc[a] = lagrange_at(zc, xq[a]);
    dLc[a] = lagrange_deriv_at(zc, xq[a]);
    Lo[a] = lagrange_at(zo, xq[a]);
  }
  // 1D tables at the Gauss points, [basis][point]: closed Lagrange values,
  // their derivatives, open Lagrange values (the factors of the tensor basis)
  P.tab_1d.assign(size_t((2 * (k + 2) + (k + 1)) * o.q1), 0.0);
  for (int a = 0; a < o.q1; ++a) {
    for (int i = 0; i < k + 2; ++i) {
      P.tab_1d[size_t(i * o.q1 + a)] = Lc[a][size_t(i)];
      P.tab_1d[size_t(((k + 2) + i) * o.q1 + a)] = dLc[a][size_t(i)];
    }
    for (int j = 0; j < k + 1; ++j) P.tab_1d[size_t((2 * (k + 2) + j) * o.q1 + a)] = Lo[a][size_t(j)];
  }
  // dof -> (d, ic, j0, j1) in local order
  std::vector<std::array<int, 4>> dof;
  for (int d = 0; d < 3; ++d)
    for (int j1 = 0; j1 < o.K1; ++j1)
      for (int j0 = 0; j0 < o.K1; ++j0)
        for (int i = 1; i <= k; ++i) dof.push_back({d, i, j0, j1});
  for (int f = 0; f < 6; ++f)
    for (int j1 = 0; j1 < o.K1; ++j1)
      for (int j0 = 0; j0 < o.K1; ++j0) dof.push_back({f >> 1, (f & 1) * o.K1, j0, j1});
  P.tab_s.assign(size_t(o.Q * o.n), 0.0);
  P.tab_d.assign(size_t(o.Q * o.n), 0.0);
  P.tab_w.assign(size_t(o.Q), 0.0);
  for (int q2 = 0; q2 < o.q1; ++q2)
    for (int q1 = 0; q1 < o.q1; ++q1)
      for (int q0 = 0; q0 < o.q1; ++q0) {
        int q = q0 + o.q1 * (q1 + o.q1 * q2);
        int qa[3] = {q0, q1, q2};
        P.tab_w[size_t(q)] = wq[q0] * wq[q1] * wq[q2];
        for (int i = 0; i < o.n; ++i) {
          int d = dof[size_t(i)][0], ic = dof[size_t(i)][1], j0 = dof[size_t(i)][2], j1 = dof[size_t(i)][3];
          int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
          double tang = Lo[qa[t0]][size_t(j0)] * Lo[qa[t1]][size_t(j1)];
          P.tab_s[size_t(q * o.n + i)] = Lc[qa[d]][size_t(ic)] * tang;
          P.tab_d[size_t(q * o.n + i)] = dLc[qa[d]][size_t(ic)] * tang;
        }
      }
  // Affine reference integrals, computed for j <= i and mirrored so the table
  // is exactly symmetric: {T[i][j], Dr[i][j]} pairs at 2 (n i + j) with
  // T[i][j] = sum_q w s_i s_j and Dr[i][j] = sum_q w div_i div_j; then
  // sr[i] = sum_q w s_i at 2 n^2.
  P.tab_ref.assign(size_t(2 * o.n * o.n + o.n), 0.0);
  for (int q = 0; q < o.Q; ++q) {
    double w = P.tab_w[size_t(q)];
    for (int i = 0; i < o.n; ++i) {
      double si = P.tab_s[size_t(q * o.n + i)], di = P.tab_d[size_t(q * o.n + i)];
      P.tab_ref[size_t(2 * o.n * o.n + i)] += w * si;
      for (int j = 0; j <= i; ++j) {
        P.tab_ref[size_t(2 * (i * o.n + j))] += w * si * P.tab_s[size_t(q * o.n + j)];
        P.tab_ref[size_t(2 * (i * o.n + j) + 1)] += w * di * P.tab_d[size_t(q * o.n + j)];
      }
    }
  }
  for (int i = 0; i < o.n; ++i)
    for (int j = 0; j < i; ++j) {
      P.tab_ref[size_t(2 * (j * o.n + i))] = P.tab_ref[size_t(2 * (i * o.n + j))];
      P.tab_ref[size_t(2 * (j * o.n + i) + 1)] = P.tab_ref[size_t(2 * (i * o.n + j) + 1)];
    }

  // Device map layout.
  MapLayout& L = P.lay;
  size_t off = 0;
  L.e2v = off;          off = align256(off + sizeof(int32_t) * 8 * size_t(ne));
  L.xyz = off;          off = align256(off + sizeof(double) * 3 * size_t(P.nv));
  L.elem_face = off;    off = align256(off + sizeof(int32_t) * 6 * size_t(ne));
  L.elem_pi = off;      off = align256(off + 8 * size_t(ne));
  L.elem_slot = off;    off = align256(off + 36 * size_t(ne));
  L.face_rowbase = off; off = align256(off + sizeof(int64_t) * size_t(nf));
  L.face_nslots = off;  off = align256(off + sizeof(int32_t) * size_t(nf));
  L.tab_s = off;        off = align256(off + sizeof(double) * P.tab_s.size());
  L.tab_d = off;        off = align256(off + sizeof(double) * P.tab_d.size());
  L.tab_w = off;        off = align256(off + sizeof(double) * P.tab_w.size());
  L.tab_ref = off;      off = align256(off + sizeof(double) * P.tab_ref.size());
  L.tab_x = off;        off = align256(off + sizeof(double) * P.tab_x.size());
  L.tab_1d = off;       off = align256(off + sizeof(double) * P.tab_1d.size());
  L.face_selfslot = off; off = align256(off + sizeof(int32_t) * size_t(nf));
  L.face_owner = off;   off = align256(off + sizeof(int32_t) * size_t(nf));
  // per-element inputs of the RT_1 affine kernels (mesh data only)
  P.k1_geo.clear();
  P.k1_meta.clear();
  if (k == 1 && P.all_affine) {
    P.k1_geo.resize(size_t(9 * ne));
    P.k1_meta.assign(size_t(K1Meta::kBytes) * size_t(ne), 0);
    for (int64_t e = 0; e < ne; ++e) {
      const int32_t* ev = &P.e2v[size_t(8 * e)];
      const int vs[3] = {ev[1], ev[2], ev[4]};
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          P.k1_geo[size_t(9 * e + 3 * r + c)] = P.xyz[size_t(3 * vs[c] + r)] - P.xyz[size_t(3 * ev[0] + r)];
      K1Meta m{};
      for (int f = 0; f < 6; ++f) {
        const int32_t F = P.elem_face[size_t(6 * e + f)];
        m.fid[f] = F;
        m.pi[f] = P.elem_pi[size_t(8 * e + f)];
        if (F >= 0) {
          m.rb[f] = P.face_rowbase[size_t(F)];
          m.ns[f] = P.face_nslots[size_t(F)];
          if (P.face_owner[size_t(2 * F)] == e) m.own |= uint8_t(1u << f);
        }
      }
      for (int q = 0; q < 36; ++q) m.slot[q] = P.elem_slot[size_t(36 * e + q)];
      std::memcpy(&P.k1_meta[size_t(K1Meta::kBytes) * size_t(e)], &m, K1Meta::kBytes);
    }
  }
  L.k1_geo = off;       off = align256(off + sizeof(double) * P.k1_geo.size());
  L.k1_meta = off;      off = align256(off + P.k1_meta.size());
  P.face_w.assign(size_t(o.K2), 1.0);
  L.face_w = off;       off = align256(off + sizeof(double) * P.face_w.size());
  L.total = off;
  P.factor_len = int64_t(o.n) * (o.n + 1) / 2;
  return HYB_OK;
}

}  // namespace hyb
