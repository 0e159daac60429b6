// Scott-Vogelius (P_k, dP_{k-1}) levels on barycentric refinements (the
// pair of Sec. 2 that is inf-sup stable on such meshes in 2D): sub-cell
// mesh and numbering, macro-element patches, and the transfers between the
// non-nested levels.
//
// Sub-cells.  Macro triangle m = (v0, v1, v2) of the n x n mesh (two
// triangles per square, top-left to bottom-right diagonal, in the order of
// the Taylor-Hood cells) with barycentre c gives sub-cells 3m + s with
// vertices (v_s, v_{s+1}, c).  Vertex coordinates are integers in units of
// 1/(3n); P_k nodes are on the lattice of spacing 1/(3kn).
//
// Transfers.  Uniform refinement of the macro mesh is nested but the
// barycentric sub-cells are not (a fine sub-cell can cross a coarse split
// line).  Velocity (continuous): nodal interpolation, the coarse sub-cell
// found by exact integer barycentric tests.  Pressure (discontinuous): the
// L^2 projection onto each fine sub-cell, which for nested spaces is the
// natural embedding; the fine sub-cell is clipped against each coarse
// sub-cell it overlaps and the pieces are integrated exactly.
#include <algorithm>
#include <cmath>

#include "vk_internal.hpp"

namespace vk {

namespace {

// position of node (a1, a2) in the lexicographic order of {a1 + a2 <= km}, a1 slower
inline int sv_local(int a1, int a2, int km) {
  int idx = 0;
  for (int b = 0; b < a1; ++b) idx += km - b + 1;
  return idx + a2;
}

inline void lattice_point(const Cell& c, const std::vector<int>& a, int* G) {
  for (int d = 0; d < 2; ++d) G[d] = a[0] * c.v[0][d] + a[1] * c.v[1][d] + a[2] * c.v[2][d];
}

}  // namespace

int LevelHost::sv_pres_dof(int e, int a1, int a2) const {
  const int km = k - 1;
  const int nbp = (km + 1) * (km + 2) / 2;
  return nvel + e * nbp + sv_local(a1, a2, km);
}

void setup_mesh_sv(LevelHost& L) {
  require(L.dim == 2, VK_EINVAL, "Scott-Vogelius levels are 2D");
  const int n = L.n, k = L.k;
  L.unit = 3 * n;
  L.cells.clear();
  auto add_macro = [&](const int (&t)[3][2]) {
    const int cx = t[0][0] + t[1][0] + t[2][0], cy = t[0][1] + t[1][1] + t[2][1];
    for (int s = 0; s < 3; ++s) {
      const int a = s, b = (s + 1) % 3;
      Cell c = {{{3 * t[a][0], 3 * t[a][1], 0}, {3 * t[b][0], 3 * t[b][1], 0}, {cx, cy, 0}, {0, 0, 0}}};
      L.cells.push_back(c);
    }
  };
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const int lo[3][2] = {{i, j}, {i + 1, j}, {i, j + 1}};
      const int up[3][2] = {{i + 1, j + 1}, {i, j + 1}, {i + 1, j}};
      add_macro(lo);
      add_macro(up);
    }
  const int M = k * L.unit;
  const Basis vb = make_basis(2, k);
  L.vmap.assign((size_t)(M + 1) * (M + 1), -1);
  for (const Cell& c : L.cells)
    for (const auto& a : vb.nodes) {
      int G[2];
      lattice_point(c, a, G);
      L.vmap[(size_t)G[1] * (M + 1) + G[0]] = -2;
    }
  int idx = 0;
  for (int y = 0; y <= M; ++y)
    for (int x = 0; x <= M; ++x) {
      int& v = L.vmap[(size_t)y * (M + 1) + x];
      v = (v == -2 && x > 0 && y > 0 && x < M && y < M) ? idx++ : -1;
    }
  const int nbp = k * (k + 1) / 2;
  L.nvel = 2 * idx;
  L.npres = (int)L.cells.size() * nbp;
  L.N = L.nvel + L.npres;
}

void dof_coords_sv(const LevelHost& L, double* xyz, int* kind) {
  const int M = L.k * L.unit, km = L.k - 1;
  for (int y = 0; y <= M; ++y)
    for (int x = 0; x <= M; ++x) {
      const int id = L.vmap[(size_t)y * (M + 1) + x];
      if (id < 0) continue;
      for (int c = 0; c < 2; ++c) {
        xyz[(size_t)(2 * id + c) * 2 + 0] = (double)x / M;
        xyz[(size_t)(2 * id + c) * 2 + 1] = (double)y / M;
        kind[2 * id + c] = c;
      }
    }
  const Basis pb = make_basis(2, km);
  for (int e = 0; e < (int)L.cells.size(); ++e)
    for (const auto& a : pb.nodes) {
      int G[2];
      lattice_point(L.cells[e], a, G);
      const int d = L.sv_pres_dof(e, a[1], a[2]);
      xyz[(size_t)d * 2 + 0] = (double)G[0] / (km * L.unit);
      xyz[(size_t)d * 2 + 1] = (double)G[1] / (km * L.unit);
      kind[d] = 2;
    }
}

void build_patches_macro(LevelHost& L, double omega, int store) {
  const Basis vb = make_basis(2, L.k);
  const int nbp = L.k * (L.k + 1) / 2;
  const int nmacro = (int)L.cells.size() / 3;
  std::vector<std::vector<int>> patches(nmacro);
  for (int m = 0; m < nmacro; ++m) {
    std::vector<int>& v = patches[m];
    for (int e = 3 * m; e < 3 * m + 3; ++e) {
      for (const auto& a : vb.nodes) {
        int G[2];
        lattice_point(L.cells[e], a, G);
        const int d0 = L.vel_dof(G, 0);
        if (d0 < 0) continue;
        v.push_back(d0);
        v.push_back(d0 + 1);
      }
      for (int t = 0; t < nbp; ++t) v.push_back(L.nvel + e * nbp + t);
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  finalize_patches(L, patches, omega, store);
}

// ---------------------------------------------------------------- transfers
namespace {

typedef long long i64;

// twice the signed area of (a, b, p)
inline i64 orient(const i64* a, const i64* b, const i64* p) {
  return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0]);
}

struct Pt {
  double x, y;
};

// part of the convex polygon P on the left of (or on) the directed line a -> b, times sgn
void clip_half(const std::vector<Pt>& P, Pt a, Pt b, double sgn, std::vector<Pt>& out) {
  out.clear();
  const size_t m = P.size();
  auto side = [&](const Pt& p) { return sgn * ((b.x - a.x) * (p.y - a.y) - (b.y - a.y) * (p.x - a.x)); };
  for (size_t i = 0; i < m; ++i) {
    const Pt& p = P[i];
    const Pt& q = P[(i + 1) % m];
    const double sp = side(p), sq = side(q);
    if (sp >= 0) out.push_back(p);
    if ((sp >= 0) != (sq >= 0)) {
      const double t = sp / (sp - sq);
      out.push_back({p.x + t * (q.x - p.x), p.y + t * (q.y - p.y)});
    }
  }
}

double poly_area(const std::vector<Pt>& P) {
  double s = 0.0;
  for (size_t i = 0; i < P.size(); ++i) {
    const Pt& p = P[i];
    const Pt& q = P[(i + 1) % P.size()];
    s += p.x * q.y - q.x * p.y;
  }
  return 0.5 * std::fabs(s);
}

// barycentric coordinates of x in the triangle T (physical coordinates)
void bary(const Pt* T, Pt x, double* lam) {
  const double d = (T[1].x - T[0].x) * (T[2].y - T[0].y) - (T[2].x - T[0].x) * (T[1].y - T[0].y);
  lam[1] = ((x.x - T[0].x) * (T[2].y - T[0].y) - (T[2].x - T[0].x) * (x.y - T[0].y)) / d;
  lam[2] = ((T[1].x - T[0].x) * (x.y - T[0].y) - (x.x - T[0].x) * (T[1].y - T[0].y)) / d;
  lam[0] = 1.0 - lam[1] - lam[2];
}

void cell_pts(const LevelHost& L, int e, Pt* T) {
  for (int i = 0; i < 3; ++i) T[i] = {(double)L.cells[e].v[i][0] / L.unit, (double)L.cells[e].v[i][1] / L.unit};
}

// solve the small dense system A X = B (A: m x m, B: m x r, row-major) by Gaussian elimination with pivoting
void small_solve(std::vector<double> A, std::vector<double>& B, int m, int r) {
  for (int c = 0; c < m; ++c) {
    int p = c;
    for (int i = c + 1; i < m; ++i)
      if (std::fabs(A[(size_t)i * m + c]) > std::fabs(A[(size_t)p * m + c])) p = i;
    if (p != c) {
      for (int j = 0; j < m; ++j) std::swap(A[(size_t)c * m + j], A[(size_t)p * m + j]);
      for (int j = 0; j < r; ++j) std::swap(B[(size_t)c * r + j], B[(size_t)p * r + j]);
    }
    for (int i = c + 1; i < m; ++i) {
      const double f = A[(size_t)i * m + c] / A[(size_t)c * m + c];
      for (int j = c; j < m; ++j) A[(size_t)i * m + j] -= f * A[(size_t)c * m + j];
      for (int j = 0; j < r; ++j) B[(size_t)i * r + j] -= f * B[(size_t)c * r + j];
    }
  }
  for (int c = m - 1; c >= 0; --c)
    for (int j = 0; j < r; ++j) {
      double s = B[(size_t)c * r + j];
      for (int i = c + 1; i < m; ++i) s -= A[(size_t)c * m + i] * B[(size_t)i * r + j];
      B[(size_t)c * r + j] = s / A[(size_t)c * m + c];
    }
}

}  // namespace

void build_prolongation_sv(const LevelHost& C, LevelHost& F) {
  require(F.n == 2 * C.n && F.k == C.k, VK_EINVAL, "levels must be one uniform refinement apart");
  const int k = F.k, km = k - 1, nc = C.n;
  const int nbp = k * (k + 1) / 2;
  std::vector<std::vector<std::pair<int, double>>> rows(F.N);

  // ---- velocity: fine node G in units 1/(6 k nc); coarse vertices (units 1/(3 nc)) scaled by 2k
  {
    const Basis vb = make_basis(2, k);
    const int span = 6 * k;  // fine lattice steps per coarse square
    const int Mf = k * F.unit;
    std::vector<double> phi(vb.size());
    for (int y = 0; y <= Mf; ++y)
      for (int x = 0; x <= Mf; ++x) {
        const int id = F.vmap[(size_t)y * (Mf + 1) + x];
        if (id < 0) continue;
        int ci[2], cn = 0, cj[2], cm = 0;
        for (int t = x / span - (x % span == 0); t <= x / span; ++t)
          if (t >= 0 && t < nc) ci[cn++] = t;
        for (int t = y / span - (y % span == 0); t <= y / span; ++t)
          if (t >= 0 && t < nc) cj[cm++] = t;
        std::vector<int> cand;
        for (int a = 0; a < cn; ++a)
          for (int b = 0; b < cm; ++b)
            for (int s = 0; s < 6; ++s) cand.push_back(6 * (cj[b] * nc + ci[a]) + s);
        std::sort(cand.begin(), cand.end());
        const i64 P[2] = {x, y};
        int hit = -1;
        i64 num[3] = {0, 0, 0}, den = 1;
        for (int cc : cand) {
          i64 V[3][2];
          for (int i = 0; i < 3; ++i)
            for (int d = 0; d < 2; ++d) V[i][d] = (i64)C.cells[cc].v[i][d] * 2 * k;
          den = orient(V[0], V[1], V[2]);
          num[0] = orient(V[1], V[2], P);
          num[1] = orient(V[2], V[0], P);
          num[2] = orient(V[0], V[1], P);
          const i64 sg = den > 0 ? 1 : -1;
          if (sg * num[0] >= 0 && sg * num[1] >= 0 && sg * num[2] >= 0) {
            hit = cc;
            break;
          }
        }
        require(hit >= 0, VK_EINVAL, "fine velocity node outside the coarse mesh");
        double klam[3];
        for (int i = 0; i < 3; ++i) klam[i] = (double)(k * num[i]) / (double)den;
        vb.eval(klam, phi.data());
        for (int j = 0; j < vb.size(); ++j) {
          if (phi[j] == 0.0) continue;
          int CG[2];
          lattice_point(C.cells[hit], vb.nodes[j], CG);
          const int c0 = C.vel_dof(CG, 0);
          if (c0 < 0) continue;
          rows[2 * id].push_back({c0, phi[j]});
          rows[2 * id + 1].push_back({c0 + 1, phi[j]});
        }
      }
  }

  // ---- pressure: local L^2 projection
  {
    const Basis pb = make_basis(2, km);
    const SimplexRule rule = simplex_rule(2, k + 1);
    const int nq = rule.npts;
    std::vector<double> ef(nbp), ec(nbp);
    std::vector<Pt> poly, tmp;
    for (int fe = 0; fe < (int)F.cells.size(); ++fe) {
      Pt Tf[3];
      cell_pts(F, fe, Tf);
      const double areaf = 0.5 * std::fabs((Tf[1].x - Tf[0].x) * (Tf[2].y - Tf[0].y) -
                                           (Tf[2].x - Tf[0].x) * (Tf[1].y - Tf[0].y));
      // the fine macro triangle lies in one coarse macro triangle: the coarse square of its centroid
      const double cx = (Tf[0].x + Tf[1].x + Tf[2].x) / 3.0, cy = (Tf[0].y + Tf[1].y + Tf[2].y) / 3.0;
      const int si = std::min(nc - 1, (int)std::floor(cx * nc)), sj = std::min(nc - 1, (int)std::floor(cy * nc));
      // fine mass matrix
      std::vector<double> Mf((size_t)nbp * nbp, 0.0);
      for (int q = 0; q < nq; ++q) {
        double kl[3];
        for (int i = 0; i < 3; ++i) kl[i] = km * rule.lam[q * 3 + i];
        pb.eval(kl, ef.data());
        const double w = rule.w[q] * 2.0 * areaf;
        for (int a = 0; a < nbp; ++a)
          for (int b = 0; b < nbp; ++b) Mf[(size_t)a * nbp + b] += w * ef[a] * ef[b];
      }
      std::vector<int> hits;
      std::vector<double> G;  // nbp x (nbp * hits)
      std::vector<std::vector<double>> Gc;
      for (int s = 0; s < 6; ++s) {
        const int cc = 6 * (sj * nc + si) + s;
        Pt Tc[3];
        cell_pts(C, cc, Tc);
        const double dc = (Tc[1].x - Tc[0].x) * (Tc[2].y - Tc[0].y) - (Tc[2].x - Tc[0].x) * (Tc[1].y - Tc[0].y);
        const double sgn = dc > 0 ? 1.0 : -1.0;
        poly.assign(Tf, Tf + 3);
        for (int e = 0; e < 3 && !poly.empty(); ++e) {
          clip_half(poly, Tc[e], Tc[(e + 1) % 3], sgn, tmp);
          poly.swap(tmp);
        }
        if (poly.size() < 3 || poly_area(poly) <= 1e-10 * areaf) continue;
        std::vector<double> g((size_t)nbp * nbp, 0.0);
        for (size_t t = 1; t + 1 < poly.size(); ++t) {
          const Pt a = poly[0], b = poly[t], c = poly[t + 1];
          const double det = std::fabs((b.x - a.x) * (c.y - a.y) - (c.x - a.x) * (b.y - a.y));
          for (int q = 0; q < nq; ++q) {
            const double* l = &rule.lam[q * 3];
            const Pt X = {l[0] * a.x + l[1] * b.x + l[2] * c.x, l[0] * a.y + l[1] * b.y + l[2] * c.y};
            double lf[3], lc[3];
            bary(Tf, X, lf);
            bary(Tc, X, lc);
            for (int i = 0; i < 3; ++i) {
              lf[i] *= km;
              lc[i] *= km;
            }
            pb.eval(lf, ef.data());
            pb.eval(lc, ec.data());
            const double w = rule.w[q] * det;
            for (int i = 0; i < nbp; ++i)
              for (int j = 0; j < nbp; ++j) g[(size_t)i * nbp + j] += w * ef[i] * ec[j];
          }
        }
        hits.push_back(cc);
        Gc.push_back(std::move(g));
      }
      require(!hits.empty(), VK_EINVAL, "fine sub-cell overlaps no coarse sub-cell");
      const int r = nbp * (int)hits.size();
      G.assign((size_t)nbp * r, 0.0);
      for (size_t h = 0; h < hits.size(); ++h)
        for (int i = 0; i < nbp; ++i)
          for (int j = 0; j < nbp; ++j) G[(size_t)i * r + h * nbp + j] = Gc[h][(size_t)i * nbp + j];
      small_solve(Mf, G, nbp, r);
      for (int i = 0; i < nbp; ++i) {
        const auto& ai = pb.nodes[i];
        const int frow = F.sv_pres_dof(fe, ai[1], ai[2]);
        for (size_t h = 0; h < hits.size(); ++h)
          for (int j = 0; j < nbp; ++j) {
            const auto& aj = pb.nodes[j];
            rows[frow].push_back({C.sv_pres_dof(hits[h], aj[1], aj[2]), G[(size_t)i * r + h * nbp + j]});
          }
      }
    }
  }

  Csr P;
  P.nrows = F.N;
  P.ncols = C.N;
  P.rowptr.assign(F.N + 1, 0);
  for (int r = 0; r < F.N; ++r) {
    auto& v = rows[r];
    std::sort(v.begin(), v.end(), [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
      return a.first < b.first;
    });
    for (auto& e : v) {
      P.col.push_back(e.first);
      P.val.push_back(e.second);
    }
    P.rowptr[r + 1] = (int)P.col.size();
  }
  F.P = std::move(P);
  F.PT = transpose(F.P);
}

}  // namespace vk
