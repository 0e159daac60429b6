// Host-side assembly of the quadrilateral Taylor-Hood pair (Q_k, Q_{k-1}) on the
// uniform n x n mesh of squares (Sec. 2, Taylor-Hood pairs; Sec. 4 also uses
// quadrilateral meshes): mesh and numbering (the Q_k nodes are the points of the
// P_k lattice of spacing 1/(k n), so the free-DoF numbering of the triangular pair
// applies unchanged), K = [A B^T; B 0] with the strain form, the right-hand side
// with Dirichlet lifting, nodal-interpolation transfers (Sec. 3, nested spaces),
// composite Vanka patches (Sec. 3.1) and the discretisation-error norms.
//
// Basis: tensor products l_a(xi) l_b(eta) of the 1D equispaced Lagrange
// polynomials of degree kk on [0, 1], evaluated in product form; node (a, b) of
// a cell with a fastest.  Quadrature: tensor Gauss-Legendre (k + 3 points per
// direction for the matrices and the load, k + 6 for the error norms).
#include <algorithm>
#include <array>
#include <cmath>

#include "vk_internal.hpp"

namespace vk {

namespace {

// l_a(t) and its derivative for a = 0..m at the point t (s = m t): prod_{c != a} (s - c) / (a - c)
void lag1d(int m, double t, double* v, double* d) {
  const double s = m * t;
  for (int a = 0; a <= m; ++a) {
    double val = 1.0, der = 0.0;
    for (int c = 0; c <= m; ++c) {
      if (c == a) continue;
      const double f = (s - c) / (a - c);
      der = der * f + val * (m / (double)(a - c));
      val *= f;
    }
    v[a] = val;
    d[a] = der;
  }
}

struct Rule2 {
  std::vector<double> x, y, w;
};

Rule2 square_rule(int q) {
  std::vector<double> g, gw;
  gauss_legendre_01(q, g, gw);
  Rule2 r;
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < q; ++i) {
      r.x.push_back(g[i]);
      r.y.push_back(g[j]);
      r.w.push_back(gw[i] * gw[j]);
    }
  return r;
}

// velocity / pressure DoFs of every square (node (a, b), a fastest)
void quad_maps(const LevelHost& L, std::vector<int>& cvd, std::vector<int>& cpd) {
  const int n = L.n, k = L.k, nbv = (k + 1) * (k + 1), nbp = k * k;
  cvd.assign((size_t)n * n * nbv * 2, 0);
  cpd.assign((size_t)n * n * nbp, 0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const int e = j * n + i;
      for (int b = 0; b <= k; ++b)
        for (int a = 0; a <= k; ++a) {
          const int G[2] = {k * i + a, k * j + b};
          for (int c = 0; c < 2; ++c) cvd[((size_t)e * nbv + b * (k + 1) + a) * 2 + c] = L.vel_dof(G, c);
        }
      for (int b = 0; b < k; ++b)
        for (int a = 0; a < k; ++a) {
          const int G[2] = {(k - 1) * i + a, (k - 1) * j + b};
          cpd[(size_t)e * nbp + b * k + a] = L.pres_dof(G);
        }
    }
}

// basis values and reference gradients of Q_kk at the rule points: (npts, (kk+1)^2)
void tensor_tables(int kk, const Rule2& r, std::vector<double>& val, std::vector<double>& gx,
                   std::vector<double>& gy) {
  const int nb = (kk + 1) * (kk + 1), nq = (int)r.w.size();
  val.assign((size_t)nq * nb, 0.0);
  gx.assign((size_t)nq * nb, 0.0);
  gy.assign((size_t)nq * nb, 0.0);
  std::vector<double> vx(kk + 1), dx(kk + 1), vy(kk + 1), dy(kk + 1);
  for (int q = 0; q < nq; ++q) {
    lag1d(kk, r.x[q], vx.data(), dx.data());
    lag1d(kk, r.y[q], vy.data(), dy.data());
    for (int b = 0; b <= kk; ++b)
      for (int a = 0; a <= kk; ++a) {
        const size_t o = (size_t)q * nb + b * (kk + 1) + a;
        val[o] = vx[a] * vy[b];
        gx[o] = dx[a] * vy[b];
        gy[o] = vx[a] * dy[b];
      }
  }
}

}  // namespace

void setup_mesh_quad(LevelHost& L) {
  const int n = L.n;
  L.cells.clear();
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) L.cells.push_back({{{i, j, 0}, {i + 1, j, 0}, {i, j + 1, 0}, {i + 1, j + 1, 0}}});
  L.unit = n;
  const int Mv = L.k * n, Mp = (L.k - 1) * n;
  L.nvel = 2 * (Mv - 1) * (Mv - 1);
  L.npres = (Mp + 1) * (Mp + 1);
  L.N = L.nvel + L.npres;
}

void build_level_quad(LevelHost& L, const Problem& pr, bool with_rhs) {
  const int k = L.k, n = L.n;
  const double nu = pr.p.viscosity, h = 1.0 / n;
  setup_mesh_quad(L);
  const int nbv = (k + 1) * (k + 1), nbp = k * k, nlv = 2 * nbv;
  std::vector<int> cvd, cpd;
  quad_maps(L, cvd, cpd);
  const int ncell = n * n;

  // pattern: the element closure without pressure-pressure pairs
  std::vector<std::vector<int>> dcells(L.N);
  for (int e = 0; e < ncell; ++e) {
    for (int j = 0; j < nlv; ++j) {
      const int d = cvd[(size_t)e * nlv + j];
      if (d >= 0) dcells[d].push_back(e);
    }
    for (int j = 0; j < nbp; ++j) dcells[cpd[(size_t)e * nbp + j]].push_back(e);
  }
  Csr& K = L.K;
  K.nrows = K.ncols = L.N;
  K.rowptr.assign(L.N + 1, 0);
  K.col.clear();
  std::vector<int> tmp;
  for (int r = 0; r < L.N; ++r) {
    tmp.clear();
    const bool rp = r >= L.nvel;
    for (int e : dcells[r]) {
      for (int j = 0; j < nlv; ++j) {
        const int d = cvd[(size_t)e * nlv + j];
        if (d >= 0) tmp.push_back(d);
      }
      if (!rp)
        for (int j = 0; j < nbp; ++j) tmp.push_back(cpd[(size_t)e * nbp + j]);
    }
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    K.col.insert(K.col.end(), tmp.begin(), tmp.end());
    K.rowptr[r + 1] = (int)K.col.size();
  }
  K.val.assign(K.col.size(), 0.0);
  dcells.clear();
  dcells.shrink_to_fit();

  // element matrices: every square is the same (Jacobian h I), computed once
  const Rule2 rule = square_rule(k + 3);
  const int nq = (int)rule.w.size();
  std::vector<double> pv, pgx, pgy, qv, qgx, qgy;
  tensor_tables(k, rule, pv, pgx, pgy);
  tensor_tables(k - 1, rule, qv, qgx, qgy);
  std::vector<double> Aloc((size_t)nlv * nlv, 0.0), Bloc((size_t)nbp * nlv, 0.0);
  std::vector<double> gxy((size_t)nbv * 2);
  for (int q = 0; q < nq; ++q) {
    const double w = rule.w[q] * h * h;
    for (int j = 0; j < nbv; ++j) {
      gxy[j * 2 + 0] = pgx[(size_t)q * nbv + j] / h;
      gxy[j * 2 + 1] = pgy[(size_t)q * nbv + j] / h;
    }
    for (int i = 0; i < nbv; ++i)
      for (int j = 0; j < nbv; ++j) {
        const double dot = gxy[i * 2] * gxy[j * 2] + gxy[i * 2 + 1] * gxy[j * 2 + 1];
        for (int c = 0; c < 2; ++c)
          for (int d = 0; d < 2; ++d) {
            double v = gxy[i * 2 + d] * gxy[j * 2 + c];
            if (c == d) v += dot;
            Aloc[(size_t)(i * 2 + c) * nlv + (j * 2 + d)] += w * nu * v;
          }
      }
    for (int p = 0; p < nbp; ++p)
      for (int j = 0; j < nbv; ++j)
        for (int d = 0; d < 2; ++d) Bloc[(size_t)p * nlv + j * 2 + d] -= w * qv[(size_t)q * nbp + p] * gxy[j * 2 + d];
  }

  auto addto = [&](int r, int c, double v) {
    const int* b = K.col.data() + K.rowptr[r];
    const int* e = K.col.data() + K.rowptr[r + 1];
    const int* it = std::lower_bound(b, e, c);
    K.val[K.rowptr[r] + (it - b)] += v;
  };
  if (with_rhs) L.b.assign(L.N, 0.0);
  std::vector<double> Floc(nlv), uD(nlv, 0.0);
  for (int e = 0; e < ncell; ++e) {
    const int ci = e % n, cj = e / n;
    const int* vd = &cvd[(size_t)e * nlv];
    const int* pd = &cpd[(size_t)e * nbp];
    if (with_rhs) {
      std::fill(Floc.begin(), Floc.end(), 0.0);
      for (int q = 0; q < nq; ++q) {
        const double w = rule.w[q] * h * h;
        const double x[3] = {(ci + rule.x[q]) * h, (cj + rule.y[q]) * h, 0.0};
        double f[3];
        field_f(pr, x, f);
        for (int i = 0; i < nbv; ++i)
          for (int c = 0; c < 2; ++c) Floc[i * 2 + c] += w * f[c] * pv[(size_t)q * nbv + i];
      }
      for (int b = 0; b <= k; ++b)
        for (int a = 0; a <= k; ++a) {
          const int j = b * (k + 1) + a;
          if (vd[j * 2] >= 0) continue;
          const double xn[3] = {(double)(k * ci + a) / (k * n), (double)(k * cj + b) / (k * n), 0.0};
          field_u(pr, xn, &uD[j * 2]);
        }
    }
    for (int a = 0; a < nlv; ++a) {
      const int r = vd[a];
      if (r < 0) continue;
      for (int c = 0; c < nlv; ++c)
        if (vd[c] >= 0) addto(r, vd[c], Aloc[(size_t)a * nlv + c]);
      for (int p = 0; p < nbp; ++p) {
        addto(r, pd[p], Bloc[(size_t)p * nlv + a]);
        addto(pd[p], r, Bloc[(size_t)p * nlv + a]);
      }
      if (with_rhs) {
        double s = Floc[a];
        for (int c = 0; c < nlv; ++c)
          if (vd[c] < 0) s -= Aloc[(size_t)a * nlv + c] * uD[c];
        L.b[r] += s;
      }
    }
    if (with_rhs)
      for (int p = 0; p < nbp; ++p) {
        double s = 0.0;
        for (int c = 0; c < nlv; ++c)
          if (vd[c] < 0) s -= Bloc[(size_t)p * nlv + c] * uD[c];
        L.b[pd[p]] += s;
      }
  }
}

// P = diag(P^V, P^Q): fine node G (spacing 1/(kk F.n) = 1/(2 kk C.n)) lies in coarse column
// G / (2 kk) (the last column for the right boundary) at local coordinate kk xi = (G - 2 kk i) / 2,
// an exact half-integer; the weight of coarse node (a, b) is l_a(xi) l_b(eta), exact zeros dropped
void build_prolongation_quad(const LevelHost& C, LevelHost& F) {
  Csr P;
  P.nrows = F.N;
  P.ncols = C.N;
  P.rowptr.assign(F.N + 1, 0);
  std::vector<std::vector<std::pair<int, double>>> rows(F.N);
  for (int part = 0; part < 2; ++part) {
    const int kk = part == 0 ? F.k : F.k - 1;
    const int M = kk * F.n;
    std::vector<double> wx(kk + 1), wy(kk + 1), dd(kk + 1);
    for (int gy = 0; gy <= M; ++gy)
      for (int gx = 0; gx <= M; ++gx) {
        const int G[2] = {gx, gy};
        int frow;
        if (part == 0) {
          frow = F.vel_dof(G, 0);
          if (frow < 0) continue;
        } else {
          frow = F.pres_dof(G);
        }
        const int ix = std::min(gx / (2 * kk), C.n - 1), iy = std::min(gy / (2 * kk), C.n - 1);
        lag1d(kk, (gx - 2 * kk * ix) / (2.0 * kk), wx.data(), dd.data());
        lag1d(kk, (gy - 2 * kk * iy) / (2.0 * kk), wy.data(), dd.data());
        for (int b = 0; b <= kk; ++b)
          for (int a = 0; a <= kk; ++a) {
            const double w = wx[a] * wy[b];
            if (w == 0.0) continue;
            const int CG[2] = {kk * ix + a, kk * iy + b};
            if (part == 0) {
              const int c0 = C.vel_dof(CG, 0);
              if (c0 < 0) continue;
              for (int c = 0; c < 2; ++c) rows[frow + c].push_back({c0 + c, w});
            } else {
              rows[frow].push_back({C.pres_dof(CG), w});
            }
          }
      }
  }
  for (int r = 0; r < F.N; ++r) {
    auto& v = rows[r];
    std::sort(v.begin(), v.end());
    for (auto& e : v) {
      P.col.push_back(e.first);
      P.val.push_back(e.second);
    }
    P.rowptr[r + 1] = (int)P.col.size();
  }
  F.P = std::move(P);
  F.PT = transpose(F.P);
}

// composite patches: vertices, edge interiors (k >= 3) and cell interiors (k >= 3) with their
// pressure DoFs and the free velocity of the closed star
void build_patches_quad(LevelHost& L, double omega, int store) {
  const int n = L.n, k = L.k, km = k - 1;
  std::vector<std::vector<int>> patches;
  auto cell_vel = [&](int i, int j, std::vector<int>& out) {
    if (i < 0 || j < 0 || i >= n || j >= n) return;
    for (int b = 0; b <= k; ++b)
      for (int a = 0; a <= k; ++a) {
        const int G[2] = {k * i + a, k * j + b};
        const int d0 = L.vel_dof(G, 0);
        if (d0 >= 0) {
          out.push_back(d0);
          out.push_back(d0 + 1);
        }
      }
  };
  auto pres = [&](int a, int b) {
    const int G[2] = {a, b};
    return L.pres_dof(G);
  };
  auto finish = [&](std::vector<int> v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    patches.push_back(std::move(v));
  };
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i <= n; ++i) {
      std::vector<int> v;
      cell_vel(i - 1, j - 1, v);
      cell_vel(i, j - 1, v);
      cell_vel(i - 1, j, v);
      cell_vel(i, j, v);
      v.push_back(pres(km * i, km * j));
      finish(std::move(v));
    }
  if (k >= 3) {
    for (int j = 0; j <= n; ++j)  // horizontal edges: column i on grid line j
      for (int i = 0; i < n; ++i) {
        std::vector<int> v;
        cell_vel(i, j - 1, v);
        cell_vel(i, j, v);
        for (int t = 1; t < km; ++t) v.push_back(pres(km * i + t, km * j));
        finish(std::move(v));
      }
    for (int j = 0; j < n; ++j)  // vertical edges: grid line i, row j
      for (int i = 0; i <= n; ++i) {
        std::vector<int> v;
        cell_vel(i - 1, j, v);
        cell_vel(i, j, v);
        for (int t = 1; t < km; ++t) v.push_back(pres(km * i, km * j + t));
        finish(std::move(v));
      }
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        std::vector<int> v;
        cell_vel(i, j, v);
        for (int b = 1; b < km; ++b)
          for (int a = 1; a < km; ++a) v.push_back(pres(km * i + a, km * j + b));
        finish(std::move(v));
      }
  }
  finalize_patches(L, patches, omega, store);
}

void solution_errors_quad(const LevelHost& L, const Problem& pr, const double* x, double* e_u, double* e_p) {
  const int k = L.k, n = L.n;
  const double h = 1.0 / n;
  const int nbv = (k + 1) * (k + 1), nbp = k * k, nlv = 2 * nbv;
  std::vector<int> cvd, cpd;
  quad_maps(L, cvd, cpd);
  const Rule2 rule = square_rule(k + 6);
  const int nq = (int)rule.w.size();
  std::vector<double> pv, pgx, pgy, qv, qgx, qgy;
  tensor_tables(k, rule, pv, pgx, pgy);
  tensor_tables(k - 1, rule, qv, qgx, qgy);
  double e1 = 0, n1 = 0, ep_int = 0, ep2 = 0, area = 0;
  std::vector<double> U(nlv), P(nbp);
  for (int e = 0; e < n * n; ++e) {
    const int ci = e % n, cj = e / n;
    const int* vd = &cvd[(size_t)e * nlv];
    const int* pd = &cpd[(size_t)e * nbp];
    for (int b = 0; b <= k; ++b)
      for (int a = 0; a <= k; ++a) {
        const int j = b * (k + 1) + a;
        if (vd[j * 2] >= 0) {
          U[j * 2] = x[vd[j * 2]];
          U[j * 2 + 1] = x[vd[j * 2 + 1]];
        } else {
          const double xn[3] = {(double)(k * ci + a) / (k * n), (double)(k * cj + b) / (k * n), 0.0};
          field_u(pr, xn, &U[j * 2]);
        }
      }
    for (int p = 0; p < nbp; ++p) P[p] = x[pd[p]];
    for (int q = 0; q < nq; ++q) {
      const double w = rule.w[q] * h * h;
      const double xq[3] = {(ci + rule.x[q]) * h, (cj + rule.y[q]) * h, 0.0};
      double uh[2] = {0, 0}, guh[4] = {0, 0, 0, 0};
      for (int j = 0; j < nbv; ++j) {
        const double v = pv[(size_t)q * nbv + j];
        const double gx = pgx[(size_t)q * nbv + j] / h, gy = pgy[(size_t)q * nbv + j] / h;
        for (int c = 0; c < 2; ++c) {
          uh[c] += U[j * 2 + c] * v;
          guh[c * 2 + 0] += U[j * 2 + c] * gx;
          guh[c * 2 + 1] += U[j * 2 + c] * gy;
        }
      }
      double ue[3], gue[9];
      field_u(pr, xq, ue);
      field_grad_u(pr, xq, gue);
      double se = 0.0, sn = 0.0;
      for (int c = 0; c < 2; ++c) {
        se += (ue[c] - uh[c]) * (ue[c] - uh[c]);
        sn += ue[c] * ue[c];
        for (int d = 0; d < 2; ++d) {
          se += (gue[c * 2 + d] - guh[c * 2 + d]) * (gue[c * 2 + d] - guh[c * 2 + d]);
          sn += gue[c * 2 + d] * gue[c * 2 + d];
        }
      }
      e1 += w * se;
      n1 += w * sn;
      double ph = 0.0;
      for (int p = 0; p < nbp; ++p) ph += P[p] * qv[(size_t)q * nbp + p];
      const double dp = 0.0 - ph;
      ep_int += w * dp;
      ep2 += w * dp * dp;
      area += w;
    }
  }
  const double mean = ep_int / area;
  *e_u = std::sqrt(e1 / n1);
  *e_p = std::sqrt(std::max(ep2 - 2.0 * mean * ep_int + mean * mean * area, 0.0));
}

}  // namespace vk
