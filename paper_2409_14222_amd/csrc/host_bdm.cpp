// Host-side assembly of (BDM_k, dP_{k-1}) with the symmetric interior-penalty form on the
// two-triangle mesh of the unit square (Sec. 2, the H(div)-L2 formulation and the bilinear
// form labelled DiscontBilinearForm; Case 3 of Sec. 3): mesh, DoF numbering, K, the
// right-hand side, the natural-embedding transfers (Sec. 3, grid transfers), the extended
// cell Vanka patches (Sec. 3.1) and the discretisation-error norms.
//
// Velocity DoFs of a cell T (a dual basis): for each edge e = (a, b), a the endpoint with
// the smaller vertex index y (n + 1) + x, t = (b - a) / |b - a| and n_e = (t_y, -t_x),
// the normal moments |e|^{-1} int_e (v.n_e) L_j(s) ds, j = 0..k, L_j the Legendre
// polynomial shifted to s in [0, 1] (s = 0 at a); in the interior the moments
// |T|^{-1} int_T v.q for an orthonormal basis of the first-kind Nedelec space
// ND_{k-1} = [P_{k-2}]^2 + x^perp P~_{k-2}: classical Gram-Schmidt (two passes), in order,
// of e_0 l_a, e_1 l_a (l_a the nodal P_{k-2} basis of the cell, the constant for k = 2)
// and (-xi_2, xi_1) l_a for the nodes a on the edge opposite the first vertex,
// xi = n (x - x_c) with x_c the centroid.  Moments against all of P_k(e) fix v.n on e, so
// the cell-wise dual bases glue into an H(div) basis; v.n = 0 on the boundary is imposed by
// dropping the boundary edge moments.  Pressure: nodal P_{k-1} per cell (a constant for k = 1).
//
// With t the unit tangent of an interior edge and n1 the unit normal out of T1, the
// tangential jump of a normal-continuous field is ((v1 - v2).t) t (.) n1, so the edge terms
// of a_h are -2 nu int [(t^T {eps(u)} n1) [v_t] + [u_t] (t^T {eps(v)} n1)] + nu alpha h_e^{-1}
// int [u_t] [v_t] with [v_t] = (v1 - v2).t ((t (.) n1):(t (.) n1) = 1/2).  Boundary edges
// carry no terms (v.n = 0 strongly, tangential stress zero naturally).
//
// Numbering: interior edges in ascending (index(a), index(b)) order with their k + 1 moments,
// then the cells (lower triangle of square (i, j) at 2 (j n + i), the upper one next) with
// their k^2 - 1 interior moments; the pressure follows cell by cell.
//
// Every cell of one orientation is a translate of every other with the same local edge
// orientations, so the dual basis, the volume matrices, the edge matrices and the transfer
// blocks are computed once per configuration and reused.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "vk_internal.hpp"

namespace vk {

namespace {

struct Tri {
  int v[3][2];  // vertex lattice points, units 1/n
};

inline Tri tri_of(int n, int c) {
  const int sq = c / 2, i = sq % n, j = sq / n;
  if (c % 2 == 0) return {{{i, j}, {i + 1, j}, {i, j + 1}}};
  return {{{i + 1, j + 1}, {i, j + 1}, {i + 1, j}}};
}

inline int vid(int n, const int* G) { return G[1] * (n + 1) + G[0]; }

struct Geom {
  double v0[2], J[2][2], Ji[2][2], det;  // x = v0 + J xh, J[:, d] = V_{d+1} - V_0
  double gl[3][2];                       // gradients of the barycentric coordinates
  Geom(const Tri& t, double h) {
    for (int d = 0; d < 2; ++d) {
      v0[d] = t.v[0][d] * h;
      J[d][0] = (t.v[1][d] - t.v[0][d]) * h;
      J[d][1] = (t.v[2][d] - t.v[0][d]) * h;
    }
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
    for (int d = 0; d < 2; ++d) {
      gl[1][d] = Ji[0][d];
      gl[2][d] = Ji[1][d];
      gl[0][d] = -Ji[0][d] - Ji[1][d];
    }
  }
  void bary(const double* x, double* lam) const {
    const double r0 = x[0] - v0[0], r1 = x[1] - v0[1];
    lam[1] = Ji[0][0] * r0 + Ji[0][1] * r1;
    lam[2] = Ji[1][0] * r0 + Ji[1][1] * r1;
    lam[0] = 1.0 - lam[1] - lam[2];
  }
  void point(const double* lam, double* x) const {
    for (int d = 0; d < 2; ++d) x[d] = v0[d] + J[d][0] * lam[1] + J[d][1] * lam[2];
  }
};

// shifted Legendre L_0..L_m at s in [0, 1]
void legendre01(int m, double s, double* L) {
  const double t = 2.0 * s - 1.0;
  L[0] = 1.0;
  if (m >= 1) L[1] = t;
  for (int j = 1; j < m; ++j) L[j + 1] = ((2 * j + 1) * t * L[j] - j * L[j - 1]) / (j + 1);
}

// dense inverse by Gauss-Jordan elimination with partial pivoting (row-major, n x n)
std::vector<double> dense_inverse(std::vector<double> a, int n) {
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)p * n + c])) p = r;
    require(a[(size_t)p * n + c] != 0.0, VK_ESINGULAR, "singular BDM dual-basis matrix");
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)p * n + j], a[(size_t)c * n + j]);
        std::swap(inv[(size_t)p * n + j], inv[(size_t)c * n + j]);
      }
    const double d = 1.0 / a[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) {
      a[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
      }
    }
  }
  return inv;
}

// The finite-element space of one level: local spaces, dual bases (per cell orientation),
// edges and DoF maps.
struct Space {
  int k = 0, n = 0, nb = 0, nloc = 0, ne = 0, ni = 0, nbp = 0, ncell = 0;
  double h = 0.0;
  Basis vb, tb, pb;  // P_k (local space), P_{k-2} (interior tests, k >= 3), P_{k-1} (pressure, k >= 2)
  std::vector<double> C[2];  // dual basis of each orientation: phi_i = sum_m C[m nloc + i] psi_m
  std::vector<double> T[2];  // orthonormal interior tests: q'_i = sum_j T[i ni + j] q_j
  // edges: cell c has local edges (v0 v1), (v1 v2), (v0 v2)
  std::vector<std::array<int, 2>> ekey;   // (index(a), index(b)) of every distinct edge
  std::vector<std::array<int, 2>> ecells; // the one or two cells of each edge (-1 if one)
  std::vector<std::array<int, 3>> cedge;  // edge id of each local edge
  std::vector<int> erank;                 // interior rank or -1
  int nint = 0, nvel = 0, N = 0;

  void init(int k_, int n_) {
    k = k_;
    n = n_;
    h = 1.0 / n;
    vb = make_basis(2, k);
    if (k >= 3) tb = make_basis(2, k - 2);
    if (k >= 2) pb = make_basis(2, k - 1);
    nb = vb.size();
    nloc = 2 * nb;
    ne = k + 1;
    ni = k * k - 1;
    nbp = k * (k + 1) / 2;
    ncell = 2 * n * n;
    // edges
    std::map<std::array<int, 2>, int> id;
    cedge.assign(ncell, {0, 0, 0});
    for (int c = 0; c < ncell; ++c) {
      const Tri t = tri_of(n, c);
      const int le[3][2] = {{0, 1}, {1, 2}, {0, 2}};
      for (int l = 0; l < 3; ++l) {
        int a = vid(n, t.v[le[l][0]]), b = vid(n, t.v[le[l][1]]);
        if (a > b) std::swap(a, b);
        const std::array<int, 2> key{a, b};
        auto it = id.find(key);
        int e;
        if (it == id.end()) {
          e = (int)ekey.size();
          id.emplace(key, e);
          ekey.push_back(key);
          ecells.push_back({c, -1});
        } else {
          e = it->second;
          ecells[e][1] = c;
        }
        cedge[c][l] = e;
      }
    }
    // interior ranks in ascending key order (std::map iterates sorted)
    erank.assign(ekey.size(), -1);
    nint = 0;
    for (auto& kv : id)
      if (ecells[kv.second][1] >= 0) erank[kv.second] = nint++;
    nvel = nint * ne + ncell * ni;
    N = nvel + ncell * nbp;
    for (int s = 0; s < 2; ++s) build_dual(s);
  }

  Tri cell(int c) const { return tri_of(n, c); }
  Geom geom(int c) const { return Geom(cell(c), h); }

  // endpoints (physical), length, tangent and normal of edge e
  void edge_frame(int e, double* a, double* b, double& len, double* t, double* nrm) const {
    for (int d = 0; d < 2; ++d) {
      a[d] = (d == 0 ? ekey[e][0] % (n + 1) : ekey[e][0] / (n + 1)) * h;
      b[d] = (d == 0 ? ekey[e][1] % (n + 1) : ekey[e][1] / (n + 1)) * h;
    }
    len = std::hypot(b[0] - a[0], b[1] - a[1]);
    t[0] = (b[0] - a[0]) / len;
    t[1] = (b[1] - a[1]) / len;
    nrm[0] = t[1];
    nrm[1] = -t[0];
  }

  // global velocity DoF (or -1) of each local function of cell c
  void cell_vel(int c, int* out) const {
    for (int l = 0; l < 3; ++l) {
      const int r = erank[cedge[c][l]];
      for (int j = 0; j < ne; ++j) out[l * ne + j] = r >= 0 ? r * ne + j : -1;
    }
    for (int m = 0; m < ni; ++m) out[3 * ne + m] = nint * ne + c * ni + m;
  }
  int pres0(int c) const { return nvel + c * nbp; }

  // local space [P_k]^2 at x: values pv[m * 2 + d] and gradients pg[(m * 2 + c) * 2 + d], m = j 2 + c
  void psi(const Geom& g, const double* x, double* pv, double* pg) const {
    double lam[3], klam[3];
    g.bary(x, lam);
    for (int i = 0; i < 3; ++i) klam[i] = k * lam[i];
    std::vector<double> l(nb), dl((size_t)nb * 3);
    vb.eval(klam, l.data());
    vb.dlam(lam, dl.data());
    for (int j = 0; j < nb; ++j) {
      double gx[2];
      for (int d = 0; d < 2; ++d)
        gx[d] = dl[j * 3 + 0] * g.gl[0][d] + dl[j * 3 + 1] * g.gl[1][d] + dl[j * 3 + 2] * g.gl[2][d];
      for (int c = 0; c < 2; ++c) {
        const int m = j * 2 + c;
        for (int d = 0; d < 2; ++d) {
          pv[m * 2 + d] = c == d ? l[j] : 0.0;
          for (int c2 = 0; c2 < 2; ++c2) pg[(m * 2 + c2) * 2 + d] = c2 == c ? gx[d] : 0.0;
        }
      }
    }
  }

  // dual basis of orientation s at x: values v[i * 2 + c], gradients gr[(i * 2 + c) * 2 + d]
  void phi(int s, const Geom& g, const double* x, double* v, double* gr) const {
    std::vector<double> pv((size_t)nloc * 2), pg((size_t)nloc * 4);
    psi(g, x, pv.data(), pg.data());
    const double* Cs = C[s].data();
    std::fill(v, v + (size_t)nloc * 2, 0.0);
    if (gr) std::fill(gr, gr + (size_t)nloc * 4, 0.0);
    for (int m = 0; m < nloc; ++m) {
      const int c = m & 1;
      const double pvm = pv[m * 2 + c];
      const double g0 = pg[(m * 2 + c) * 2 + 0], g1 = pg[(m * 2 + c) * 2 + 1];
      const double* row = Cs + (size_t)m * nloc;
      for (int i = 0; i < nloc; ++i) {
        const double w = row[i];
        if (w == 0.0) continue;
        v[i * 2 + c] += w * pvm;
        if (gr) {
          gr[(i * 2 + c) * 2 + 0] += w * g0;
          gr[(i * 2 + c) * 2 + 1] += w * g1;
        }
      }
    }
  }

  // raw interior tests q_j at the point with barycentric lam / physical x (xc the centroid)
  void raw_tests(const double* lam, const double* x, const double* xc, double* q) const {
    const int nt = k >= 2 ? k * (k - 1) / 2 : 0;  // dim P_{k-2}
    if (nt == 0) return;
    std::vector<double> l(nt, 1.0);
    if (k >= 3) {
      double klam[3];
      for (int i = 0; i < 3; ++i) klam[i] = (k - 2) * lam[i];
      tb.eval(klam, l.data());
    }
    const double xi0 = n * (x[0] - xc[0]), xi1 = n * (x[1] - xc[1]);
    int j = 0;
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < nt; ++a, ++j) {
        q[j * 2 + 0] = c == 0 ? l[a] : 0.0;
        q[j * 2 + 1] = c == 1 ? l[a] : 0.0;
      }
    for (int a = 0; a < nt; ++a) {
      const bool on_edge = k == 2 || tb.nodes[a][0] == 0;  // lambda_0 = 0: a_1 + a_2 = k - 2
      if (!on_edge) continue;
      q[j * 2 + 0] = -xi1 * l[a];
      q[j * 2 + 1] = xi0 * l[a];
      ++j;
    }
  }

  // orthonormal interior tests of a cell with geometry g and orientation s at the points of the
  // collapsed rule with k + 2 points: physical points xs, weights ws of |T|^{-1} int_T, values qs
  void interior_tests(int s, const Geom& g, std::vector<double>& xs, std::vector<double>& ws,
                      std::vector<double>& qs) const {
    const SimplexRule r = simplex_rule(2, k + 2);
    const int np = r.npts;
    xs.resize((size_t)np * 2);
    ws.resize(np);
    qs.assign((size_t)np * ni * 2, 0.0);
    if (ni == 0) return;
    double xc[2];
    const double third[3] = {1.0 / 3, 1.0 / 3, 1.0 / 3};
    g.point(third, xc);
    std::vector<double> raw((size_t)np * ni * 2);
    for (int p = 0; p < np; ++p) {
      g.point(&r.lam[p * 3], &xs[p * 2]);
      ws[p] = 2.0 * r.w[p];
      raw_tests(&r.lam[p * 3], &xs[p * 2], xc, &raw[(size_t)p * ni * 2]);
    }
    const std::vector<double>& Ts = T[s];
    for (int p = 0; p < np; ++p)
      for (int i = 0; i < ni; ++i)
        for (int c = 0; c < 2; ++c) {
          double v = 0.0;
          for (int j = 0; j <= i; ++j) v += Ts[(size_t)i * ni + j] * raw[((size_t)p * ni + j) * 2 + c];
          qs[((size_t)p * ni + i) * 2 + c] = v;
        }
  }

  void build_dual(int s) {
    const int c0 = s;  // cell 0 (lower) or 1 (upper) of square (0, 0)
    const Geom g = geom(c0);
    // Gram-Schmidt coefficients of the interior tests
    T[s].assign((size_t)ni * ni, 0.0);
    if (ni > 0) {
      const SimplexRule r = simplex_rule(2, k + 2);
      const int np = r.npts;
      double xc[2];
      const double third[3] = {1.0 / 3, 1.0 / 3, 1.0 / 3};
      g.point(third, xc);
      std::vector<double> raw((size_t)np * ni * 2), w(np);
      for (int p = 0; p < np; ++p) {
        double x[2];
        g.point(&r.lam[p * 3], x);
        w[p] = 2.0 * r.w[p];
        raw_tests(&r.lam[p * 3], x, xc, &raw[(size_t)p * ni * 2]);
      }
      // classical Gram-Schmidt, two passes, on the values at the rule points
      std::vector<double> done((size_t)ni * np * 2), cur((size_t)np * 2), dots(ni), cvec(ni);
      for (int i = 0; i < ni; ++i) {
        std::fill(cvec.begin(), cvec.end(), 0.0);
        cvec[i] = 1.0;
        for (int p = 0; p < np; ++p)
          for (int c = 0; c < 2; ++c) cur[p * 2 + c] = raw[((size_t)p * ni + i) * 2 + c];
        for (int pass = 0; pass < 2; ++pass) {
          for (int j = 0; j < i; ++j) {
            double sum = 0.0;
            const double* dj = &done[(size_t)j * np * 2];
            for (int p = 0; p < np; ++p) sum += w[p] * (cur[p * 2] * dj[p * 2] + cur[p * 2 + 1] * dj[p * 2 + 1]);
            dots[j] = sum;
          }
          for (int j = 0; j < i; ++j) {
            const double* dj = &done[(size_t)j * np * 2];
            for (int p = 0; p < 2 * np; ++p) cur[p] -= dots[j] * dj[p];
            for (int m = 0; m < ni; ++m) cvec[m] -= dots[j] * T[s][(size_t)j * ni + m];
          }
        }
        double nn = 0.0;
        for (int p = 0; p < np; ++p) nn += w[p] * (cur[p * 2] * cur[p * 2] + cur[p * 2 + 1] * cur[p * 2 + 1]);
        const double nr = std::sqrt(nn);
        for (int m = 0; m < ni; ++m) T[s][(size_t)i * ni + m] = cvec[m] / nr;
        for (int p = 0; p < 2 * np; ++p) done[(size_t)i * np * 2 + p] = cur[p] / nr;
      }
    }
    // D[r][m]: functional r applied to psi_m
    std::vector<double> D((size_t)nloc * nloc, 0.0);
    std::vector<double> pv((size_t)nloc * 2), pg((size_t)nloc * 4), L(ne);
    std::vector<double> gq, gw;
    gauss_legendre_01(k + 2, gq, gw);
    for (int l = 0; l < 3; ++l) {
      double a[2], b[2], len, t[2], nr[2];
      edge_frame(cedge[c0][l], a, b, len, t, nr);
      for (size_t q = 0; q < gq.size(); ++q) {
        const double x[2] = {a[0] + gq[q] * (b[0] - a[0]), a[1] + gq[q] * (b[1] - a[1])};
        psi(g, x, pv.data(), pg.data());
        legendre01(k, gq[q], L.data());
        for (int j = 0; j < ne; ++j)
          for (int m = 0; m < nloc; ++m)
            D[(size_t)(l * ne + j) * nloc + m] += gw[q] * L[j] * (pv[m * 2] * nr[0] + pv[m * 2 + 1] * nr[1]);
      }
    }
    if (ni > 0) {
      std::vector<double> xs, ws, qs;
      interior_tests(s, g, xs, ws, qs);
      for (size_t p = 0; p < ws.size(); ++p) {
        psi(g, &xs[p * 2], pv.data(), pg.data());
        for (int i = 0; i < ni; ++i)
          for (int m = 0; m < nloc; ++m)
            D[(size_t)(3 * ne + i) * nloc + m] +=
                ws[p] * (qs[(p * ni + i) * 2] * pv[m * 2] + qs[(p * ni + i) * 2 + 1] * pv[m * 2 + 1]);
      }
    }
    C[s] = dense_inverse(D, nloc);
  }

  // pressure basis of cell geometry g at x (nbp values)
  void pressure(const Geom& g, const double* x, double* out) const {
    if (k == 1) {
      out[0] = 1.0;
      return;
    }
    double lam[3], klam[3];
    g.bary(x, lam);
    for (int i = 0; i < 3; ++i) klam[i] = (k - 1) * lam[i];
    pb.eval(klam, out);
  }
};

// symmetric strain part and divergence of a gradient gr[(i * 2 + c) * 2 + d]
inline double eps_td(const double* g, const double* t, const double* n1) {
  // t^T eps n1 with eps = (G + G^T) / 2, G[c][d] = d v_c / d x_d
  double s = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int d = 0; d < 2; ++d) s += t[c] * 0.5 * (g[c * 2 + d] + g[d * 2 + c]) * n1[d];
  return s;
}

double penalty_of(const Problem& pr, int k) {
  return pr.p.penalty > 0.0 ? pr.p.penalty : 2.0 * (k + 1) * (k + 1);
}

Space make_space(const LevelHost& L) {
  Space S;
  S.init(L.k, L.n);
  return S;
}

}  // namespace

void setup_mesh_bdm(LevelHost& L) {
  const int n = L.n, k = L.k;
  L.cells.clear();
  for (int c = 0; c < 2 * n * n; ++c) {
    const Tri t = tri_of(n, c);
    Cell cc{};
    for (int v = 0; v < 3; ++v)
      for (int d = 0; d < 2; ++d) cc.v[v][d] = t.v[v][d];
    L.cells.push_back(cc);
  }
  L.unit = n;
  const int nint = 3 * n * n - 2 * n;  // interior edges of the two-triangle mesh
  L.nvel = nint * (k + 1) + 2 * n * n * (k * k - 1);
  L.npres = 2 * n * n * (k * (k + 1) / 2);
  L.N = L.nvel + L.npres;
}

void build_level_bdm(LevelHost& L, const Problem& pr, bool with_rhs) {
  setup_mesh_bdm(L);
  const Space S = make_space(L);
  require(S.nvel == L.nvel && S.N == L.N, VK_EINVAL, "BDM DoF count mismatch");
  const int k = S.k, nloc = S.nloc, nbp = S.nbp, ncell = S.ncell;
  const double nu = pr.p.viscosity, alpha = penalty_of(pr, k);

  // pattern: cell c couples its velocity and pressure; edge terms couple the two cells of an edge
  std::vector<std::vector<int>> vcells(L.N);  // cells whose velocity columns a row sees
  std::vector<int> vd(nloc), vd2(nloc);
  for (int c = 0; c < ncell; ++c) {
    S.cell_vel(c, vd.data());
    std::vector<int> group{c};
    for (int l = 0; l < 3; ++l) {
      const auto& ec = S.ecells[S.cedge[c][l]];
      if (ec[1] >= 0) group.push_back(ec[0] == c ? ec[1] : ec[0]);
    }
    for (int i = 0; i < nloc; ++i)
      if (vd[i] >= 0) vcells[vd[i]].insert(vcells[vd[i]].end(), group.begin(), group.end());
  }
  Csr& K = L.K;
  K.nrows = K.ncols = L.N;
  K.rowptr.assign(L.N + 1, 0);
  K.col.clear();
  std::vector<int> tmp;
  for (int r = 0; r < L.N; ++r) {
    tmp.clear();
    if (r < S.nvel) {
      auto& g = vcells[r];
      std::sort(g.begin(), g.end());
      g.erase(std::unique(g.begin(), g.end()), g.end());
      for (int c : g) {
        S.cell_vel(c, vd.data());
        for (int i = 0; i < nloc; ++i)
          if (vd[i] >= 0) tmp.push_back(vd[i]);
      }
      // pressure of the cells holding r
      for (int c : g) {
        S.cell_vel(c, vd.data());
        bool holds = false;
        for (int i = 0; i < nloc; ++i) holds |= vd[i] == r;
        if (holds)
          for (int p = 0; p < nbp; ++p) tmp.push_back(S.pres0(c) + p);
      }
    } else {
      const int c = (r - S.nvel) / nbp;
      S.cell_vel(c, vd.data());
      for (int i = 0; i < nloc; ++i)
        if (vd[i] >= 0) tmp.push_back(vd[i]);
    }
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    K.col.insert(K.col.end(), tmp.begin(), tmp.end());
    K.rowptr[r + 1] = (int)K.col.size();
  }
  K.val.assign(K.col.size(), 0.0);
  vcells.clear();
  vcells.shrink_to_fit();
  auto addto = [&](int r, int c, double v) {
    const int* b = K.col.data() + K.rowptr[r];
    const int* e = K.col.data() + K.rowptr[r + 1];
    const int* it = std::lower_bound(b, e, c);
    K.val[K.rowptr[r] + (it - b)] += v;
  };

  // volume matrices and basis tables of the two orientations
  const SimplexRule rule = simplex_rule(2, k + 3);
  const int nq = rule.npts;
  std::vector<double> Avol[2], Bvol[2], Phi[2];
  std::vector<double> v((size_t)nloc * 2), gr((size_t)nloc * 4), pq(nbp);
  for (int s = 0; s < 2; ++s) {
    const Geom g = S.geom(s);
    const double adet = std::fabs(g.det);
    Avol[s].assign((size_t)nloc * nloc, 0.0);
    Bvol[s].assign((size_t)nbp * nloc, 0.0);
    Phi[s].assign((size_t)nq * nloc * 2, 0.0);
    std::vector<double> eps((size_t)nloc * 4), div(nloc);
    for (int q = 0; q < nq; ++q) {
      double x[2];
      g.point(&rule.lam[q * 3], x);
      S.phi(s, g, x, v.data(), gr.data());
      std::copy(v.begin(), v.end(), Phi[s].begin() + (size_t)q * nloc * 2);
      S.pressure(g, x, pq.data());
      const double w = rule.w[q] * adet;
      for (int i = 0; i < nloc; ++i) {
        const double* G = &gr[(size_t)i * 4];
        eps[i * 4 + 0] = G[0];
        eps[i * 4 + 1] = 0.5 * (G[1] + G[2]);
        eps[i * 4 + 2] = eps[i * 4 + 1];
        eps[i * 4 + 3] = G[3];
        div[i] = G[0] + G[3];
      }
      for (int i = 0; i < nloc; ++i)
        for (int j = 0; j < nloc; ++j) {
          double s2 = 0.0;
          for (int m = 0; m < 4; ++m) s2 += eps[i * 4 + m] * eps[j * 4 + m];
          Avol[s][(size_t)i * nloc + j] += 2.0 * nu * w * s2;
        }
      for (int p = 0; p < nbp; ++p)
        for (int j = 0; j < nloc; ++j) Bvol[s][(size_t)p * nloc + j] -= w * pq[p] * div[j];
    }
  }
  if (with_rhs) L.b.assign(L.N, 0.0);
  for (int c = 0; c < ncell; ++c) {
    const int s = c & 1;
    S.cell_vel(c, vd.data());
    const int p0 = S.pres0(c);
    for (int i = 0; i < nloc; ++i) {
      const int r = vd[i];
      if (r < 0) continue;
      for (int j = 0; j < nloc; ++j)
        if (vd[j] >= 0) addto(r, vd[j], Avol[s][(size_t)i * nloc + j]);
      for (int p = 0; p < nbp; ++p) {
        addto(r, p0 + p, Bvol[s][(size_t)p * nloc + i]);
        addto(p0 + p, r, Bvol[s][(size_t)p * nloc + i]);
      }
    }
    if (with_rhs) {
      const Geom g = S.geom(c);
      const double adet = std::fabs(g.det);
      for (int q = 0; q < nq; ++q) {
        double x[3] = {0, 0, 0}, f[3];
        g.point(&rule.lam[q * 3], x);
        field_f(pr, x, f);
        const double w = rule.w[q] * adet;
        const double* P = &Phi[s][(size_t)q * nloc * 2];
        for (int i = 0; i < nloc; ++i)
          if (vd[i] >= 0) L.b[vd[i]] += w * (f[0] * P[i * 2] + f[1] * P[i * 2 + 1]);
      }
    }
  }

  // interior edges: matrices cached by (orientation and local edge of T1, the same of T2)
  std::map<std::array<int, 4>, std::vector<double>> cache;
  std::vector<double> gq, gw;
  gauss_legendre_01(k + 2, gq, gw);
  const int n2 = 2 * nloc;
  for (size_t e = 0; e < S.ekey.size(); ++e) {
    if (S.erank[e] < 0) continue;
    double a[2], b[2], len, t[2], ne_[2];
    S.edge_frame((int)e, a, b, len, t, ne_);
    int T1 = S.ecells[e][0], T2 = S.ecells[e][1];
    {
      // T1 is the cell that n_e points out of
      const Tri tt = S.cell(T1);
      const double cx = (tt.v[0][0] + tt.v[1][0] + tt.v[2][0]) * S.h / 3.0;
      const double cy = (tt.v[0][1] + tt.v[1][1] + tt.v[2][1]) * S.h / 3.0;
      if ((cx - 0.5 * (a[0] + b[0])) * ne_[0] + (cy - 0.5 * (a[1] + b[1])) * ne_[1] > 0) std::swap(T1, T2);
    }
    int l1 = 0, l2 = 0;
    for (int l = 0; l < 3; ++l) {
      if (S.cedge[T1][l] == (int)e) l1 = l;
      if (S.cedge[T2][l] == (int)e) l2 = l;
    }
    const std::array<int, 4> key{T1 & 1, l1, T2 & 1, l2};
    auto it = cache.find(key);
    if (it == cache.end()) {
      std::vector<double> M((size_t)n2 * n2, 0.0), jump(n2), avg(n2);
      const Geom g1 = S.geom(T1), g2 = S.geom(T2);
      for (size_t q = 0; q < gq.size(); ++q) {
        const double x[2] = {a[0] + gq[q] * (b[0] - a[0]), a[1] + gq[q] * (b[1] - a[1])};
        const double w = gw[q] * len;
        for (int side = 0; side < 2; ++side) {
          S.phi(side == 0 ? (T1 & 1) : (T2 & 1), side == 0 ? g1 : g2, x, v.data(), gr.data());
          const double sg = side == 0 ? 1.0 : -1.0;
          for (int i = 0; i < nloc; ++i) {
            jump[side * nloc + i] = sg * (v[i * 2] * t[0] + v[i * 2 + 1] * t[1]);
            avg[side * nloc + i] = 0.5 * eps_td(&gr[(size_t)i * 4], t, ne_);
          }
        }
        for (int i = 0; i < n2; ++i)
          for (int j = 0; j < n2; ++j)
            M[(size_t)i * n2 + j] += w * (-2.0 * nu * (jump[i] * avg[j] + avg[i] * jump[j]) +
                                          nu * alpha / len * jump[i] * jump[j]);
      }
      it = cache.emplace(key, std::move(M)).first;
    }
    const std::vector<double>& M = it->second;
    S.cell_vel(T1, vd.data());
    S.cell_vel(T2, vd2.data());
    for (int i = 0; i < n2; ++i) {
      const int r = i < nloc ? vd[i] : vd2[i - nloc];
      if (r < 0) continue;
      for (int j = 0; j < n2; ++j) {
        const int cidx = j < nloc ? vd[j] : vd2[j - nloc];
        if (cidx >= 0) addto(r, cidx, M[(size_t)i * n2 + j]);
      }
    }
  }
}

// Natural embedding (Sec. 3, grid transfers): row f of the velocity block is the fine functional
// f applied to the coarse basis functions of one coarse cell holding the fine entity (a fine edge
// on a coarse edge sees the same normal trace from both sides, the lower triangle is taken); the
// pressure rows are the coarse pressure basis of the parent cell at the fine nodes.  Entries below
// 1e-12 in magnitude (zeros up to rounding) are dropped.  Blocks are cached by the coarse cell's
// orientation and the fine entity's position relative to the coarse square.
void build_prolongation_bdm(const LevelHost& Cl, LevelHost& Fl) {
  const Space C = make_space(Cl), F = make_space(Fl);
  const int k = F.k, nloc = C.nloc, nbp = F.nbp, nc = C.n;
  std::vector<std::vector<std::pair<int, double>>> rows(F.N);
  std::map<std::vector<int>, std::vector<double>> cache;
  std::vector<double> v((size_t)nloc * 2), L(F.ne), gq, gw, cvals;
  std::vector<int> cvd(nloc);
  gauss_legendre_01(k + 2, gq, gw);
  auto put = [&](int r, const int* cd, const double* vals, int cnt) {
    for (int j = 0; j < cnt; ++j)
      if (cd[j] >= 0 && std::fabs(vals[j]) >= 1e-12) rows[r].push_back({cd[j], vals[j]});
  };
  // coarse cell holding a point given as 4 x (fine lattice point sum of two) or 6 x (sum of three)
  auto locate = [&](int sx, int sy, int unit, int& sq_i, int& sq_j) {
    sq_i = std::min(sx / unit, nc - 1);
    sq_j = std::min(sy / unit, nc - 1);
    const int u = sx - unit * sq_i, w = sy - unit * sq_j;
    return 2 * (sq_j * nc + sq_i) + (u + w <= unit ? 0 : 1);
  };
  // velocity: fine interior edges
  for (size_t e = 0; e < F.ekey.size(); ++e) {
    const int r = F.erank[e];
    if (r < 0) continue;
    const int ax = F.ekey[e][0] % (F.n + 1), ay = F.ekey[e][0] / (F.n + 1);
    const int bx = F.ekey[e][1] % (F.n + 1), by = F.ekey[e][1] / (F.n + 1);
    int si, sj;
    const int cc = locate(ax + bx, ay + by, 4, si, sj);
    const std::vector<int> key{0, cc & 1, ax - 2 * si, ay - 2 * sj, bx - 2 * si, by - 2 * sj};
    auto it = cache.find(key);
    if (it == cache.end()) {
      double a[2], b[2], len, t[2], nr[2];
      F.edge_frame((int)e, a, b, len, t, nr);
      const Geom g = C.geom(cc);
      std::vector<double> blk((size_t)F.ne * nloc, 0.0);
      for (size_t q = 0; q < gq.size(); ++q) {
        const double x[2] = {a[0] + gq[q] * (b[0] - a[0]), a[1] + gq[q] * (b[1] - a[1])};
        C.phi(cc & 1, g, x, v.data(), nullptr);
        legendre01(k, gq[q], L.data());
        for (int j = 0; j < F.ne; ++j)
          for (int i = 0; i < nloc; ++i)
            blk[(size_t)j * nloc + i] += gw[q] * L[j] * (v[i * 2] * nr[0] + v[i * 2 + 1] * nr[1]);
      }
      it = cache.emplace(key, std::move(blk)).first;
    }
    C.cell_vel(cc, cvd.data());
    for (int j = 0; j < F.ne; ++j) put(r * F.ne + j, cvd.data(), &it->second[(size_t)j * nloc], nloc);
  }
  // velocity interiors and pressure: fine cells
  std::vector<double> xs, ws, qs, pq(C.nbp);
  for (int c = 0; c < F.ncell; ++c) {
    const Tri t = F.cell(c);
    int si, sj;
    const int cc = locate(t.v[0][0] + t.v[1][0] + t.v[2][0], t.v[0][1] + t.v[1][1] + t.v[2][1], 6, si, sj);
    std::vector<int> key{1, cc & 1};
    for (int vv = 0; vv < 3; ++vv) {
      key.push_back(t.v[vv][0] - 2 * si);
      key.push_back(t.v[vv][1] - 2 * sj);
    }
    auto it = cache.find(key);
    if (it == cache.end()) {
      const Geom gf = F.geom(c), gc = C.geom(cc);
      std::vector<double> blk((size_t)(F.ni + nbp) * std::max(nloc, C.nbp), 0.0);
      const int wdt = std::max(nloc, C.nbp);
      if (F.ni > 0) {
        F.interior_tests(c & 1, gf, xs, ws, qs);
        for (size_t p = 0; p < ws.size(); ++p) {
          C.phi(cc & 1, gc, &xs[p * 2], v.data(), nullptr);
          for (int m = 0; m < F.ni; ++m)
            for (int i = 0; i < nloc; ++i)
              blk[(size_t)m * wdt + i] +=
                  ws[p] * (qs[(p * F.ni + m) * 2] * v[i * 2] + qs[(p * F.ni + m) * 2 + 1] * v[i * 2 + 1]);
        }
      }
      // pressure nodes of the fine cell: V0 + J a / (k - 1) (the centroid for k = 1)
      for (int p = 0; p < nbp; ++p) {
        double lam[3];
        if (k == 1) {
          lam[0] = lam[1] = lam[2] = 1.0 / 3.0;
        } else {
          for (int i = 0; i < 3; ++i) lam[i] = (double)F.pb.nodes[p][i] / (k - 1);
        }
        double x[2];
        gf.point(lam, x);
        C.pressure(gc, x, pq.data());
        for (int j = 0; j < C.nbp; ++j) blk[(size_t)(F.ni + p) * wdt + j] = pq[j];
      }
      it = cache.emplace(key, std::move(blk)).first;
    }
    const int wdt = std::max(nloc, C.nbp);
    C.cell_vel(cc, cvd.data());
    for (int m = 0; m < F.ni; ++m) put(F.nint * F.ne + c * F.ni + m, cvd.data(), &it->second[(size_t)m * wdt], nloc);
    std::vector<int> cpd(C.nbp);
    for (int j = 0; j < C.nbp; ++j) cpd[j] = C.pres0(cc) + j;
    for (int p = 0; p < nbp; ++p) put(F.pres0(c) + p, cpd.data(), &it->second[(size_t)(F.ni + p) * wdt], C.nbp);
  }
  Csr P;
  P.nrows = F.N;
  P.ncols = C.N;
  P.rowptr.assign(F.N + 1, 0);
  for (int r = 0; r < F.N; ++r) {
    auto& vv = rows[r];
    std::sort(vv.begin(), vv.end());
    for (auto& e : vv) {
      P.col.push_back(e.first);
      P.val.push_back(e.second);
    }
    P.rowptr[r + 1] = (int)P.col.size();
  }
  Fl.P = std::move(P);
  Fl.PT = transpose(Fl.P);
}

// Extended cell patches (Sec. 3.1): per cell, its pressure and the velocity on the closure of the
// cell and of the cells sharing an edge with it
void build_patches_bdm(LevelHost& L, double omega, int store) {
  const Space S = make_space(L);
  std::vector<std::vector<int>> patches(S.ncell);
  std::vector<int> vd(S.nloc);
  for (int c = 0; c < S.ncell; ++c) {
    std::vector<int>& p = patches[c];
    std::vector<int> group{c};
    for (int l = 0; l < 3; ++l) {
      const auto& ec = S.ecells[S.cedge[c][l]];
      if (ec[1] >= 0) group.push_back(ec[0] == c ? ec[1] : ec[0]);
    }
    for (int g : group) {
      S.cell_vel(g, vd.data());
      for (int i = 0; i < S.nloc; ++i)
        if (vd[i] >= 0) p.push_back(vd[i]);
    }
    for (int q = 0; q < S.nbp; ++q) p.push_back(S.pres0(c) + q);
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
  }
  finalize_patches(L, patches, omega, store);
}

// relative broken H^1 velocity error and mean-free L^2 pressure error (collapsed rule, k + 6 points)
void solution_errors_bdm(const LevelHost& L, const Problem& pr, const double* x, double* e_u, double* e_p) {
  const Space S = make_space(L);
  const int nloc = S.nloc, nbp = S.nbp;
  const SimplexRule rule = simplex_rule(2, S.k + 6);
  const int nq = rule.npts;
  // basis values and gradients at the rule points, per orientation (translates share them)
  std::vector<double> tv[2], tg[2], tp[2];
  for (int s = 0; s < 2; ++s) {
    const Geom g = S.geom(s);
    tv[s].resize((size_t)nq * nloc * 2);
    tg[s].resize((size_t)nq * nloc * 4);
    tp[s].resize((size_t)nq * nbp);
    for (int q = 0; q < nq; ++q) {
      double x[2];
      g.point(&rule.lam[q * 3], x);
      S.phi(s, g, x, &tv[s][(size_t)q * nloc * 2], &tg[s][(size_t)q * nloc * 4]);
      S.pressure(g, x, &tp[s][(size_t)q * nbp]);
    }
  }
  std::vector<double> U(nloc);
  std::vector<int> vd(nloc);
  double e1 = 0, n1 = 0, ep_int = 0, ep2 = 0, area = 0;
  for (int c = 0; c < S.ncell; ++c) {
    const int s = c & 1;
    const Geom g = S.geom(c);
    const double adet = std::fabs(g.det);
    S.cell_vel(c, vd.data());
    for (int i = 0; i < nloc; ++i) U[i] = vd[i] >= 0 ? x[vd[i]] : 0.0;
    for (int q = 0; q < nq; ++q) {
      double xq[3] = {0, 0, 0};
      g.point(&rule.lam[q * 3], xq);
      const double* v = &tv[s][(size_t)q * nloc * 2];
      const double* gr = &tg[s][(size_t)q * nloc * 4];
      double uh[2] = {0, 0}, guh[4] = {0, 0, 0, 0};
      for (int i = 0; i < nloc; ++i) {
        for (int cc = 0; cc < 2; ++cc) uh[cc] += U[i] * v[i * 2 + cc];
        for (int m = 0; m < 4; ++m) guh[m] += U[i] * gr[(size_t)i * 4 + m];
      }
      double ue[3], gue[9];
      field_u(pr, xq, ue);
      field_grad_u(pr, xq, gue);
      double se = 0.0, sn = 0.0;
      for (int cc = 0; cc < 2; ++cc) {
        se += (ue[cc] - uh[cc]) * (ue[cc] - uh[cc]);
        sn += ue[cc] * ue[cc];
        for (int d = 0; d < 2; ++d) {
          se += (gue[cc * 2 + d] - guh[cc * 2 + d]) * (gue[cc * 2 + d] - guh[cc * 2 + d]);
          sn += gue[cc * 2 + d] * gue[cc * 2 + d];
        }
      }
      const double w = rule.w[q] * adet;
      e1 += w * se;
      n1 += w * sn;
      double ph = 0.0;
      for (int p = 0; p < nbp; ++p) ph += x[S.pres0(c) + p] * tp[s][(size_t)q * nbp + p];
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

// DoF sites: edge moments at the edge midpoint, interior moments at the centroid (kind 0),
// pressure at its node (kind 2)
void dof_coords_bdm(const LevelHost& L, double* xyz, int* kind) {
  const Space S = make_space(L);
  for (size_t e = 0; e < S.ekey.size(); ++e) {
    const int r = S.erank[e];
    if (r < 0) continue;
    double a[2], b[2], len, t[2], nr[2];
    S.edge_frame((int)e, a, b, len, t, nr);
    for (int j = 0; j < S.ne; ++j) {
      xyz[(r * S.ne + j) * 2] = 0.5 * (a[0] + b[0]);
      xyz[(r * S.ne + j) * 2 + 1] = 0.5 * (a[1] + b[1]);
      kind[r * S.ne + j] = 0;
    }
  }
  for (int c = 0; c < S.ncell; ++c) {
    const Geom g = S.geom(c);
    const double third[3] = {1.0 / 3, 1.0 / 3, 1.0 / 3};
    double xc[2];
    g.point(third, xc);
    for (int m = 0; m < S.ni; ++m) {
      const int d = S.nint * S.ne + c * S.ni + m;
      xyz[d * 2] = xc[0];
      xyz[d * 2 + 1] = xc[1];
      kind[d] = 0;
    }
    for (int p = 0; p < S.nbp; ++p) {
      double lam[3] = {1.0 / 3, 1.0 / 3, 1.0 / 3};
      if (S.k > 1)
        for (int i = 0; i < 3; ++i) lam[i] = (double)S.pb.nodes[p][i] / (S.k - 1);
      double x[2];
      g.point(lam, x);
      const int d = S.pres0(c) + p;
      xyz[d * 2] = x[0];
      xyz[d * 2 + 1] = x[1];
      kind[d] = 2;
    }
  }
}

}  // namespace vk
