// Host-side assembly of one multigrid level: structured mesh, Taylor-Hood
// (or Scott-Vogelius, whose mesh and numbering come from host_sv.cpp) DoF
// numbering, K = [A B^T; B 0] on the free DoFs, right-hand side with
// Dirichlet lifting (Sec. 2 weak form, Sec. 3 per-level saddle-point
// matrix), and the prolongation by nodal interpolation (Sec. 3, grid
// transfers: natural embedding of the nested spaces).
#include <algorithm>
#include <array>
#include <thread>
#include <cmath>

#include "vk_internal.hpp"

namespace vk {

static const double PI = 3.14159265358979323846;

int LevelHost::vel_dof(const int* G, int c) const {
  if (family == VK_SV) {
    const int M = k * unit;
    if (G[0] <= 0 || G[1] <= 0 || G[0] >= M || G[1] >= M) return -1;
    const int id = vmap[(size_t)G[1] * (M + 1) + G[0]];
    return id < 0 ? -1 : 2 * id + c;
  }
  const int M = k * n;
  int idx = 0;
  for (int d = dim - 1; d >= 0; --d) {
    if (G[d] <= 0 || G[d] >= M) return -1;
    idx = idx * (M - 1) + (G[d] - 1);
  }
  return dim * idx + c;
}

int LevelHost::pres_dof(const int* G) const {
  const int M = (k - 1) * n;
  int idx = 0;
  for (int d = dim - 1; d >= 0; --d) idx = idx * (M + 1) + G[d];
  return nvel + idx;
}

static void make_cells(LevelHost& L) {
  const int n = L.n;
  L.cells.clear();
  if (L.dim == 2) {
    // square (i,j) cut from top-left to bottom-right: (BL, BR, TL) and (TR, TL, BR)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        Cell lo = {{{i, j, 0}, {i + 1, j, 0}, {i, j + 1, 0}, {0, 0, 0}}};
        Cell up = {{{i + 1, j + 1, 0}, {i, j + 1, 0}, {i + 1, j, 0}, {0, 0, 0}}};
        L.cells.push_back(lo);
        L.cells.push_back(up);
      }
  } else {
    // six Kuhn tetrahedra per cube, one per ordering of the axes, all sharing
    // the cube diagonal; orderings in lexicographic order of the permutation
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int l = 0; l < n; ++l)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          for (auto& p : perms) {
            Cell c;
            int v[3] = {i, j, l};
            for (int d = 0; d < 3; ++d) c.v[0][d] = v[d];
            for (int s = 0; s < 3; ++s) {
              v[p[s]] += 1;
              for (int d = 0; d < 3; ++d) c.v[s + 1][d] = v[d];
            }
            L.cells.push_back(c);
          }
  }
}

void setup_mesh(LevelHost& L) {
  if (L.family == VK_SV) {
    setup_mesh_sv(L);
    return;
  }
  if (L.family == VK_TH_QUAD) {
    setup_mesh_quad(L);
    return;
  }
  if (L.family == VK_BDM) {
    setup_mesh_bdm(L);
    return;
  }
  make_cells(L);
  L.unit = L.n;
  const int Mv = L.k * L.n, Mp = (L.k - 1) * L.n;
  int nint = 1, np = 1;
  for (int d = 0; d < L.dim; ++d) {
    nint *= (Mv - 1);
    np *= (Mp + 1);
  }
  L.nvel = L.dim * nint;
  L.npres = np;
  L.N = L.nvel + L.npres;
}

// exact velocity, forcing (returns dim components)
void field_u(const Problem& pr, const double* x, double* u) {
  const double X = x[0], Y = x[1];
  switch (pr.p.forcing) {
    case VK_F_BASELINE_MMS:
      u[0] = std::sin(PI * X) * std::sin(PI * Y);
      u[1] = std::cos(PI * X) * std::cos(PI * Y);
      break;
    case VK_F_PAPER_MMS:
      u[0] = std::sin(PI * X) * std::cos(PI * Y);
      u[1] = -std::cos(PI * X) * std::sin(PI * Y);
      break;
    case VK_F_CUBE_MMS: {
      const double Z = x[2];
      u[0] = std::sin(PI * X) * std::cos(PI * Y) - std::sin(PI * X) * std::cos(PI * Z);
      u[1] = std::sin(PI * Y) * std::cos(PI * Z) - std::cos(PI * X) * std::sin(PI * Y);
      u[2] = std::sin(PI * Z) * std::cos(PI * X) - std::cos(PI * Y) * std::sin(PI * Z);
      break;
    }
    default:
      for (int c = 0; c < pr.p.dim; ++c) u[c] = 0.0;
  }
}

// exact velocity gradient g[c * dim + d] = d u_c / d x_d of the manufactured fields (zero otherwise)
void field_grad_u(const Problem& pr, const double* x, double* g) {
  const double X = x[0], Y = x[1];
  const double sx = std::sin(PI * X), cx = std::cos(PI * X), sy = std::sin(PI * Y), cy = std::cos(PI * Y);
  switch (pr.p.forcing) {
    case VK_F_BASELINE_MMS:
      g[0] = PI * cx * sy;  g[1] = PI * sx * cy;
      g[2] = -PI * sx * cy; g[3] = -PI * cx * sy;
      break;
    case VK_F_PAPER_MMS:
      g[0] = PI * cx * cy;  g[1] = -PI * sx * sy;
      g[2] = PI * sx * sy;  g[3] = -PI * cx * cy;
      break;
    case VK_F_CUBE_MMS: {
      const double sz = std::sin(PI * x[2]), cz = std::cos(PI * x[2]);
      g[0] = PI * cx * (cy - cz); g[1] = -PI * sx * sy;       g[2] = PI * sx * sz;
      g[3] = PI * sx * sy;        g[4] = PI * cy * (cz - cx); g[5] = -PI * sy * sz;
      g[6] = -PI * sz * sx;       g[7] = PI * sy * sz;        g[8] = PI * cz * (cx - cy);
      break;
    }
    default:
      for (int c = 0; c < pr.p.dim * pr.p.dim; ++c) g[c] = 0.0;
  }
}

void field_f(const Problem& pr, const double* x, double* f) {
  const double nu = pr.p.viscosity;
  if (pr.p.forcing == VK_F_RANDOM) {
    const int M = pr.p.n_modes;
    for (int c = 0; c < 2; ++c) {
      double s = 0.0;
      for (int a = 1; a <= M; ++a)
        for (int b = 1; b <= M; ++b)
          s += pr.coeffs[(c * M + (a - 1)) * M + (b - 1)] * std::sin(a * PI * x[0]) * std::sin(b * PI * x[1]) /
               (double)(a * a + b * b);
      f[c] = s;
    }
    return;
  }
  // divergence-free eigenfunction fields with p = 0: f = -nu Laplace u = 2 nu pi^2 u
  double u[3];
  field_u(pr, x, u);
  for (int c = 0; c < pr.p.dim; ++c) f[c] = 2.0 * nu * PI * PI * u[c];
}

// local P_kk node j of a cell -> global lattice point (units 1/(kk n))
static inline void node_lattice(const Cell& c, const std::vector<int>& a, int dim, int* G) {
  for (int d = 0; d < dim; ++d) {
    int g = 0;
    for (int i = 0; i <= dim; ++i) g += a[i] * c.v[i][d];
    G[d] = g;
  }
}

// local -> global DoFs of every cell (-1: Dirichlet velocity)
void cell_dof_maps(const LevelHost& L, const Basis& vb, const Basis& pb, std::vector<int>& cvd,
                   std::vector<int>& cpd) {
  const int dim = L.dim, nbv = vb.size(), nbp = pb.size(), nlv = nbv * dim;
  const int ncell = (int)L.cells.size();
  cvd.assign((size_t)ncell * nlv, 0);
  cpd.assign((size_t)ncell * nbp, 0);
  for (int e = 0; e < ncell; ++e) {
    int G[3];
    for (int j = 0; j < nbv; ++j) {
      node_lattice(L.cells[e], vb.nodes[j], dim, G);
      for (int c = 0; c < dim; ++c) cvd[(size_t)e * nlv + j * dim + c] = L.vel_dof(G, c);
    }
    for (int j = 0; j < nbp; ++j) {
      if (L.family == VK_SV) {
        cpd[(size_t)e * nbp + j] = L.sv_pres_dof(e, pb.nodes[j][1], pb.nodes[j][2]);
        continue;
      }
      node_lattice(L.cells[e], pb.nodes[j], dim, G);
      cpd[(size_t)e * nbp + j] = L.pres_dof(G);
    }
  }
}

// Discretisation errors of a solution on level L (Sec. 4, stopping criteria): the relative H^1
// error of the velocity (Dirichlet nodes carry the exact nodal values, as in the lifting) and the
// L^2 error of the pressure after removing the L^2 mean of the difference, integrated with the
// collapsed Gauss rule of k + 6 points per direction.
void solution_errors(const LevelHost& L, const Problem& pr, const double* x, double* e_u, double* e_p) {
  if (L.family == VK_TH_QUAD) {
    solution_errors_quad(L, pr, x, e_u, e_p);
    return;
  }
  if (L.family == VK_BDM) {
    solution_errors_bdm(L, pr, x, e_u, e_p);
    return;
  }
  const int dim = L.dim, k = L.k, unit = L.unit;
  const Basis vb = make_basis(dim, k), pb = make_basis(dim, k - 1);
  const int nbv = vb.size(), nbp = pb.size(), nlv = nbv * dim;
  const SimplexRule rule = simplex_rule(dim, k + 6);
  const int nq = rule.npts;
  std::vector<int> cvd, cpd;
  cell_dof_maps(L, vb, pb, cvd, cpd);
  std::vector<double> phv((size_t)nq * nbv), php((size_t)nq * nbp), dv((size_t)nq * nbv * (dim + 1));
  for (int q = 0; q < nq; ++q) {
    double kl[4], kl1[4];
    for (int i = 0; i <= dim; ++i) {
      kl[i] = k * rule.lam[q * (dim + 1) + i];
      kl1[i] = (k - 1) * rule.lam[q * (dim + 1) + i];
    }
    vb.eval(kl, &phv[(size_t)q * nbv]);
    pb.eval(kl1, &php[(size_t)q * nbp]);
    vb.dlam(&rule.lam[q * (dim + 1)], &dv[(size_t)q * nbv * (dim + 1)]);
  }
  double e1 = 0, n1 = 0, ep_int = 0, ep2 = 0, area = 0;
  std::vector<double> U(nlv), P(nbp);
  for (int e = 0; e < (int)L.cells.size(); ++e) {
    const Cell& C = L.cells[e];
    double J[3][3], Ji[3][3];
    for (int d = 0; d < dim; ++d)
      for (int i = 0; i < dim; ++i) J[d][i] = (double)(C.v[i + 1][d] - C.v[0][d]) / unit;
    double det;
    if (dim == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      Ji[0][0] = J[1][1] / det; Ji[0][1] = -J[0][1] / det;
      Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
    } else {
      det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
            J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    const double adet = std::fabs(det);
    double gl[4][3];
    for (int d = 0; d < dim; ++d) {
      double sgl = 0.0;
      for (int i = 1; i <= dim; ++i) {
        gl[i][d] = Ji[i - 1][d];
        sgl += Ji[i - 1][d];
      }
      gl[0][d] = -sgl;
    }
    const int* vd = &cvd[(size_t)e * nlv];
    const int* pd = &cpd[(size_t)e * nbp];
    for (int j = 0; j < nbv; ++j) {
      if (vd[j * dim] >= 0) {
        for (int c = 0; c < dim; ++c) U[j * dim + c] = x[vd[j * dim + c]];
      } else {
        int G[3];
        node_lattice(C, vb.nodes[j], dim, G);
        double xn[3];
        for (int d = 0; d < dim; ++d) xn[d] = (double)G[d] / (k * unit);
        field_u(pr, xn, &U[j * dim]);
      }
    }
    for (int p = 0; p < nbp; ++p) P[p] = x[pd[p]];
    for (int q = 0; q < nq; ++q) {
      const double w = rule.w[q] * adet;
      double xq[3];
      for (int d = 0; d < dim; ++d) {
        double sx = C.v[0][d] / (double)unit;
        for (int i = 1; i <= dim; ++i) sx += J[d][i - 1] * rule.lam[q * (dim + 1) + i];
        xq[d] = sx;
      }
      double uh[3] = {0, 0, 0}, guh[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      const double* vq = &phv[(size_t)q * nbv];
      const double* dq = &dv[(size_t)q * nbv * (dim + 1)];
      for (int j = 0; j < nbv; ++j) {
        double gphi[3];
        for (int d = 0; d < dim; ++d) {
          double sg = 0.0;
          for (int i = 0; i <= dim; ++i) sg += dq[j * (dim + 1) + i] * gl[i][d];
          gphi[d] = sg;
        }
        for (int c = 0; c < dim; ++c) {
          uh[c] += U[j * dim + c] * vq[j];
          for (int d = 0; d < dim; ++d) guh[c * dim + d] += U[j * dim + c] * gphi[d];
        }
      }
      double ue[3], gue[9];
      field_u(pr, xq, ue);
      field_grad_u(pr, xq, gue);
      double se = 0.0, sn = 0.0;
      for (int c = 0; c < dim; ++c) {
        se += (ue[c] - uh[c]) * (ue[c] - uh[c]);
        sn += ue[c] * ue[c];
        for (int d = 0; d < dim; ++d) {
          se += (gue[c * dim + d] - guh[c * dim + d]) * (gue[c * dim + d] - guh[c * dim + d]);
          sn += gue[c * dim + d] * gue[c * dim + d];
        }
      }
      e1 += w * se;
      n1 += w * sn;
      double ph = 0.0;
      const double* pq = &php[(size_t)q * nbp];
      for (int p = 0; p < nbp; ++p) ph += P[p] * pq[p];
      const double dp = 0.0 - ph;  // the manufactured pressures are zero
      ep_int += w * dp;
      ep2 += w * dp * dp;
      area += w;
    }
  }
  const double mean = ep_int / area;
  *e_u = std::sqrt(e1 / n1);
  *e_p = std::sqrt(std::max(ep2 - 2.0 * mean * ep_int + mean * mean * area, 0.0));
}

void build_level(LevelHost& L, const Problem& pr, bool with_rhs) {
  if (L.family == VK_TH_QUAD) {
    build_level_quad(L, pr, with_rhs);
    return;
  }
  if (L.family == VK_BDM) {
    build_level_bdm(L, pr, with_rhs);
    return;
  }
  const int dim = L.dim, k = L.k;
  const double nu = pr.p.viscosity;
  setup_mesh(L);
  const int unit = L.unit;

  const Basis vb = make_basis(dim, k), pb = make_basis(dim, k - 1);
  const int nbv = vb.size(), nbp = pb.size();
  const int nlv = nbv * dim;
  const SimplexRule rule = simplex_rule(dim, k + 3);
  const int nq = rule.npts;

  const int ncell = (int)L.cells.size();
  std::vector<int> cvd, cpd;
  cell_dof_maps(L, vb, pb, cvd, cpd);

  // sparsity pattern: the element closure (all DoF pairs sharing a cell, no
  // pressure-pressure pairs); rows collected through DoF -> cells lists
  std::vector<std::vector<int>> dcells(L.N);
  for (int e = 0; e < ncell; ++e) {
    for (int j = 0; j < nlv; ++j) {
      int d = cvd[(size_t)e * nlv + j];
      if (d >= 0) dcells[d].push_back(e);
    }
    for (int j = 0; j < nbp; ++j) dcells[cpd[(size_t)e * nbp + j]].push_back(e);
  }
  Csr& K = L.K;
  K.nrows = K.ncols = L.N;
  K.rowptr.assign(L.N + 1, 0);
  std::vector<int> tmp;
  for (int r = 0; r < L.N; ++r) {
    tmp.clear();
    const bool rp = r >= L.nvel;
    for (int e : dcells[r]) {
      for (int j = 0; j < nlv; ++j) {
        int d = cvd[(size_t)e * nlv + j];
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

  auto addto = [&](int r, int c, double v) {
    const int* b = K.col.data() + K.rowptr[r];
    const int* e = K.col.data() + K.rowptr[r + 1];
    const int* it = std::lower_bound(b, e, c);
    K.val[K.rowptr[r] + (it - b)] += v;
  };

  // basis values and barycentric derivatives at the quadrature points (the
  // same on every cell; the geometry enters through grad lambda)
  std::vector<double> phv((size_t)nq * nbv), php((size_t)nq * nbp), dv((size_t)nq * nbv * (dim + 1));
  for (int q = 0; q < nq; ++q) {
    double kl[4], kl1[4];
    for (int i = 0; i <= dim; ++i) {
      kl[i] = k * rule.lam[q * (dim + 1) + i];
      kl1[i] = (k - 1) * rule.lam[q * (dim + 1) + i];
    }
    vb.eval(kl, &phv[(size_t)q * nbv]);
    pb.eval(kl1, &php[(size_t)q * nbp]);
    vb.dlam(&rule.lam[q * (dim + 1)], &dv[(size_t)q * nbv * (dim + 1)]);
  }

  if (with_rhs) L.b.assign(L.N, 0.0);
  struct Shape {
    std::array<double, 9> key;
    std::vector<double> A, B;
  };
  std::vector<Shape> shapes;
  std::vector<double> Floc(nlv), uD(nlv);
  std::vector<double> gx((size_t)nbv * dim);
  for (int e = 0; e < ncell; ++e) {
    const Cell& C = L.cells[e];
    // affine map x = x0 + J xi, J columns = (x_i - x_0), x = v / n
    double J[3][3], Ji[3][3];
    for (int d = 0; d < dim; ++d)
      for (int i = 0; i < dim; ++i) J[d][i] = (double)(C.v[i + 1][d] - C.v[0][d]) / unit;
    double det;
    if (dim == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      Ji[0][0] = J[1][1] / det; Ji[0][1] = -J[0][1] / det;
      Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
    } else {
      det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
            J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    const double adet = std::fabs(det);
    // grad lambda_i (i >= 1) = row i-1 of J^{-1}; grad lambda_0 = -sum
    double gl[4][3];
    for (int d = 0; d < dim; ++d) {
      double s = 0.0;
      for (int i = 1; i <= dim; ++i) {
        gl[i][d] = Ji[i - 1][d];
        s += Ji[i - 1][d];
      }
      gl[0][d] = -s;
    }
    // the element matrices depend on the cell only through its Jacobian: computed once per
    // distinct Jacobian (the structured meshes have a handful) and reused bitwise
    std::array<double, 9> key{};
    for (int d = 0; d < dim; ++d)
      for (int i = 0; i < dim; ++i) key[d * 3 + i] = J[d][i];
    auto hit = std::find_if(shapes.begin(), shapes.end(), [&](const Shape& sh) { return sh.key == key; });
    if (hit == shapes.end()) {
      Shape sh;
      sh.key = key;
      sh.A.assign((size_t)nlv * nlv, 0.0);
      sh.B.assign((size_t)nbp * nlv, 0.0);
      for (int q = 0; q < nq; ++q) {
        const double w = rule.w[q] * adet;
        const double* dq = &dv[(size_t)q * nbv * (dim + 1)];
        for (int j = 0; j < nbv; ++j)
          for (int d = 0; d < dim; ++d) {
            double s = 0.0;
            for (int i = 0; i <= dim; ++i) s += dq[j * (dim + 1) + i] * gl[i][d];
            gx[j * dim + d] = s;
          }
        // A[(i,c),(j,d)] += w nu (delta_cd grad phi_i . grad phi_j + d_d phi_i d_c phi_j)
        for (int i = 0; i < nbv; ++i)
          for (int j = 0; j < nbv; ++j) {
            double dot = 0.0;
            for (int d = 0; d < dim; ++d) dot += gx[i * dim + d] * gx[j * dim + d];
            for (int c = 0; c < dim; ++c)
              for (int d = 0; d < dim; ++d) {
                double v = gx[i * dim + d] * gx[j * dim + c];
                if (c == d) v += dot;
                sh.A[(size_t)(i * dim + c) * nlv + (j * dim + d)] += w * nu * v;
              }
          }
        // B[q,(j,d)] += -w psi_q d_d phi_j
        const double* pq = &php[(size_t)q * nbp];
        for (int p = 0; p < nbp; ++p)
          for (int j = 0; j < nbv; ++j)
            for (int d = 0; d < dim; ++d) sh.B[(size_t)p * nlv + j * dim + d] -= w * pq[p] * gx[j * dim + d];
      }
      shapes.push_back(std::move(sh));
      hit = shapes.end() - 1;
    }
    const std::vector<double>& Aloc = hit->A;
    const std::vector<double>& Bloc = hit->B;
    std::fill(Floc.begin(), Floc.end(), 0.0);
    for (int q = 0; q < nq && with_rhs; ++q) {
      const double w = rule.w[q] * adet;
      {
        double x[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) {
          double s = C.v[0][d] / (double)unit;
          for (int i = 1; i <= dim; ++i) s += J[d][i - 1] * rule.lam[q * (dim + 1) + i];
          x[d] = s;
        }
        double f[3];
        field_f(pr, x, f);
        const double* vq = &phv[(size_t)q * nbv];
        for (int i = 0; i < nbv; ++i)
          for (int c = 0; c < dim; ++c) Floc[i * dim + c] += w * f[c] * vq[i];
      }
    }
    const int* vd = &cvd[(size_t)e * nlv];
    const int* pd = &cpd[(size_t)e * nbp];
    // Dirichlet data: nodal values of the exact velocity at boundary nodes
    if (with_rhs) {
      for (int j = 0; j < nbv; ++j) {
        if (vd[j * dim] >= 0) continue;
        int G[3];
        node_lattice(C, vb.nodes[j], dim, G);
        double x[3];
        for (int d = 0; d < dim; ++d) x[d] = (double)G[d] / (k * unit);
        field_u(pr, x, &uD[j * dim]);
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

// Load vector <f, v> of the smooth random forcing on the free DoFs of a 2D
// level with zero boundary velocity (no lifting term), made consistent.
// Only the forcing is integrated (no matrix), with sin(a pi x) and
// sin(b pi y) tabulated per quadrature point; the per-point value is summed
// in the same (a, b) order as the general path, so both give the same bits.
void assemble_random_load(int family, int k, int n, int n_modes, const double* coeffs, double* out) {
  LevelHost L;
  L.dim = 2;
  L.k = k;
  L.n = n;
  L.family = family;
  setup_mesh(L);
  const int unit = L.unit;
  const Basis vb = make_basis(2, k);
  const int nbv = vb.size();
  const SimplexRule rule = simplex_rule(2, k + 3);
  const int nq = rule.npts, M = n_modes;
  std::vector<double> phv((size_t)nq * nbv);
  for (int q = 0; q < nq; ++q) {
    double kl[3];
    for (int i = 0; i < 3; ++i) kl[i] = k * rule.lam[q * 3 + i];
    vb.eval(kl, &phv[(size_t)q * nbv]);
  }
  std::vector<double> b(L.N, 0.0), sx(M + 1), sy(M + 1), Floc(2 * nbv);
  for (const Cell& C : L.cells) {
    double J[2][2];
    for (int d = 0; d < 2; ++d)
      for (int i = 0; i < 2; ++i) J[d][i] = (double)(C.v[i + 1][d] - C.v[0][d]) / unit;
    const double adet = std::fabs(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
    std::fill(Floc.begin(), Floc.end(), 0.0);
    for (int q = 0; q < nq; ++q) {
      double x[2];
      for (int d = 0; d < 2; ++d) {
        double s = C.v[0][d] / (double)unit;
        for (int i = 1; i <= 2; ++i) s += J[d][i - 1] * rule.lam[q * 3 + i];
        x[d] = s;
      }
      for (int a = 1; a <= M; ++a) {
        sx[a] = std::sin(a * PI * x[0]);
        sy[a] = std::sin(a * PI * x[1]);
      }
      double f[2];
      for (int cc = 0; cc < 2; ++cc) {
        double s = 0.0;
        for (int a = 1; a <= M; ++a)
          for (int bb = 1; bb <= M; ++bb)
            s += coeffs[(cc * M + (a - 1)) * M + (bb - 1)] * sx[a] * sy[bb] / (double)(a * a + bb * bb);
        f[cc] = s;
      }
      const double w = rule.w[q] * adet;
      const double* vq = &phv[(size_t)q * nbv];
      for (int i = 0; i < nbv; ++i)
        for (int cc = 0; cc < 2; ++cc) Floc[i * 2 + cc] += w * f[cc] * vq[i];
    }
    for (int j = 0; j < nbv; ++j) {
      int G[3];
      node_lattice(C, vb.nodes[j], 2, G);
      const int d0 = L.vel_dof(G, 0);
      if (d0 < 0) continue;
      b[d0] += Floc[j * 2];
      b[d0 + 1] += Floc[j * 2 + 1];
    }
  }
  // pressure rows carry no load; the constant-pressure projection leaves b unchanged
  std::copy(b.begin(), b.end(), out);
}

// ---------------------------------------------------------------- prolongation
// Fine lattice point G (units 1/(kk nf)), nf = 2 nc.  The containing coarse
// cell is found from the structured mesh; barycentric coordinates are exact
// multiples of 1/(2 kk), so kk * lambda is an exact half-integer and the
// interpolation weights that vanish are exact zeros (dropped).
static void locate(int dim, int nc, int kk, const int* G, Cell& cell, double* klam) {
  const int span = 2 * kk;  // fine lattice points per coarse cell edge
  int base[3], off[3];
  for (int d = 0; d < dim; ++d) {
    int i = G[d] / span;
    if (i >= nc) i = nc - 1;
    base[d] = i;
    off[d] = G[d] - i * span;  // 0..span
  }
  if (dim == 2) {
    const int i = base[0], j = base[1];
    if (off[0] + off[1] <= span) {  // lower triangle (BL, BR, TL)
      cell = {{{i, j, 0}, {i + 1, j, 0}, {i, j + 1, 0}, {0, 0, 0}}};
      klam[0] = 0.5 * (span - off[0] - off[1]);
      klam[1] = 0.5 * off[0];
      klam[2] = 0.5 * off[1];
    } else {  // upper triangle (TR, TL, BR)
      cell = {{{i + 1, j + 1, 0}, {i, j + 1, 0}, {i + 1, j, 0}, {0, 0, 0}}};
      klam[0] = 0.5 * (off[0] + off[1] - span);
      klam[1] = 0.5 * (span - off[0]);
      klam[2] = 0.5 * (span - off[1]);
    }
  } else {
    // Kuhn tetrahedron of the axis ordering with off[p0] >= off[p1] >= off[p2]
    int p[3] = {0, 1, 2};
    std::stable_sort(p, p + 3, [&](int a, int b) { return off[a] > off[b]; });
    int v[3] = {base[0], base[1], base[2]};
    for (int d = 0; d < 3; ++d) cell.v[0][d] = v[d];
    for (int s = 0; s < 3; ++s) {
      v[p[s]] += 1;
      for (int d = 0; d < 3; ++d) cell.v[s + 1][d] = v[d];
    }
    klam[0] = 0.5 * (span - off[p[0]]);
    klam[1] = 0.5 * (off[p[0]] - off[p[1]]);
    klam[2] = 0.5 * (off[p[1]] - off[p[2]]);
    klam[3] = 0.5 * off[p[2]];
  }
}

void build_prolongation(const LevelHost& C, LevelHost& F) {
  if (F.family == VK_SV) {
    build_prolongation_sv(C, F);
    return;
  }
  if (F.family == VK_TH_QUAD) {
    build_prolongation_quad(C, F);
    return;
  }
  if (F.family == VK_BDM) {
    build_prolongation_bdm(C, F);
    return;
  }
  const int dim = F.dim;
  Csr P;
  P.nrows = F.N;
  P.ncols = C.N;
  P.rowptr.assign(F.N + 1, 0);
  std::vector<std::vector<std::pair<int, double>>> rows(F.N);
  for (int part = 0; part < 2; ++part) {
    const int kk = part == 0 ? F.k : F.k - 1;
    const Basis cb = make_basis(dim, kk);
    const int M = kk * F.n;
    int total = 1;
    for (int d = 0; d < dim; ++d) total *= (M + 1);
    std::vector<double> phi(cb.size());
    for (int idx = 0; idx < total; ++idx) {
      int G[3] = {0, 0, 0}, r = idx;
      for (int d = 0; d < dim; ++d) {
        G[d] = r % (M + 1);
        r /= (M + 1);
      }
      int frow0;
      if (part == 0) {
        frow0 = F.vel_dof(G, 0);
        if (frow0 < 0) continue;
      } else {
        frow0 = F.pres_dof(G);
      }
      Cell cell;
      double klam[4];
      locate(dim, C.n, kk, G, cell, klam);
      cb.eval(klam, phi.data());
      for (int j = 0; j < cb.size(); ++j) {
        if (phi[j] == 0.0) continue;
        int CG[3];
        node_lattice(cell, cb.nodes[j], dim, CG);
        if (part == 0) {
          if (C.vel_dof(CG, 0) < 0) continue;
          for (int c = 0; c < dim; ++c) rows[frow0 + c].push_back({C.vel_dof(CG, c), phi[j]});
        } else {
          rows[frow0].push_back({C.pres_dof(CG), phi[j]});
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

void dof_coords(const LevelHost& L, double* xyz, int* kind) {
  if (L.family == VK_SV) {
    dof_coords_sv(L, xyz, kind);
    return;
  }
  if (L.family == VK_BDM) {
    dof_coords_bdm(L, xyz, kind);
    return;
  }
  const int dim = L.dim, Mv = L.k * L.n, Mp = (L.k - 1) * L.n;
  const int nint = L.nvel / dim;
  for (int idx = 0; idx < nint; ++idx) {
    int r = idx;
    double x[3];
    for (int d = 0; d < dim; ++d) {
      x[d] = (double)(r % (Mv - 1) + 1) / Mv;
      r /= (Mv - 1);
    }
    for (int c = 0; c < dim; ++c) {
      for (int d = 0; d < dim; ++d) xyz[(size_t)(dim * idx + c) * dim + d] = x[d];
      kind[dim * idx + c] = c;
    }
  }
  for (int idx = 0; idx < L.npres; ++idx) {
    int r = idx;
    for (int d = 0; d < dim; ++d) {
      xyz[(size_t)(L.nvel + idx) * dim + d] = (double)(r % (Mp + 1)) / Mp;
      r /= (Mp + 1);
    }
    kind[L.nvel + idx] = dim;
  }
}

// ---------------------------------------------------------------- coarsest level
std::vector<double> bordered_inverse(const LevelHost& L) {
  const int N = L.N, M = N + 1;
  std::vector<double> A((size_t)M * M, 0.0);
  for (int r = 0; r < N; ++r)
    for (int q = L.K.rowptr[r]; q < L.K.rowptr[r + 1]; ++q) A[(size_t)r * M + L.K.col[q]] = L.K.val[q];
  const double zv = 1.0 / std::sqrt((double)L.npres);
  for (int r = L.nvel; r < N; ++r) {
    A[(size_t)r * M + N] = zv;
    A[(size_t)N * M + r] = zv;
  }
  // Gauss-Jordan inversion with partial pivoting (row swaps undone as column
  // swaps at the end).  A pivot below M * eps * max|a| means the coarsest
  // system is singular beyond the constant pressure (e.g. spurious pressure
  // modes on a too coarse mesh) and is reported instead of inverted.
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  const double tiny = M * 2.220446049250313e-16 * amax;
  std::vector<int> perm(M);
  // Blocked by panels of B pivots, the same pivots and updates as the column-by-column
  // algorithm: the panel (all rows, B columns) is eliminated step by step (pivot search on the
  // current panel column, full-row swaps); then, with D the pivot rows of the panel as they were
  // before (C the other rows) and R the pivot rows outside the panel,
  //   pivot rows -> D^{-1} R,   other rows -> E - C D^{-1} R      (E: their columns outside the panel)
  // with the trailing product split over host threads by rows (each entry summed in panel order,
  // independent of the thread count).
  constexpr int B = 32;
  const int nth = std::max(1, std::min<int>({16, (int)std::thread::hardware_concurrency(), M / 64}));
  std::vector<double> P0((size_t)M * B), Rn((size_t)B * M);
  for (int c0 = 0; c0 < M; c0 += B) {
    const int cb = std::min(B, M - c0);
    for (int r = 0; r < M; ++r)
      for (int t = 0; t < cb; ++t) P0[(size_t)r * B + t] = A[(size_t)r * M + c0 + t];
    for (int sidx = 0; sidx < cb; ++sidx) {
      const int c = c0 + sidx;
      int p = c;
      double best = std::fabs(A[(size_t)c * M + c]);
      for (int r = c + 1; r < M; ++r) {
        const double v = std::fabs(A[(size_t)r * M + c]);
        if (v > best) { best = v; p = r; }
      }
      require(best > tiny, VK_ESINGULAR, "coarsest bordered matrix is singular (refine the coarsest mesh)");
      perm[c] = p;
      if (p != c) {
        for (int j = 0; j < M; ++j) std::swap(A[(size_t)c * M + j], A[(size_t)p * M + j]);
        for (int t = 0; t < B; ++t) std::swap(P0[(size_t)c * B + t], P0[(size_t)p * B + t]);
      }
      double* ac = &A[(size_t)c * M + c0];  // the pivot row's panel part
      const double piv = ac[sidx];
      for (int t = 0; t < cb; ++t) ac[t] = t == sidx ? 1.0 / piv : ac[t] / piv;
      for (int r = 0; r < M; ++r) {
        if (r == c) continue;
        double* ar = &A[(size_t)r * M + c0];
        const double f = ar[sidx];
        if (f == 0.0) continue;
        for (int t = 0; t < cb; ++t) ar[t] = t == sidx ? -f * ac[t] : ar[t] - f * ac[t];
      }
    }
    // Rn = D^{-1} R: the panel rows of the pivots now hold D^{-1}
    for (int sidx = 0; sidx < cb; ++sidx)
      for (int j = 0; j < M; ++j) {
        if (j >= c0 && j < c0 + cb) continue;
        double acc = 0.0;
        for (int t = 0; t < cb; ++t) acc += A[(size_t)(c0 + sidx) * M + c0 + t] * A[(size_t)(c0 + t) * M + j];
        Rn[(size_t)sidx * M + j] = acc;
      }
    auto trailing = [&](int t0) {
      const int r0 = (int)((int64_t)M * t0 / nth), r1 = (int)((int64_t)M * (t0 + 1) / nth);
      for (int r = r0; r < r1; ++r) {
        if (r >= c0 && r < c0 + cb) continue;
        double* ar = &A[(size_t)r * M];
        for (int t = 0; t < cb; ++t) {
          const double f = P0[(size_t)r * B + t];
          if (f == 0.0) continue;
          const double* rn = &Rn[(size_t)t * M];
          for (int j = 0; j < c0; ++j) ar[j] -= f * rn[j];
          for (int j = c0 + cb; j < M; ++j) ar[j] -= f * rn[j];
        }
      }
    };
    {
      std::vector<std::thread> pool;
      for (int t = 1; t < nth; ++t) pool.emplace_back(trailing, t);
      trailing(0);
      for (auto& th : pool) th.join();
    }
    for (int sidx = 0; sidx < cb; ++sidx)
      for (int j = 0; j < M; ++j)
        if (j < c0 || j >= c0 + cb) A[(size_t)(c0 + sidx) * M + j] = Rn[(size_t)sidx * M + j];
  }
  for (int c = M - 1; c >= 0; --c)
    if (perm[c] != c)
      for (int r = 0; r < M; ++r) std::swap(A[(size_t)r * M + c], A[(size_t)r * M + perm[c]]);
  std::vector<double> out((size_t)N * N);
  for (int r = 0; r < N; ++r)
    for (int c = 0; c < N; ++c) out[(size_t)r * N + c] = A[(size_t)r * M + c];
  return out;
}

}  // namespace vk
