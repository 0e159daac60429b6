// Host-side finite-element building blocks: quadrature on simplices and the
// equispaced Lagrange basis in barycentric form (Sec. 2, Taylor-Hood spaces).
#include <algorithm>
#include <iterator>
#include <cmath>

#include "vk_internal.hpp"

namespace vk {

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on the Legendre
// polynomial P_q (three-term recurrence), started from the Chebyshev-like guess
// cos(pi (i + 3/4) / (q + 1/2)).
static void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w);

void gauss_legendre_01(int q, std::vector<double>& x, std::vector<double>& w) { gauss_legendre01(q, x, w); }

static void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int m = 2; m <= q; ++m) {
        double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = t; p0 = 1.0; }
      dp = q * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    // recompute the derivative at the converged root
    double p0 = 1.0, p1 = t;
    for (int m = 2; m <= q; ++m) {
      double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = t; p0 = 1.0; }
    dp = q * (t * p1 - p0) / (t * t - 1.0);
    // map from [-1,1] (descending roots) to [0,1] ascending
    x[q - 1 - i] = 0.5 * (t + 1.0);
    w[q - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // = 0.5 * 2 / ((1-t^2) P'^2)
  }
}

SimplexRule simplex_rule(int dim, int q) {
  std::vector<double> g, gw;
  gauss_legendre01(q, g, gw);
  SimplexRule r;
  r.dim = dim;
  if (dim == 2) {
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        double s = g[i], t = g[j];
        double x = s, y = t * (1.0 - s);
        r.lam.insert(r.lam.end(), {1.0 - x - y, x, y});
        r.w.push_back(gw[i] * gw[j] * (1.0 - s));
      }
  } else {
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j)
        for (int l = 0; l < q; ++l) {
          double s = g[i], t = g[j], u = g[l];
          double x = s, y = t * (1.0 - s), z = u * (1.0 - s) * (1.0 - t);
          r.lam.insert(r.lam.end(), {1.0 - x - y - z, x, y, z});
          r.w.push_back(gw[i] * gw[j] * gw[l] * (1.0 - s) * (1.0 - s) * (1.0 - t));
        }
  }
  r.npts = (int)r.w.size();
  return r;
}

Basis make_basis(int dim, int k) {
  Basis b;
  b.dim = dim;
  b.k = k;
  // all multi-indices (a_0..a_dim) with sum k
  std::vector<int> a(dim + 1, 0);
  if (dim == 2) {
    for (int a1 = 0; a1 <= k; ++a1)
      for (int a2 = 0; a1 + a2 <= k; ++a2) b.nodes.push_back({k - a1 - a2, a1, a2});
  } else {
    for (int a1 = 0; a1 <= k; ++a1)
      for (int a2 = 0; a1 + a2 <= k; ++a2)
        for (int a3 = 0; a1 + a2 + a3 <= k; ++a3) b.nodes.push_back({k - a1 - a2 - a3, a1, a2, a3});
  }
  return b;
}

// L_m(t) with s = k t given: prod_{j<m} (s - j) / (j + 1)
static inline double lagr(int m, double s) {
  double v = 1.0;
  for (int j = 0; j < m; ++j) v *= (s - j) / (j + 1);
  return v;
}

// d/dt L_m(t) = sum_j k/(j+1) prod_{j' != j} (s - j')/(j'+1)
static inline double dlagr(int m, double s, int k) {
  double d = 0.0;
  for (int j = 0; j < m; ++j) {
    double v = (double)k / (j + 1);
    for (int jj = 0; jj < m; ++jj)
      if (jj != j) v *= (s - jj) / (jj + 1);
    d += v;
  }
  return d;
}

void Basis::eval(const double* klam, double* phi) const {
  for (int j = 0; j < size(); ++j) {
    double v = 1.0;
    for (int i = 0; i <= dim; ++i) v *= lagr(nodes[j][i], klam[i]);
    phi[j] = v;
  }
}

void Basis::dlam(const double* lam, double* d) const {
  double s[4];
  for (int i = 0; i <= dim; ++i) s[i] = k * lam[i];
  for (int j = 0; j < size(); ++j) {
    for (int i = 0; i <= dim; ++i) {
      double v = dlagr(nodes[j][i], s[i], k);
      for (int i2 = 0; i2 <= dim; ++i2)
        if (i2 != i) v *= lagr(nodes[j][i2], s[i2]);
      d[j * (dim + 1) + i] = v;
    }
  }
}

Csr transpose(const Csr& a) {
  Csr t;
  t.nrows = a.ncols;
  t.ncols = a.nrows;
  t.rowptr.assign(t.nrows + 1, 0);
  for (int c : a.col) t.rowptr[c + 1]++;
  for (int i = 0; i < t.nrows; ++i) t.rowptr[i + 1] += t.rowptr[i];
  t.col.resize(a.col.size());
  t.val.resize(a.val.size());
  std::vector<int> pos(t.rowptr.begin(), t.rowptr.end() - 1);
  for (int r = 0; r < a.nrows; ++r)
    for (int q = a.rowptr[r]; q < a.rowptr[r + 1]; ++q) {
      int c = a.col[q];
      t.col[pos[c]] = r;
      t.val[pos[c]] = a.val[q];
      pos[c]++;
    }
  return t;
}

std::vector<int> row_groups(const Csr& a, int cap) {
  std::vector<int> g;
  int r = 0;
  while (r < a.nrows) {
    g.push_back(r);
    const int b = a.rowptr[r], m = a.rowptr[r + 1] - b;
    int e = r + 1;
    while (e < a.nrows && e - r < cap && a.rowptr[e + 1] - a.rowptr[e] == m &&
           std::equal(a.col.begin() + b, a.col.begin() + b + m, a.col.begin() + a.rowptr[e]))
      ++e;
    r = e;
  }
  g.push_back(a.nrows);
  return g;
}

UnionGroups union_groups(const Csr& a, const std::vector<int>& runs, const std::vector<int>& run_order) {
  for (int r = 0; r < a.nrows; ++r)
    for (int q = a.rowptr[r] + 1; q < a.rowptr[r + 1]; ++q)
      require(a.col[q - 1] < a.col[q], VK_EINVAL, "union groups need ascending column lists");
  UnionGroups g;
  g.gptr.push_back(0);
  g.uptr.push_back(0);
  std::vector<int> cur, merged;  // the open group's column union
  int64_t cur_nnz = 0;
  auto close = [&]() {
    if (g.grow.size() == (size_t)g.gptr.back()) return;
    const int rows = (int)g.grow.size() - g.gptr.back();
    g.voff.push_back(g.nval);
    const int padded = ((int)cur.size() + 15) / 16 * 16;
    for (int i = 0; i < padded; ++i) g.ucol.push_back(cur[std::min(i, (int)cur.size() - 1)]);
    g.nval += (int64_t)padded * rows;
    g.gptr.push_back((int)g.grow.size());
    g.uptr.push_back((int)g.ucol.size());
    cur.clear();
    cur_nnz = 0;
  };
  for (const int ri : run_order) {
    const int r0 = runs[ri], r1 = runs[ri + 1];
    const int* c0 = a.col.data() + a.rowptr[r0];
    const int m = a.rowptr[r0 + 1] - a.rowptr[r0];
    merged.clear();
    std::set_union(cur.begin(), cur.end(), c0, c0 + m, std::back_inserter(merged));
    const int rows = (int)g.grow.size() - g.gptr.back() + (r1 - r0);
    const int64_t nnz = cur_nnz + (int64_t)(r1 - r0) * m;
    if (!cur.empty() && ((int)merged.size() > kUnionMaxCols || rows > kUnionMaxRows ||
                         (double)rows * (double)merged.size() > kUnionMaxFill * (double)nnz)) {
      close();
      cur.assign(c0, c0 + m);
    } else {
      cur.swap(merged);
    }
    cur_nnz += (int64_t)(r1 - r0) * m;
    for (int r = r0; r < r1; ++r) g.grow.push_back(r);
  }
  close();
  return g;
}

std::vector<double> union_values(const Csr& a, const UnionGroups& g) {
  std::vector<double> v((size_t)g.nval, 0.0);
  for (int gi = 0; gi < g.ngroups(); ++gi) {
    const int G = g.gptr[gi + 1] - g.gptr[gi];
    const int* u = g.ucol.data() + g.uptr[gi];
    double* blk = v.data() + g.voff[gi];
    for (int t = 0; t < G; ++t) {
      const int r = g.grow[g.gptr[gi] + t];
      int j = 0;  // position in the union (ascending; the padding repeats the last column, left at zero)
      for (int q = a.rowptr[r]; q < a.rowptr[r + 1]; ++q) {
        while (u[j] < a.col[q]) ++j;
        blk[(int64_t)(j / 4) * G * 4 + t * 4 + j % 4] = a.val[q];
      }
    }
  }
  return v;
}

std::vector<int> runs_in_patch_order(const std::vector<int>& runs, const std::vector<int>& pptr,
                                     const std::vector<int>& pdofs) {
  const int nruns = (int)runs.size() - 1;
  const int nrows = runs.back();
  std::vector<int> run_of(nrows);
  for (int ri = 0; ri < nruns; ++ri)
    for (int r = runs[ri]; r < runs[ri + 1]; ++r) run_of[r] = ri;
  std::vector<char> seen(nruns, 0);
  std::vector<int> order;
  order.reserve(nruns);
  for (int p = 0; p + 1 < (int)pptr.size(); ++p)
    for (int q = pptr[p]; q < pptr[p + 1]; ++q) {
      const int ri = run_of[pdofs[q]];
      if (!seen[ri]) {
        seen[ri] = 1;
        order.push_back(ri);
      }
    }
  for (int ri = 0; ri < nruns; ++ri)
    if (!seen[ri]) order.push_back(ri);
  return order;
}

}  // namespace vk
