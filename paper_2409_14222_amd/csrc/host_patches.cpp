// Composite ("topological") Vanka patches, Sec. 3.1.
//
// One patch per topological entity that carries pressure DoFs of P_{k-1}:
// vertices, edge interiors (k >= 3) and cell interiors (k >= 4 in 2D).  A
// patch holds the entity's pressure DoFs and every free velocity DoF on the
// closure of the entity's star (the cells around a vertex, the one or two
// cells of an edge, the cell itself).  DoF lists are ascending; patches are
// ordered by their smallest pressure DoF.  The STAR option keeps vertex
// patches only and adds the pressure DoFs of the open vertex star (vertex,
// incident edge interiors, incident cell interiors).
//
// The relaxation weights (a reading of Algorithm 1's weighting operators):
// DoF d is scaled by omega / mult(d), mult = number of patches containing d.
#include <algorithm>
#include <map>

#include "vk_internal.hpp"

namespace vk {

namespace {

struct Builder {
  const LevelHost& L;
  int k, n, dim;
  Basis vb;
  explicit Builder(const LevelHost& l) : L(l), k(l.k), n(l.n), dim(l.dim), vb(make_basis(l.dim, l.k)) {}

  // all free velocity DoFs of a cell's closure
  void cell_vel(const Cell& c, std::vector<int>& out) const {
    for (const auto& a : vb.nodes) {
      int G[3];
      for (int d = 0; d < dim; ++d) {
        int g = 0;
        for (int i = 0; i <= dim; ++i) g += a[i] * c.v[i][d];
        G[d] = g;
      }
      const int d0 = L.vel_dof(G, 0);
      if (d0 < 0) continue;
      for (int c2 = 0; c2 < dim; ++c2) out.push_back(d0 + c2);
    }
  }
};

inline Cell tri_lower(int i, int j) { return {{{i, j, 0}, {i + 1, j, 0}, {i, j + 1, 0}, {0, 0, 0}}}; }
inline Cell tri_upper(int i, int j) { return {{{i + 1, j + 1, 0}, {i, j + 1, 0}, {i + 1, j, 0}, {0, 0, 0}}}; }

}  // namespace

void build_patches(LevelHost& L, int construct, double omega, int store) {
  if (construct == VK_PATCH_MACRO) {
    require(L.family == VK_SV, VK_EINVAL, "macro patches belong to Scott-Vogelius levels");
    build_patches_macro(L, omega, store);
    return;
  }
  if (L.family == VK_BDM) {
    require(construct == VK_PATCH_EXTENDED, VK_EINVAL, "BDM levels use extended cell patches");
    build_patches_bdm(L, omega, store);
    return;
  }
  require(construct != VK_PATCH_EXTENDED, VK_EINVAL, "extended cell patches belong to BDM levels");
  if (L.family == VK_TH_QUAD) {
    require(construct == VK_PATCH_COMPOSITE, VK_EINVAL, "quadrilateral levels use composite patches");
    build_patches_quad(L, omega, store);
    return;
  }
  require(L.family == VK_TH, VK_EINVAL, "Scott-Vogelius levels use macro patches");
  Builder B(L);
  const int n = L.n, k = L.k, km = k - 1;
  std::vector<std::vector<int>> patches;

  auto finish = [&](std::vector<int> v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    patches.push_back(std::move(v));
  };

  if (L.dim == 2) {
    auto pres = [&](int a, int b) {
      int G[2] = {a, b};
      return L.pres_dof(G);
    };
    auto inside = [&](int i, int j) { return i >= 0 && j >= 0 && i < n && j < n; };
    // cells around vertex (i, j): lower of square (i,j); both of (i-1,j) and (i,j-1); upper of (i-1,j-1)
    auto vertex_cells = [&](int i, int j, std::vector<Cell>& cs) {
      if (inside(i, j)) cs.push_back(tri_lower(i, j));
      if (inside(i - 1, j)) { cs.push_back(tri_lower(i - 1, j)); cs.push_back(tri_upper(i - 1, j)); }
      if (inside(i, j - 1)) { cs.push_back(tri_lower(i, j - 1)); cs.push_back(tri_upper(i, j - 1)); }
      if (inside(i - 1, j - 1)) cs.push_back(tri_upper(i - 1, j - 1));
    };
    // interior pressure DoFs of the edge from vertex p to vertex q
    auto edge_pres = [&](int pi, int pj, int qi, int qj, std::vector<int>& out) {
      for (int t = 1; t < km; ++t) out.push_back(pres(km * pi + t * (qi - pi), km * pj + t * (qj - pj)));
    };
    auto cell_pres = [&](const Cell& c, std::vector<int>& out) {
      for (int a1 = 1; a1 < km; ++a1)
        for (int a2 = 1; a1 + a2 < km; ++a2) {
          const int a0 = km - a1 - a2;
          out.push_back(pres(a0 * c.v[0][0] + a1 * c.v[1][0] + a2 * c.v[2][0],
                             a0 * c.v[0][1] + a1 * c.v[1][1] + a2 * c.v[2][1]));
        }
    };

    std::vector<Cell> cs;
    for (int j = 0; j <= n; ++j)
      for (int i = 0; i <= n; ++i) {
        std::vector<int> v;
        cs.clear();
        vertex_cells(i, j, cs);
        for (const Cell& c : cs) B.cell_vel(c, v);
        v.push_back(pres(km * i, km * j));
        if (construct == VK_PATCH_STAR) {
          // open star: incident edge interiors and incident cell interiors
          const int nb[6][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {-1, 1}, {1, -1}};
          for (auto& o : nb) {
            const int qi = i + o[0], qj = j + o[1];
            if (qi < 0 || qj < 0 || qi > n || qj > n) continue;
            edge_pres(i, j, qi, qj, v);
          }
          for (const Cell& c : cs) cell_pres(c, v);
        }
        finish(std::move(v));
      }
    if (construct == VK_PATCH_COMPOSITE && k >= 3) {
      // edges: horizontal (i,j)-(i+1,j), vertical (i,j)-(i,j+1), diagonal (i,j+1)-(i+1,j)
      for (int j = 0; j <= n; ++j)
        for (int i = 0; i < n; ++i) {
          std::vector<int> v;
          if (j < n) B.cell_vel(tri_lower(i, j), v);
          if (j > 0) B.cell_vel(tri_upper(i, j - 1), v);
          edge_pres(i, j, i + 1, j, v);
          finish(std::move(v));
        }
      for (int j = 0; j < n; ++j)
        for (int i = 0; i <= n; ++i) {
          std::vector<int> v;
          if (i < n) B.cell_vel(tri_lower(i, j), v);
          if (i > 0) B.cell_vel(tri_upper(i - 1, j), v);
          edge_pres(i, j, i, j + 1, v);
          finish(std::move(v));
        }
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          std::vector<int> v;
          B.cell_vel(tri_lower(i, j), v);
          B.cell_vel(tri_upper(i, j), v);
          edge_pres(i, j + 1, i + 1, j, v);
          finish(std::move(v));
        }
    }
    if (construct == VK_PATCH_COMPOSITE && k >= 4) {
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          for (int up = 0; up < 2; ++up) {
            const Cell c = up ? tri_upper(i, j) : tri_lower(i, j);
            std::vector<int> v;
            B.cell_vel(c, v);
            cell_pres(c, v);
            finish(std::move(v));
          }
    }
  } else {
    require(k == 2, VK_EINVAL, "3D patches are implemented for P2-P1 (vertex pressures only)");
    // vertex -> incident cells from the cell list
    const int nv1 = n + 1;
    std::vector<std::vector<int>> vc((size_t)nv1 * nv1 * nv1);
    for (int e = 0; e < (int)L.cells.size(); ++e)
      for (int i = 0; i < 4; ++i) {
        const int* v = L.cells[e].v[i];
        vc[((size_t)v[2] * nv1 + v[1]) * nv1 + v[0]].push_back(e);
      }
    for (int z = 0; z <= n; ++z)
      for (int y = 0; y <= n; ++y)
        for (int x = 0; x <= n; ++x) {
          std::vector<int> v;
          for (int e : vc[((size_t)z * nv1 + y) * nv1 + x]) B.cell_vel(L.cells[e], v);
          int G[3] = {x, y, z};
          v.push_back(L.pres_dof(G));
          finish(std::move(v));
        }
  }

  finalize_patches(L, patches, omega, store);
}

void finalize_patches(LevelHost& L, std::vector<std::vector<int>>& patches, double omega, int store) {
  // order by smallest pressure DoF
  std::vector<std::pair<int, int>> key(patches.size());
  for (size_t p = 0; p < patches.size(); ++p) {
    int m = L.N;
    for (int d : patches[p])
      if (d >= L.nvel) m = std::min(m, d);
    key[p] = {m, (int)p};
  }
  std::sort(key.begin(), key.end());
  const int J = (int)patches.size();
  L.pptr.assign(J + 1, 0);
  L.pdofs.clear();
  L.max_n = 0;
  L.sum_n2 = 0;
  for (int i = 0; i < J; ++i) {
    const auto& v = patches[key[i].second];
    L.pdofs.insert(L.pdofs.end(), v.begin(), v.end());
    L.pptr[i + 1] = (int)L.pdofs.size();
    L.max_n = std::max(L.max_n, (int)v.size());
    L.sum_n2 += (int64_t)v.size() * v.size();
  }
  // inverse map: DoF -> slots, ascending patch id
  L.dptr.assign(L.N + 1, 0);
  for (int d : L.pdofs) L.dptr[d + 1]++;
  for (int d = 0; d < L.N; ++d) L.dptr[d + 1] += L.dptr[d];
  L.dslot.assign(L.pdofs.size(), 0);
  std::vector<int> pos(L.dptr.begin(), L.dptr.end() - 1);
  for (int i = 0; i < J; ++i)
    for (int s = L.pptr[i]; s < L.pptr[i + 1]; ++s) L.dslot[pos[L.pdofs[s]]++] = s;
  L.scale.assign(L.N, 0.0);
  for (int d = 0; d < L.N; ++d) {
    const int mult = L.dptr[d + 1] - L.dptr[d];
    require(mult > 0, VK_EINVAL, "patches do not cover every DoF");
    L.scale[d] = omega / mult;
  }
  // processing order: largest patches first (stable in patch id)
  L.order.resize(J);
  for (int i = 0; i < J; ++i) L.order[i] = i;
  std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) {
    return (L.pptr[a + 1] - L.pptr[a]) > (L.pptr[b + 1] - L.pptr[b]);
  });
  // inverse storage: column-major, leading dimension rounded to the rows one
  // lane loads per 16-byte access (2 doubles / 4 floats), laid out in
  // processing order, 32-byte aligned
  const int rpl = store == VK_STORE_FP32 ? 4 : 2;
  L.inv_off.assign(J, 0);
  int64_t off = 0;
  for (int t = 0; t < J; ++t) {
    const int p = L.order[t];
    const int nn = L.pptr[p + 1] - L.pptr[p];
    const int ld = (nn + rpl - 1) / rpl * rpl;
    L.inv_off[p] = off;
    off += (int64_t)ld * nn;
    off = (off + 3) / 4 * 4;
  }
  L.inv_elems = off;
  // symmetric tiled storage (one right-hand side): lower-triangular 8x8 tiles, same order
  L.inv_off_tri.assign(J, 0);
  off = 0;
  for (int t = 0; t < J; ++t) {
    const int p = L.order[t];
    const int nn = L.pptr[p + 1] - L.pptr[p];
    const int nb = (nn + 7) / 8, nvr = (nn - 8 * (nb - 1) + rpl - 1) / rpl;
    L.inv_off_tri[p] = off;
    // full 8 x 8 tiles above the last block row, then its tiles cut to nvr chunks of rpl rows
    off += (int64_t)(nb - 1) * nb / 2 * 64 + (int64_t)nb * 8 * rpl * nvr;
  }
  L.inv_elems_tri = off;
}

}  // namespace vk
