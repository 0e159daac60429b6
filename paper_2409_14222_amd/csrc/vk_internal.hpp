// Internal data structures of the vk library (host side).
#pragma once

#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/vk.h"

namespace vk {

struct Error : std::runtime_error {
  vk_status code;
  Error(vk_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

inline void require(bool ok, vk_status code, const std::string& msg) {
  if (!ok) throw Error(code, msg);
}

struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int> rowptr, col;
  std::vector<double> val;
  int64_t nnz() const { return (int64_t)col.size(); }
};

Csr transpose(const Csr& a);
// starts of the maximal runs (capped at `cap` rows) of consecutive rows with identical column lists,
// followed by nrows: a many-right-hand-side product reads each input row once per run
std::vector<int> row_groups(const Csr& a, int cap);

// Rows gathered into groups that share one ascending column list (the union of their rows'
// lists, padded to a multiple of 16 with its last column): a many-right-hand-side product loads
// each listed input row once for the whole group and multiplies a stored zero where a row has no
// entry.  Values are dense per group, [step of 4 columns][row of the group][4].
struct UnionGroups {
  std::vector<int> gptr, grow;  // group g: rows grow[gptr[g] .. gptr[g + 1])
  std::vector<int> uptr, ucol;  // its columns ucol[uptr[g] .. uptr[g + 1])
  std::vector<int64_t> voff;    // offset of its value block
  int64_t nval = 0;             // total values
  int ngroups() const { return (int)gptr.size() - 1; }
};
constexpr int kUnionMaxRows = 16;     // rows per group (one block of the 16 x 16 matrix-core product)
constexpr int kUnionMaxCols = 96;     // columns before padding (a single run may exceed it alone)
constexpr double kUnionMaxFill = 2.0;  // stored values over the group's nonzeros
// Groups of a's rows: the runs of `runs` (row_groups) taken in `run_order`, each appended to the
// open group while the group stays within the three limits above.  Rows of a must have ascending
// column lists.
UnionGroups union_groups(const Csr& a, const std::vector<int>& runs, const std::vector<int>& run_order);
// the dense value blocks of `g` (g.nval values)
std::vector<double> union_values(const Csr& a, const UnionGroups& g);
// run indices of `runs` in the order their rows first appear in the patch lists (patch id order),
// then the runs no patch touches
std::vector<int> runs_in_patch_order(const std::vector<int>& runs, const std::vector<int>& pptr,
                                     const std::vector<int>& pdofs);

// ---------------------------------------------------------------- FEM kernels (host_fem.cpp)
// Collapsed Gauss-Legendre rule on the reference simplex with q points per
// direction: points as barycentric coordinates (dim+1 per point) and weights
// summing to the reference volume (1/2 or 1/6).
struct SimplexRule {
  int dim = 0, npts = 0;
  std::vector<double> lam;  // npts * (dim+1)
  std::vector<double> w;    // npts
};
SimplexRule simplex_rule(int dim, int q);

// Equispaced P_k Lagrange basis in barycentric (Silvester) form.  Node a is a
// multi-index of dim+1 non-negative integers summing to k; the basis function
// is prod_i L_{a_i}(lambda_i), L_m(t) = prod_{j<m} (k t - j) / (j + 1).
struct Basis {
  int dim = 0, k = 0;
  std::vector<std::vector<int>> nodes;  // multi-indices (dim+1 entries)
  int size() const { return (int)nodes.size(); }
  // values phi[j] at barycentric point lam (k * lam_i may be given exactly)
  void eval(const double* klam, double* phi) const;
  // derivatives d phi_j / d lambda_i (nbasis x (dim+1)), at barycentric lam
  void dlam(const double* lam, double* d) const;
};
Basis make_basis(int dim, int k);

// ---------------------------------------------------------------- levels (host_assemble.cpp)
struct Cell {
  int v[4][3];  // vertex lattice coordinates (units 1/n), dim+1 vertices
};

struct LevelHost {
  int dim = 2, k = 2, n = 0;
  int family = VK_TH;        // VK_TH, VK_SV (barycentric sub-cells), VK_TH_QUAD or VK_BDM
  int unit = 0;              // cell vertex coordinates are integers in units of 1/unit (n, or 3n for VK_SV)
  std::vector<int> vmap;     // VK_SV: velocity lattice point y * (k unit + 1) + x -> interior node or -1
  int N = 0, nvel = 0, npres = 0;
  std::vector<Cell> cells;
  Csr K;
  Csr P, PT;                 // prolongation from level-1 (rows: this level) and its transpose
  // runs of consecutive rows with identical column lists (at most 8 rows): starts, then the row count
  std::vector<int> kgrp, pgrp, ptgrp;
  // K's rows in union groups for more than 8 right-hand sides (built on first need, levels >= 1)
  mutable UnionGroups kunion;
  mutable bool kunion_built = false;
  std::vector<double> b;     // right-hand side (finest level only)
  // patches (host_patches.cpp)
  std::vector<int> pptr, pdofs;   // patch i: pdofs[pptr[i] .. pptr[i+1])
  std::vector<int> dptr, dslot;   // DoF d: slots dslot[dptr[d] .. dptr[d+1]) ascending patch id
  std::vector<double> scale;      // smoother weight: (omega, or 1 for Chebyshev) x (1 / multiplicity, or 1)
  std::vector<int> order;         // patch processing order (largest first)
  std::vector<int64_t> inv_off;   // element offset of each patch inverse (indexed by patch id)
  int64_t inv_elems = 0;
  // the same for the symmetric tiled storage: the 8x8 tiles (I, J), I >= J, of the inverse,
  // tile I (I + 1) / 2 + J, each column-major (64 elements)
  std::vector<int64_t> inv_off_tri;
  int64_t inv_elems_tri = 0;
  int max_n = 0;
  int64_t sum_n2 = 0;

  int vel_dof(const int* G, int c) const;  // -1 on the boundary
  int pres_dof(const int* G) const;         // VK_TH only
  // VK_SV: pressure DoF of local node (a1, a2) of sub-cell e (node V0 + (a1 E1 + a2 E2) / (k - 1))
  int sv_pres_dof(int e, int a1, int a2) const;
};

struct Problem {
  vk_problem p;
  std::vector<double> coeffs;
};

// cells, DoF numbering and counts of a level (dim, k, n, family set by the caller)
void setup_mesh(LevelHost& L);
void build_level(LevelHost& L, const Problem& pr, bool with_rhs);
void cell_dof_maps(const LevelHost& L, const Basis& vb, const Basis& pb, std::vector<int>& cvd, std::vector<int>& cpd);
void field_u(const Problem& pr, const double* x, double* u);
void field_grad_u(const Problem& pr, const double* x, double* g);
void field_f(const Problem& pr, const double* x, double* f);
// relative H^1 velocity error and mean-free L^2 pressure error of x (free DoFs of L)
void solution_errors(const LevelHost& L, const Problem& pr, const double* x, double* e_u, double* e_p);
// Gauss-Legendre rule on [0, 1] (host_fem.cpp)
void gauss_legendre_01(int q, std::vector<double>& x, std::vector<double>& w);
// quadrilateral Taylor-Hood (host_quad.cpp)
void setup_mesh_quad(LevelHost& L);
void build_level_quad(LevelHost& L, const Problem& pr, bool with_rhs);
void build_prolongation_quad(const LevelHost& coarse, LevelHost& fine);
void build_patches_quad(LevelHost& L, double omega, int store);
void solution_errors_quad(const LevelHost& L, const Problem& pr, const double* x, double* e_u, double* e_p);
void build_prolongation(const LevelHost& coarse, LevelHost& fine);
void build_patches(LevelHost& L, int construct, double omega, int store);
// ordering, inverse map, relaxation scale and inverse storage of collected patch DoF lists
void finalize_patches(LevelHost& L, std::vector<std::vector<int>>& patches, double omega, int store);
void dof_coords(const LevelHost& L, double* xyz, int* kind);
// load vector of the random forcing (zero boundary velocity) on the finest-level numbering of (family, k, n)
void assemble_random_load(int family, int k, int n, int n_modes, const double* coeffs, double* out);

// (BDM_k, dP_{k-1}) interior-penalty levels (host_bdm.cpp)
void setup_mesh_bdm(LevelHost& L);
void build_level_bdm(LevelHost& L, const Problem& pr, bool with_rhs);
void build_prolongation_bdm(const LevelHost& coarse, LevelHost& fine);
void build_patches_bdm(LevelHost& L, double omega, int store);
void solution_errors_bdm(const LevelHost& L, const Problem& pr, const double* x, double* e_u, double* e_p);
void dof_coords_bdm(const LevelHost& L, double* xyz, int* kind);

// Scott-Vogelius levels (host_sv.cpp)
void setup_mesh_sv(LevelHost& L);
void build_prolongation_sv(const LevelHost& coarse, LevelHost& fine);
void build_patches_macro(LevelHost& L, double omega, int store);
void dof_coords_sv(const LevelHost& L, double* xyz, int* kind);

// Top-left N x N block of the inverse of the bordered matrix [K z; z^T 0],
// z = constant pressure / sqrt(#pressure); row-major.
std::vector<double> bordered_inverse(const LevelHost& L);
// eigenvalues of the upper Hessenberg n x n matrix H (row-major); false on
// non-finite input or no convergence
bool hessenberg_eigs(int n, const double* H, std::vector<std::complex<double>>& ev);

}  // namespace vk
