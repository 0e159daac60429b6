// Internal data structures of the vk library (host side).
#pragma once

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
  int N = 0, nvel = 0, npres = 0;
  std::vector<Cell> cells;
  Csr K;
  Csr P, PT;                 // prolongation from level-1 (rows: this level) and its transpose
  std::vector<double> b;     // right-hand side (finest level only)
  // patches (host_patches.cpp)
  std::vector<int> pptr, pdofs;   // patch i: pdofs[pptr[i] .. pptr[i+1])
  std::vector<int> dptr, dslot;   // DoF d: slots dslot[dptr[d] .. dptr[d+1]) ascending patch id
  std::vector<double> scale;      // omega / multiplicity
  std::vector<int> order;         // patch processing order (largest first)
  std::vector<int64_t> inv_off;   // element offset of each patch inverse (indexed by patch id)
  int64_t inv_elems = 0;
  int max_n = 0;
  int64_t sum_n2 = 0;

  int vel_dof(const int* G, int c) const;  // -1 on the boundary
  int pres_dof(const int* G) const;
};

struct Problem {
  vk_problem p;
  std::vector<double> coeffs;
};

void build_level(LevelHost& L, const Problem& pr, bool with_rhs);
void build_prolongation(const LevelHost& coarse, LevelHost& fine);
void build_patches(LevelHost& L, int construct, double omega, int store);
void dof_coords(const LevelHost& L, double* xyz, int* kind);
void assemble_random_load(int k, int n, int n_modes, const double* coeffs, double* out);

// Top-left N x N block of the inverse of the bordered matrix [K z; z^T 0],
// z = constant pressure / sqrt(#pressure); row-major.
std::vector<double> bordered_inverse(const LevelHost& L);

}  // namespace vk
