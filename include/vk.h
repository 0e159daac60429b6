/*
 * vk.h -- C ABI of the MI355X (gfx950) matrix-full additive Vanka multigrid
 * Stokes solver.
 *
 * The method is the monolithic h-multigrid preconditioned FGMRES solver of
 * Rafiei & MacLachlan, "Achieving h- and p-robust monolithic multigrid
 * solvers for the Stokes equations": Taylor-Hood (P_k, P_{k-1}) on
 * structured triangle meshes of the unit square (Sec. 3, Case 1; Sec. 4 for
 * the mesh), and (P2, P1) on Kuhn tetrahedral meshes of the unit cube as an
 * extension.  The relaxation is additive subspace correction over composite
 * ("topological") Vanka patches (Sec. 3.1, Algorithm 1), implemented
 * matrix-full: patch submatrices are gathered from the assembled global CSR
 * matrix by DoF index lists and inverted once.
 *
 * Conventions
 *  - Every function returns vk_status: 0 = VK_OK, > 0 = warning with valid
 *    outputs, < 0 = error (outputs undefined).  vk_last_error() returns a
 *    thread-local message for the last non-zero status.  No C++ exception
 *    crosses this boundary.
 *  - Levels are numbered 0 (coarsest, n_coarse) .. n_levels-1 (finest,
 *    n_coarse * 2^(n_levels-1)).
 *  - "d_" pointers are device pointers (HIP), "h_" pointers host pointers;
 *    all are owned by the caller, who keeps them alive while a call that
 *    uses them is in flight.  Vectors at the boundary are always float64.
 *  - Device memory is owned by the caller: the library reports how many bytes
 *    it needs (vk_hierarchy_workspace_bytes), the caller allocates one buffer
 *    and binds it together with a HIP stream (vk_hierarchy_bind).  The library
 *    never allocates or frees device memory; vk_solve allocates a small pinned
 *    host buffer (2 x 3 (restart + 2) doubles) on its first call for the
 *    Hessenberg read-back, released by vk_hierarchy_destroy.  All device work
 *    is enqueued on the bound stream; calls return without synchronising
 *    unless stated.
 *  - Free-DoF numbering: velocity lattice points of the P_k lattice (spacing
 *    1/(k n)) that are not on the boundary, lexicographic with x fastest,
 *    components interleaved (dof = dim * idx + c); then all points of the
 *    P_{k-1} pressure lattice, lexicographic with x fastest.  Dirichlet
 *    velocity DoFs are eliminated (lifted into the right-hand side).
 *  - A hierarchy is not thread-safe; distinct hierarchies are independent.
 */
#ifndef VK_H
#define VK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int vk_status;

enum {
  VK_OK = 0,
  VK_NOT_CONVERGED = 1, /* solve reached maxit; outputs valid */
  VK_EINVAL = -1,       /* bad argument */
  VK_ENOMEM = -2,       /* workspace too small / host allocation failed */
  VK_EHIP = -3,         /* a HIP runtime call failed */
  VK_ESINGULAR = -4,    /* a patch matrix had a zero pivot */
  VK_ENAN = -5,         /* non-finite input or breakdown to NaN */
  VK_EBUSY = -6,        /* resource busy */
  VK_ESTATE = -7        /* call out of order (e.g. solve before bind) */
};

enum {
  VK_TH = 0, /* Taylor-Hood (P_k, P_{k-1}), continuous pressure */
  VK_SV = 1, /* Scott-Vogelius (P_k, dP_{k-1}) on the barycentric refinement of each level (Sec. 2) */
  VK_TH_QUAD = 2 /* Taylor-Hood (Q_k, Q_{k-1}) on the n x n mesh of squares (2D, 2 <= k <= 8): tensor
                    equispaced Lagrange bases, the same free-DoF numbering as VK_TH (the Q_k nodes
                    are the points of the P_k lattice), composite patches of vertices, edge
                    interiors and cell interiors (Sec. 3.1) */,
  VK_BDM = 3 /* (BDM_k, dP_{k-1}) with the symmetric interior-penalty form (Sec. 2, the H(div)-L2
                formulation; Case 3 of Sec. 3), 2D, 1 <= k <= 8, VK_F_PAPER_MMS only (its u.n and
                tangential stress vanish on the boundary), VK_PATCH_EXTENDED.  Velocity DoFs are
                moments: per interior edge e = (a, b) (a the endpoint of smaller index y (n+1) + x,
                t = (b - a)/|b - a|, n_e = (t_y, -t_x)) the k + 1 moments |e|^-1 int_e v.n_e L_j(s),
                L_j the shifted Legendre polynomials; per cell the k^2 - 1 moments |T|^-1 int_T v.q
                against the Gram-Schmidt orthonormalisation of e_0 l_a, e_1 l_a, (-xi_2, xi_1) l_a
                (l_a nodal P_{k-2}, the last for the nodes on the edge opposite the first vertex,
                xi = n (x - centroid)), spanning the first-kind Nedelec space ND_{k-1}.  Numbering:
                interior edges in ascending (index(a), index(b)) order, then cell interiors, then
                the nodal P_{k-1} pressure cell by cell (cell 2 (j n + i) is the lower triangle of
                square (i, j)).  Transfers: the natural embedding of the nested spaces (Sec. 3) */
};

enum {
  VK_F_BASELINE_MMS = 0, /* u = (sin pi x sin pi y, cos pi x cos pi y), p = 0 */
  VK_F_PAPER_MMS = 1,    /* u = (sin pi x cos pi y, -cos pi x sin pi y), p = 0 (Sec. 4) */
  VK_F_RANDOM = 2,       /* sum_{a,b} g[c][a][b] sin(a pi x) sin(b pi y)/(a^2+b^2), u = 0 on the boundary */
  VK_F_CUBE_MMS = 3      /* 3D divergence-free sin/cos field, p = 0 */
};

enum {
  VK_PATCH_COMPOSITE = 0,
  VK_PATCH_STAR = 1,
  VK_PATCH_MACRO = 2,
  VK_PATCH_EXTENDED = 3 /* VK_BDM: one patch per cell with its pressure and the free velocity on the
                           closure of the cell and of the cells sharing an edge with it (Sec. 3.1) */
};
enum { VK_STORE_FP64 = 0, VK_STORE_FP32 = 1 };
enum { VK_SMOOTH_DAMPED = 0, VK_SMOOTH_CHEBYSHEV = 1 };
enum { VK_WEIGHT_MULTIPLICITY = 0, VK_WEIGHT_NONE = 1 };

/* Problem statement (Sec. 2 weak form; Sec. 3 hierarchy; Sec. 4 mesh). */
typedef struct vk_problem {
  int dim;          /* 2 (triangles) or 3 (Kuhn tetrahedra, k = 2 only) */
  int family;       /* VK_TH, VK_SV (2D, 2 <= k <= 4, VK_PATCH_MACRO), VK_TH_QUAD (2D, 2 <= k <= 8)
                       or VK_BDM (2D, 1 <= k <= 8, VK_PATCH_EXTENDED) */
  int k;            /* velocity order, pressure order k-1; 2 <= k <= 8 in 2D (VK_BDM: from 1) */
  int n_coarse;     /* cells per direction on level 0 (>= 1) */
  int n_levels;     /* >= 2 */
  double viscosity; /* nu > 0 in a(u,v) = 2 nu int eps(u):eps(v) */
  int forcing;      /* VK_F_* */
  int n_modes;      /* VK_F_RANDOM: modes per direction M (coefficients 2*M*M) */
  const double* h_forcing_coeffs; /* VK_F_RANDOM: g[c][a][b], copied at create */
  double penalty;   /* VK_BDM: alpha of the penalty term 2 nu alpha h_e^-1 int [u]^t:[v]^t, which the
                       paper leaves open; 0 selects 2 (k + 1)^2 (2.3 to 4.6 times the smallest value
                       that keeps a_h coercive on these meshes); ignored by the other families */
} vk_problem;

/* Relaxation options (Sec. 3.1, Algorithm 1 as a damped smoother). */
typedef struct vk_patch_opts {
  int construct; /* VK_TH: VK_PATCH_COMPOSITE (vertex + edge + cell patches) or VK_PATCH_STAR;
                    VK_SV: VK_PATCH_MACRO (one patch per macro triangle: the pressure of its three
                    sub-cells and the free velocity on its closure) */
  int store;     /* VK_STORE_FP64, or VK_STORE_FP32: inverses factored in FP64, stored and applied in FP32 */
  double omega;  /* global damping of VK_SMOOTH_DAMPED (unused by VK_SMOOTH_CHEBYSHEV) */
  int smoother;  /* VK_SMOOTH_DAMPED: nu sweeps x += omega W B (b - K x) (Algorithm 1);
                    VK_SMOOTH_CHEBYSHEV: nu steps of the Chebyshev iteration preconditioned by
                    W B (Sec. 3) on the interval [lambda / 4, 1.1 lambda] of each level, lambda
                    the largest real part of the Ritz values of est_steps Arnoldi steps (two
                    classical Gram-Schmidt passes) on W B K from the start vector below,
                    computed by vk_patches_setup.  B = sum_i R_i^T K_i^{-1} R_i */
  int weighting; /* W: VK_WEIGHT_MULTIPLICITY (1 / number of patches containing the DoF) or
                    VK_WEIGHT_NONE (identity) */
  int est_steps; /* Arnoldi steps of the estimate, 1..200 (0 = 10); the workspace holds
                    max(max_restart, est_steps) + 1 basis vectors */
  uint64_t est_seed; /* start vector of level l: entry i is 2 u - 1, u = (m >> 11) 2^-53 with m
                        the SplitMix64 output function of the 64-bit counter seed
                        + l 0xD1B54A32D192ED03 + (i + 1) 0x9E3779B97F4A7C15 */
} vk_patch_opts;

typedef struct vk_level_info {
  int n;           /* cells per direction */
  int n_free;      /* free DoFs N */
  int n_velocity;  /* free velocity DoFs (the first n_velocity of the numbering) */
  int64_t nnz;     /* CSR nonzeros of K */
  int n_patches;   /* J (0 on level 0, which is solved directly) */
  int64_t sum_n;   /* sum of patch sizes */
  int64_t sum_n2;  /* sum of squared patch sizes */
  int max_n;       /* largest patch */
  int64_t p_nnz;   /* nonzeros of the prolongation from level-1 (0 on level 0) */
  int64_t inv_elems_full; /* stored elements of the patch inverses, column-major (bound for > 1 RHS) */
  int64_t inv_elems_tri;  /* stored elements in the symmetric tiled storage (bound for 1 RHS): the
                             8 x 8 tiles on and below the diagonal, zero-padded; the tiles of the
                             last block row keep only the 16-byte row chunks (2 doubles / 4 floats)
                             that hold rows below n */
  double cheb_lambda;     /* VK_SMOOTH_CHEBYSHEV: the eigenvalue estimate of W B K after
                             vk_patches_setup (0 otherwise, and on level 0) */
  int cheb_steps;         /* Arnoldi steps taken (fewer than est_steps on an exact breakdown) */
} vk_level_info;

typedef struct vk_solve_opts {
  int restart;  /* FGMRES restart length m (30) */
  int maxit;    /* total iteration cap (100) */
  double rtol;  /* stop when ||b - K x||_2 <= rtol ||b||_2 (1e-10) */
  int nu_pre;   /* pre-smoothing sweeps per level (2) */
  int nu_post;  /* post-smoothing sweeps per level (2) */
  int use_graphs; /* 1: replay each Arnoldi step (V-cycle, SpMV, CGS2) from a HIP graph
                     captured on first use; needs a non-default bound stream */
} vk_solve_opts;

typedef struct vk_solve_info {
  int iterations;        /* total FGMRES iterations */
  int converged;         /* 1 if the true relative residual is <= rtol */
  double rel_residual;   /* ||b - K x|| / ||b|| of the returned x */
  double* h_history;     /* optional, caller-owned, maxit+1 entries: residual estimates */
} vk_solve_info;

/* Thread-local message of the last failing call ("" if none). */
const char* vk_last_error(void);

typedef struct vk_hierarchy vk_hierarchy;

/* Host-side setup of every level (Sec. 3): structured meshes, Taylor-Hood
 * spaces, K = [A B^T; B 0] on the free DoFs (rediscretised per level), the
 * finest right-hand side with Dirichlet lifting, prolongations by nodal
 * interpolation (restriction = transpose) and the patch DoF lists and
 * inverse map (Sec. 3.1).  No device memory is touched.  VK_EINVAL on bad
 * sizes; *out receives a hierarchy to be freed with vk_hierarchy_destroy.
 *
 * VK_SV (the Scott-Vogelius pair named in Sec. 2, stable on barycentric
 * refinements): each level's n x n macro mesh is split at every triangle's
 * barycentre c into sub-cells (v0,v1,c), (v1,v2,c), (v2,v0,c), numbered
 * 3 m + s.  Velocity DoFs: the interior P_k nodes of the sub-cell mesh (a
 * lattice of spacing 1/(3kn)) in lexicographic order, x fastest, components
 * interleaved.  Pressure DoFs: sub-cell by sub-cell, and inside a sub-cell
 * the node V0 + (a1 (V1-V0) + a2 (V2-V0))/(k-1) in lexicographic (a1, a2)
 * order, a1 slower.  The levels are not nested: velocity is transferred by
 * nodal interpolation, pressure by the exact L^2 projection of the coarse
 * discontinuous pressure onto each fine sub-cell (the natural embedding
 * when spaces are nested). */
vk_status vk_hierarchy_create(const vk_problem* prob, const vk_patch_opts* opts, vk_hierarchy** out);

/* Frees host memory.  Device memory (the bound workspace) stays the caller's. */
vk_status vk_hierarchy_destroy(vk_hierarchy* h);

/* Bytes of device workspace needed by vk_hierarchy_bind (all levels, the
 * patch inverses in the chosen precision, the V-cycle vectors and an FGMRES
 * basis of max_restart vectors, each for up to max_rhs (1..64) right-hand
 * sides solved together). */
vk_status vk_hierarchy_workspace_bytes(const vk_hierarchy* h, int max_restart, int max_rhs, size_t* bytes);

/* Carves the caller's buffer d_workspace (>= the reported bytes, 256-byte
 * aligned) and enqueues the upload of every level on hip_stream (a
 * hipStream_t; NULL = default stream).  VK_ENOMEM if bytes is too small. */
vk_status vk_hierarchy_bind(vk_hierarchy* h, void* d_workspace, size_t bytes, int max_restart, int max_rhs,
                            void* hip_stream);

/* Matrix-full patch setup on the device: gathers every K_i = K[I_i, I_i]
 * from the CSR matrix (Sec. 3.1), inverts it by Gauss-Jordan elimination in
 * FP64 and stores the inverse (FP64 or FP32).  Patches of up to 224 DoFs are
 * eliminated with partial pivoting (largest |entry| of the column, ties to the
 * lowest row); larger ones (224 < n <= 768, vertex stars of P6..P8, Q7, Q8) by blocked
 * Gauss-Jordan without pivoting, which relies on the patch ordering (velocity
 * DoFs before pressure DoFs: the pivots run through the positive definite
 * velocity block, then the negative definite pressure Schur complement) and
 * reports a pivot of magnitude <= n eps max|K_i| as singular.  With
 * VK_SMOOTH_CHEBYSHEV it then estimates lambda on every level l >= 1 (the
 * Arnoldi vectors run on the device through the FGMRES basis, the small
 * Hessenberg eigenproblem on the host, vk_hessenberg_eigenvalues).
 * Synchronises; VK_ESINGULAR (and the level/patch in vk_last_error) on a zero
 * pivot (pivoted path) or a pivot under that floor (unpivoted path); VK_ENAN if
 * the estimate is not a positive finite number. */
vk_status vk_patches_setup(vk_hierarchy* h);

vk_status vk_level_info_get(const vk_hierarchy* h, int level, vk_level_info* info);

/* Host copies of level data, for tests.  Arrays sized from vk_level_info. */
vk_status vk_level_csr(const vk_hierarchy* h, int level, int* h_rowptr, int* h_col, double* h_val);
vk_status vk_level_prolongation(const vk_hierarchy* h, int level, int* h_rowptr, int* h_col,
                                double* h_val); /* P from level-1 to level, rows = level's DoFs */
vk_status vk_level_patches(const vk_hierarchy* h, int level, int* h_ptr, int* h_dofs);
/* K's rows of level >= 1 in union groups, the layout of the K products of more than 8
 * right-hand sides (host copies, for tests).  h_sizes[0..3] receive the group count, the row
 * count (n_free), the listed columns and the stored values.  With non-null arrays (sized from
 * those counts) also: h_gptr (groups + 1 starts into h_grow), h_grow (K's rows: runs of
 * identical column lists taken in patch order, at most 16 rows per group), h_uptr (groups + 1
 * starts into h_ucol), h_ucol (a group's ascending column union, padded to a multiple of 16 by
 * repeating its last column), h_voff (groups, start of a group's values) and h_val (per group
 * the dense G x U block in steps of 4 listed columns, [step][row][4], zeros where a row has no
 * entry and in the padding).  Builds the groups on first use.  VK_EINVAL for a bad level or a
 * null h_sizes; the arrays are all given or all null. */
vk_status vk_level_union_groups(const vk_hierarchy* h, int level, int64_t* h_sizes, int* h_gptr, int* h_grow,
                                int* h_uptr, int* h_ucol, int64_t* h_voff, double* h_val);
/* Discretisation errors of a finest-level solution h_x (host, n_free values) against the
 * manufactured solution of the problem's field (Sec. 4, stopping criteria): h_err[0] = the
 * relative H^1 error of the velocity ||u - u_h||_1 / ||u||_1 (boundary nodes take the exact
 * nodal values), h_err[1] = the L^2 error of the pressure after removing the L^2 mean of
 * p - p_h (the exact pressures are zero).  Collapsed Gauss quadrature with k + 6 points per
 * direction on every cell.  VK_EINVAL for VK_F_RANDOM (no exact solution). */
vk_status vk_solution_errors(const vk_hierarchy* h, const double* h_x, double* h_err);

/* The coarsest level's solve operator as computed at create (row-major n_free x n_free, host):
 * the leading block of the inverse of the bordered matrix [K_0 z; z^T 0], z the normalised
 * constant pressure (blocked Gauss-Jordan with partial pivoting in FP64). */
vk_status vk_coarse_inverse(const vk_hierarchy* h, double* h_out);
vk_status vk_dof_coords(const vk_hierarchy* h, int level, double* h_xyz /* N*dim */, int* h_kind /* N */);
/* Finest-level right-hand side, made consistent (constant pressure removed). */
vk_status vk_rhs(const vk_hierarchy* h, double* h_b);

/* Copies the dense matrices K_i (count patches from first, each n_i x n_i,
 * column-major, packed back to back) gathered on the device, to d_out. */
vk_status vk_patch_gather(vk_hierarchy* h, int level, int first, int count, double* d_out);
/* Copies the stored inverse of one patch (n_i x n_i column-major, as float64) to d_out. */
vk_status vk_patch_inverse(vk_hierarchy* h, int level, int patch, double* d_out);

/* d_y = K_level d_x */
vk_status vk_spmv(vk_hierarchy* h, int level, const double* d_x, double* d_y);
/* d_Y = K_level d_X for nrhs (1..max_rhs of the bind) right-hand sides, [N][nrhs] row-major, the
   product the many-right-hand-side smoother and FGMRES use: each row sums its entries in
   ascending column order (X finite), for more than 8 columns over groups of rows that share one
   column list on the FP64 matrix cores, with the same bits as at 8 columns or fewer.
   VK_EINVAL for nrhs out of range. */
vk_status vk_spmv_multi(vk_hierarchy* h, int level, const double* d_X, double* d_Y, int nrhs);
/* d_rc = P_level^T d_rf (restriction from level to level-1) */
vk_status vk_restrict(vk_hierarchy* h, int level, const double* d_rf, double* d_rc);
/* d_ef += P_level d_ec (prolongation from level-1 to level) */
vk_status vk_prolong_add(vk_hierarchy* h, int level, const double* d_ec, double* d_ef);
/* nsweeps smoothing steps on K_level x = b with the hierarchy's smoother.
 * VK_SMOOTH_DAMPED (Algorithm 1): x <- x + omega W B (b - K x).
 * VK_SMOOTH_CHEBYSHEV (Sec. 3), with theta = (a + c) / 2, delta = (c - a) / 2 for
 * the interval [a, c] = [lambda / 4, 1.1 lambda], sigma = theta / delta:
 *   rho = 1 / sigma;  d = W B (b - K x) / theta;  x += d;  then nsweeps - 1 times
 *   rho' = 1 / (2 sigma - rho);  d = rho' rho d + (2 rho' / delta) W B (b - K x);
 *   x += d;  rho = rho'
 * so the error is multiplied by T_nsweeps((theta - W B K) / delta) / T_nsweeps(sigma). */
vk_status vk_smooth(vk_hierarchy* h, int level, const double* d_b, double* d_x, int nsweeps);
/* vk_smooth for callers that cannot allocate device memory at call time (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same sweeps and kernels, bitwise the same result, with the
 * sweep's scratch (residual, patch corrections, Chebyshev direction) taken
 * from a fixed static device array of 32 MiB held by each GPU the library runs
 * on, instead of the hierarchy's workspace.  The hierarchy must be bound and
 * set up (its matrix and inverses stay in the caller's workspace).  No
 * allocation of any kind; VK_EINVAL (with the sizes in vk_last_error) if the
 * level needs more than 32 MiB: 8 N + s sum n (+ 8 N for Chebyshev) bytes, each
 * piece rounded up to 256, s = 8 (FP64) or 4 (FP32 inverses); the P4-P3 64x64
 * finest level needs 12.4 MB.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one device (two streams, two threads) race and must be
 * serialised by the caller.  Nothing in the array needs to start at zero; it
 * keeps the last call's contents.  Kernel and sweep timing are not recorded. */
vk_status vk_smooth_noalloc(vk_hierarchy* h, int level, const double* d_b, double* d_x, int nsweeps);
/* Coarsest-level solve of the bordered system [K_0 z; z^T 0][e; mu] = [r; 0]. */
vk_status vk_coarse_solve(vk_hierarchy* h, const double* d_r, double* d_e);
/* One V(nu_pre, nu_post) cycle on the finest level with zero initial guess: d_e = B d_r. */
vk_status vk_vcycle(vk_hierarchy* h, const double* d_r, double* d_e, int nu_pre, int nu_post);
/* FGMRES preconditioned by one V-cycle per iteration (Sec. 3; Sec. 4 settings).
 * d_b is made consistent in a private copy; d_x receives the solution with
 * zero-sum pressure.  Synchronous.  VK_NOT_CONVERGED if rtol was not met. */
vk_status vk_solve(vk_hierarchy* h, const double* d_b, double* d_x, const vk_solve_opts* opts,
                   vk_solve_info* info);

/* Many right-hand sides in lockstep.  Multivectors are row-major [N][nrhs]
 * (the nrhs values of one DoF are contiguous), 1 <= nrhs <= max_rhs of the
 * bind.  Each column runs the single-vector algorithm (its own Krylov basis,
 * Hessenberg matrix and stopping test); the kernels process all columns at
 * once and never mix them, so a column's result does not depend on the other
 * columns.  With FP32 inverses the patch applies are FP32 matrix-core GEMMs
 * (Delta_i = K_i^{-1} T[I_i, :]); FP64 inverses use vector FMAs and need
 * patches of at most 128 DoFs. */
vk_status vk_smooth_multi(vk_hierarchy* h, int level, const double* d_B, double* d_X, int nrhs, int nsweeps);
vk_status vk_vcycle_multi(vk_hierarchy* h, const double* d_R, double* d_E, int nrhs, int nu_pre, int nu_post);
/* info: nrhs entries (caller-owned), one per column.  VK_NOT_CONVERGED if any column missed rtol.
 * use_graphs: every Arnoldi step processes all nrhs columns (finished ones included), so its
 * kernel sequence depends on (step, nrhs, nu) only and is captured once and replayed. */
vk_status vk_solve_multi(vk_hierarchy* h, const double* d_B, double* d_X, int nrhs, const vk_solve_opts* opts,
                         vk_solve_info* info);
/* Finest-level right-hand side (consistent) of the smooth random forcing
 * sum_{a,b=1..M} g[c][a-1][b-1] sin(a pi x) sin(b pi y) / (a^2 + b^2) with zero
 * boundary velocity; coeffs: 2 * M * M values, host. */
vk_status vk_rhs_random(const vk_hierarchy* h, int n_modes, const double* h_coeffs, double* h_b);

/* Launch shapes of one level.  They change only speed, never results: the
 * CSR products and the patch apply sum in a canonical order that does not
 * depend on the lanes per row, the waves per patch, the cache policy or the
 * load depth. */
typedef struct vk_tuning {
  int k_lanes;           /* lanes per CSR row of K (4, 8, 16, 32, 64) */
  int p_lanes;           /* lanes per row of the prolongation from level-1 */
  int pt_lanes;          /* lanes per row of its transpose (restriction) */
  int apply_waves_large; /* wavefronts per patch, patches with more than 64 DoFs (1, 2, 4; also 8, 16
                            on levels with the symmetric tiled storage) */
  int apply_waves_small; /* wavefronts per patch, the others */
  int apply_nontemporal_large; /* 1: stream the large patches' inverses with non-temporal loads */
  int apply_nontemporal_small; /* same for the small patches */
  int apply_depth_large; /* symmetric tiled storage: tile steps of loads in flight per lane (2 or 4) */
  int apply_depth_small; /* same for the small patches */
  int apply_merged;      /* 1: one launch over all patches with the large patches' shape (fewer
                            launches on latency-bound coarse levels) */
} vk_tuning;

/* Autotuner (batching pattern of the path): times every candidate launch
 * shape on each level's own data (reps launches each, HIP events) and keeps
 * the fastest.  Synchronises.  Needs vk_patches_setup first. */
vk_status vk_autotune(vk_hierarchy* h, int reps);
vk_status vk_tuning_get(const vk_hierarchy* h, int level, vk_tuning* t);
/* Pins launch shapes (e.g. a cached autotuner result); VK_EINVAL on unsupported values. */
vk_status vk_tuning_set(vk_hierarchy* h, int level, const vk_tuning* t);
/* The autotuner with a tuning cache (a text file at `path`, host): if the file holds shapes for
 * every level under this hierarchy's key (device architecture and CU count, problem, patch
 * construction, storage, smoother, weights, max right-hand sides), they are set and *hit = 1;
 * otherwise vk_autotune runs and its shapes are appended to the file (created if missing),
 * *hit = 0.  Lines of other keys are kept; a later line of a key overrides an earlier one.
 * VK_EINVAL if the file cannot be written. */
vk_status vk_autotune_cached(vk_hierarchy* h, int reps, const char* path, int* hit);

/* Timing of the finest-level patch apply (single vector: the two size-class
 * dispatches; many right-hand sides: the patch GEMM), HIP events around every
 * launch while enabled: launches and total milliseconds since the last reset. */
vk_status vk_kernel_timing(vk_hierarchy* h, int enable, int reset, int64_t* launches, double* total_ms);
/* Timing of whole finest-level smoothing sweeps (the residual SpMV/SpMM, the
 * patch apply and the scatter of one sweep, HIP events around the three
 * launches; outside graph capture): the time the Vanka DoF-sweep rate is
 * measured over.  Same enable/reset/read semantics as vk_kernel_timing. */
vk_status vk_sweep_timing(vk_hierarchy* h, int enable, int reset, int64_t* sweeps, double* total_ms);

/* ---------------------------------------------------------------- serving
 * Continuous batching of Stokes solves (2D Taylor-Hood, coarsest mesh 4 x 4,
 * n = 8, 16, 32, ... and order k): one hierarchy per (n, k) is kept resident
 * in a caller-owned device pool (first-fit, admission by exact footprint,
 * least-recently-used idle hierarchies evicted when a new one does not fit);
 * each serves up to `slots` requests as columns of the many-right-hand-side
 * kernels, every column with its own FGMRES state, so requests join and
 * leave between iterations.  The viscosity of a request enters through the
 * exact identity K_nu = D_L K_1 D_R (D_L = diag(nu I, I), D_R = diag(I, I/nu)),
 * so one hierarchy serves every viscosity; FGMRES runs on K_nu itself.  A
 * request's result does not depend on the other requests in flight.  The
 * server is not thread-safe; one thread drives it with vk_server_tick. */
typedef struct vk_server vk_server;

typedef struct vk_server_opts {
  int slots;      /* concurrent requests per resident hierarchy (1..64) */
  int store;      /* VK_STORE_FP64 or VK_STORE_FP32 patch inverses */
  double omega;   /* smoother damping (0.5) */
  int nu_sweeps;  /* V(nu, nu) (2) */
  int restart;    /* FGMRES restart (30) */
  int maxit;      /* iteration cap per request (100) */
  double rtol;    /* relative residual target (1e-10) */
  int max_queue;  /* submissions beyond this many waiting requests return VK_EBUSY */
} vk_server_opts;

typedef struct vk_request {
  int n, k;          /* mesh n x n (4 * 2^m, >= 8) and velocity order k */
  double viscosity;  /* nu > 0 */
  const double* h_b; /* right-hand side on the free DoFs of (n, k), copied at submit */
} vk_request;

typedef struct vk_result {
  int state;          /* 0 queued, 1 running, 2 done */
  vk_status status;   /* when done: VK_OK, VK_NOT_CONVERGED, VK_ENOMEM (never fits the pool), ... */
  int iterations;
  double rel_residual;
  double latency_s;   /* submit -> completion, when done */
} vk_result;

typedef struct vk_server_stats {
  int64_t completed;
  int queued, running, resident_hierarchies;
  size_t pool_bytes_used;
  int64_t evictions;
  double p50_latency_s, p99_latency_s;
  double solves_per_s; /* completed / (last completion - first submission) */
} vk_server_stats;

const char* vk_server_last_error(void);
/* d_pool: caller-owned device memory (256-byte aligned) the server carves hierarchies from.
 * hip_streams: n_streams (1..64) caller-owned, non-null HIP streams (hipStream_t, e.g. torch
 * streams) on the pool's device; resident hierarchies take them in turn, so up to n_streams
 * residents overlap on the device.  The server never creates or destroys a stream; the streams
 * must outlive it.  Residents sharing a stream run one after the other; results are the same. */
vk_status vk_server_create(const vk_server_opts* opts, void* d_pool, size_t pool_bytes, void* const* hip_streams,
                           int n_streams, vk_server** out);
vk_status vk_server_destroy(vk_server* s);
/* Builds and uploads the (n, k) hierarchy now (host assembly is the slow part of admission). */
vk_status vk_server_prepare(vk_server* s, int n, int k);
vk_status vk_server_problem_size(vk_server* s, int n, int k, int* n_free);
/* Queues a request; h_x (n_free doubles, caller-owned) receives the solution
 * when it completes.  VK_EBUSY if the queue is full. */
vk_status vk_server_submit(vk_server* s, const vk_request* req, double* h_x, uint64_t* ticket);
/* Admits queued requests into free slots, advances every running request by
 * one FGMRES iteration and retires the converged ones.  *active = running + queued. */
vk_status vk_server_tick(vk_server* s, int* active);
vk_status vk_server_poll(vk_server* s, uint64_t ticket, vk_result* res);
vk_status vk_server_stats_get(vk_server* s, vk_server_stats* stats);

/* Eigenvalues of an upper Hessenberg n x n matrix (row-major h_H, host; the
 * entries below the subdiagonal are ignored), 1 <= n <= 512, by the shifted
 * QR algorithm in complex arithmetic (Givens rotations, Wilkinson shifts,
 * deflation at negligible subdiagonals).  h_re / h_im: n values each, in the
 * order of deflation (no sorting).  VK_ENAN on non-finite input or if 100 n
 * QR steps do not converge. */
vk_status vk_hessenberg_eigenvalues(int n, const double* h_H, double* h_re, double* h_im);

/* Load vector of the smooth random forcing (as VK_F_RANDOM) on the free DoFs
 * of the 2D (n, k) problem with zero boundary velocity, no hierarchy needed. */
vk_status vk_load_random(int k, int n, int n_modes, const double* h_coeffs, double* h_b);

#ifdef __cplusplus
}
#endif

#endif /* VK_H */
