// Launchers of the many-right-hand-side kernels (kernels_multi.hip; the patch GEMMs in patch_gemm.hip).
// Multivectors are row-major [N][R], 1 <= R <= 64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vk {

// Y = A X (mode 0), Y = B - A X (mode 1), Y += A X (mode 2); grp: the ngroups + 1 starts of the
// runs of rows with identical column lists (at most 8 rows each, from row_groups); gmax: the
// longest of those runs (1..8; the kernel is compiled for runs up to 2, 4 or 8 rows)
void launch_spmm(int mode, int gmax, int ngroups, const int* grp, int R, const int* rowptr, const int* col,
                 const double* val, const double* X, const double* B, double* Y, hipStream_t s);
// the same product for 1 <= R <= 64 over union groups (UnionGroups of vk_internal.hpp: rows grow
// of group g sharing the column list ucol[uptr[g] ..] padded to a multiple of 16, dense values at
// gval + voff[g] in steps of 4 columns), at most 16 rows per group, on the FP64 matrix cores;
// bitwise the results of launch_spmm; `nontemporal` streams the values, B and Y past the caches
// (for products larger than the last-level cache; never changes results)
void launch_spmm_union(int mode, int ngroups, const int* gptr, const int* grow, const int* uptr, const int* ucol,
                       const int64_t* voff, const double* gval, int R, const double* X, const double* B, double* Y,
                       bool nontemporal, hipStream_t s);
// Delta_i = K_i^{-1} T[I_i, :] for `count` patches (meta as for the single-vector apply);
// FP32 inverses run on the matrix cores (FP32 accumulation), FP64 inverses (n <= 128) on vector FMAs.
// nmax: the largest patch among the `count` (sizes the LDS block).
void launch_patch_gemm(bool fp32, int count, int nmax, const int4* meta, const int* pdofs, const void* inv,
                       const double* T, int R, void* delta, hipStream_t s);
void launch_scatter_multi(bool fp32, bool set, int N, int R, const int* dptr, const int* dslot, const void* delta,
                          const double* scale, double* X, hipStream_t s);
// the same with any ScatterMode of kernels.hpp (direction DV: [N][R] like X)
void launch_scatter_multi_mode(bool fp32, int mode, int N, int R, const int* dptr, const int* dslot,
                               const void* delta, const double* scale, double c1, double c2, double* DV, double* X,
                               hipStream_t s);
void launch_dense_gemm(int N, int R, const double* M, const double* Rv, double* E, hipStream_t s);
// row chunks of the column reductions (fixes their summation order)
constexpr int kColBlocks = 256;
// largest basis the fused CGS2 pass holds in registers
constexpr int kFusedMaxNv = 32;
// W += sign * sum_v V_v h[v] for v < nvc[c] (nvc == nullptr: nv), the arithmetic of launch_axpy_cols,
// then out[v][c] = <V_v, W>_c for v < nv (self: out[0][c] = <W, W>_c) over the row chunks of
// launch_dots_cols; nv <= kFusedMaxNv
void launch_axpy_dots_cols(bool self, int n, int R, int nv, const int* nvc, double sign, const double* V,
                           int64_t ldv, const double* h, double* W, double* partial, double* out, hipStream_t s);
// out[v][c] = sum_i V_v[i][c] W[i][c], v < nv; partial holds nv * kColBlocks * 64 doubles
void launch_dots_cols(int n, int R, int nv, const double* V, int64_t ldv, const double* W, double* partial,
                      double* out, hipStream_t s);
// W[i][c] += sign sum_{v < nvc[c] (or nv)} V_v[i][c] h[v][c]
void launch_axpy_cols(int n, int R, int nv, const int* nvc, double sign, const double* V, int64_t ldv,
                      const double* h, double* W, hipStream_t s);
// Y[i][c] = X[i][c] / sqrt(nn[c]), 0 where nn[c] <= 0
void launch_div_sqrt_cols(int n, int R, const double* X, const double* nn, double* Y, hipStream_t s);
// remove the constant pressure (rows p0..n) of the columns with mask[c] != 0;
// partial >= kColBlocks * 64 + 64 doubles
void launch_project_cols(int n, int p0, int R, double zv, const int* mask, double* X, double* partial,
                         hipStream_t s);

// serving: per-column slices V[jc[c]] with per-column velocity/pressure scalings
void launch_gather_slice(int n, int R, int nvel, const double* V, int64_t slice, const int* jc, const double* sv,
                         const double* sp, double* out, hipStream_t s);
void launch_scatter_slice(int n, int R, int nvel, const double* in, const double* sv, const double* sp,
                          const int* jc, double* V, int64_t slice, hipStream_t s);
// r = bb - diag(sv on velocity rows, 1 on pressure rows) t
void launch_residual_scaled(int n, int R, int nvel, const double* bb, const double* t, const double* sv, double* r,
                            hipStream_t s);
// column c of X[n][R] from x[n] (x == nullptr: zeros) / to x[n]
void launch_column_put(int n, int R, int c, const double* x, double* X, hipStream_t s);
void launch_column_get(int n, int R, int c, const double* X, double* x, hipStream_t s);

}  // namespace vk
