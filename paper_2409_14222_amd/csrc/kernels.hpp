// Launchers of the gfx950 kernels (kernels.hip; the patch apply in patch_apply.hip).  All enqueue on `s`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vk {

// y = A x (mode 0), y = b - A x (mode 1), y += A x (mode 2); `lanes` (4..64,
// a power of two) per row.  Results do not depend on `lanes`.
void launch_csr(int mode, int nrows, int lanes, const int* rowptr, const int* col, const double* val,
                const double* x, const double* b, double* y, hipStream_t s);
int csr_default_lanes(double mean_row);

// Matrix-full patch setup: gather K_i = K[I_i, I_i] into LDS, invert it by
// Gauss-Jordan with partial pivoting (FP64), store the inverse as double or
// float: column-major (leading dimension rounded to 2 doubles / 4 floats), or
// with `tri` the symmetric tiled storage (the 8 x 8 tiles on and below the
// diagonal; the padding must have been zeroed).  `list` holds `count` patch ids
// whose size is <= nmax (32, 64, 128, 224, 512 or 768).  `singular` receives the smallest
// patch id with a zero pivot (initialise to INT_MAX).  nmax 512 and 768 (blocked, unpivoted, in
// global memory) need `slots` scratch slots of slot_elems >= n^2 doubles each.
void launch_gather_invert(int nmax, bool fp32, bool tri, int count, const int* list, const int* pptr,
                          const int* pdofs, const int* rowptr, const int* col, const double* val,
                          const int64_t* inv_off, void* inv, int* singular, double* scratch, int64_t slot_elems,
                          int slots, hipStream_t s);

// Dense K_i tiles (n_i x n_i, column-major, packed) of patches first..first+count-1.
void launch_gather_dense(int nmax, int first, int count, const int* pptr, const int* pdofs, const int* rowptr,
                         const int* col, const double* val, const int64_t* out_off, double* out, hipStream_t s);

// Copy one stored inverse (double or float, padded or tiled) to a dense n x n double array.
void launch_copy_inverse(bool fp32, bool tri, int n, const void* inv, int64_t off, double* out, hipStream_t s);

// delta_i = K_i^{-1} t[I_i] for `count` patches (n_i <= nmax) described by
// meta[0..count) ({first slot, n, inverse offset low, high}), from column-major
// or (`tri`) symmetric tiled inverses, with `waves` (1, 2 or 4) wavefronts per
// patch; `nontemporal` streams the inverses past the caches; `depth` (2 or 4)
// sets the tile steps of loads in flight of the tiled apply.  Results depend on
// none of waves, nontemporal and depth.
void launch_patch_apply(bool fp32, bool tri, int nmax, int waves, bool nontemporal, int depth, int count,
                        const int4* meta, const int* pdofs, const void* inv, const double* t, void* delta,
                        hipStream_t s);

// Epilogues of the scatter of the weighted corrections y[d] = scale[d] * sum_{slots of d} delta[slot]:
// kScatterAdd x += y; kScatterSet x = y; the Chebyshev steps keep a direction dv:
// kChebFirstSet dv = c2 y, x = dv; kChebFirstAdd dv = c2 y, x += dv; kChebNext dv = c1 dv + c2 y, x += dv.
enum ScatterMode { kScatterAdd = 0, kScatterSet = 1, kChebFirstSet = 2, kChebFirstAdd = 3, kChebNext = 4 };

// the values of x and dv that the epilogue reads (the others are left 0), so that a kernel can
// request them before its sums
template <int MODE>
__device__ __forceinline__ void scatter_prev(const double* x, const double* dv, int64_t o, double& xo, double& dvo) {
  xo = (MODE == kScatterAdd || MODE == kChebFirstAdd || MODE == kChebNext) ? x[o] : 0.0;
  dvo = MODE == kChebNext ? dv[o] : 0.0;
}

template <int MODE>
__device__ __forceinline__ void scatter_put(double y, double c1, double c2, double xo, double dvo, double* x, double* dv,
                                            int64_t o) {
  if (MODE == kScatterAdd) {
    x[o] = xo + y;
  } else if (MODE == kScatterSet) {
    x[o] = y;
  } else {
    const double d = MODE == kChebNext ? c1 * dvo + c2 * y : c2 * y;
    dv[o] = d;
    if (MODE == kChebFirstSet) x[o] = d;
    else x[o] = xo + d;
  }
}

template <int MODE>
__device__ __forceinline__ void scatter_store(double y, double c1, double c2, double* x, double* dv, int64_t o) {
  double xo, dvo;
  scatter_prev<MODE>(x, dv, o, xo, dvo);
  scatter_put<MODE>(y, c1, c2, xo, dvo, x, dv, o);
}

// x[d] += scale[d] * sum_{slots of d, ascending patch id} delta[slot]
void launch_scatter(bool fp32, int N, const int* dptr, const int* dslot, const void* delta, const double* scale,
                    double* x, hipStream_t s);

// scatter with any ScatterMode (c1, c2, dv as documented there)
void launch_scatter_mode(bool fp32, int mode, int N, const int* dptr, const int* dslot, const void* delta,
                         const double* scale, double c1, double c2, double* dv, double* x, hipStream_t s);

// v[i] = 2 u - 1, u = (splitmix64_mix(seed + level * 0xD1B54A32D192ED03 + (i + 1) * 0x9E3779B97F4A7C15) >> 11) 2^-53
void launch_splitmix_vector(int n, uint64_t seed, int level, double* v, hipStream_t s);

// x[d] = scale[d] * sum delta (first sweep from a zero iterate)
void launch_scatter_set(bool fp32, int N, const int* dptr, const int* dslot, const void* delta,
                        const double* scale, double* x, hipStream_t s);

// e = M r, M dense row-major N x N
void launch_dense_gemv(int N, const double* M, const double* r, double* e, hipStream_t s);

// Deterministic reductions.  `partial` holds at least kReduceBlocks * nv doubles.
constexpr int kReduceBlocks = 256;
// out[v] = sum_i V[v*ldv + i] * w[i], v < nv  (w may alias none of V)
void launch_multidot(int n, int nv, const double* V, int64_t ldv, const double* w, double* partial, double* out,
                     hipStream_t s);
// w[i] += sign * sum_v V[v*ldv + i] * h[v]
void launch_multiaxpy(int n, int nv, double sign, const double* V, int64_t ldv, const double* h, double* w,
                      hipStream_t s);
// w[i] += sign * sum_v V[v*ldv + i] * h[v], then out[v] = V_v . w (v < nv), or out[0] = w . w when
// self: one pass over V with the same values as launch_multiaxpy followed by launch_multidot.
// nv <= kFusedMaxNv1.
constexpr int kFusedMaxNv1 = 32;
void launch_axpy_multidot(bool self, int n, int nv, double sign, const double* V, int64_t ldv, const double* h,
                          double* w, double* partial, double* out, hipStream_t s);
// y = x / alpha
void launch_div(int n, const double* x, double alpha, double* y, hipStream_t s);
// y = y / sqrt(nn[0]), nn a device scalar (squared norm)
void launch_div_norm(int n, double* y, const double* nn, hipStream_t s);
void launch_copy(int n, const double* x, double* y, hipStream_t s);
void launch_fill(int n, double v, double* y, hipStream_t s);
// x[p] -= (sum_{q in [p0,n)} x[q] zv) zv for p in [p0, n): removal of the constant pressure
void launch_project(int n, int p0, double zv, double* x, double* partial, hipStream_t s);

}  // namespace vk
