// gfx950 kernels for many right-hand sides solved in lockstep.
//
// Multivectors are row-major [N][R]: the R values of one DoF are contiguous,
// so a wave reading one DoF for all right-hand sides is one coalesced access.
// No kernel mixes columns: column c of every output depends only on column c
// of the inputs, so a right-hand side gets the same bits whatever else is in
// the batch.  Reductions have a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "kernels_multi.hpp"

namespace vk {

static inline int pow2_at_least(int r) {
  int p = 1;
  while (p < r) p <<= 1;
  return p;
}

// ============================================================================
// SpMM: Y = A X (mode 0), Y = B - A X (mode 1), Y += A X (mode 2), one lane
// per right-hand side.  Rows come in runs with identical column lists (the
// two components of a velocity node; the pressure DoFs of a discontinuous
// cell; at most 8 rows): Rp lanes take one run, read each needed row of X
// once for the whole run, and sum every row of the run in ascending entry
// order.  Entries are taken 8 at a time so that 8 row loads of X are in
// flight per lane.
// ============================================================================
template <int MODE, int G>
__device__ __forceinline__ void spmm_run(int r0, int c, int R, const int* __restrict__ rowptr,
                                         const int* __restrict__ col, const double* __restrict__ val,
                                         const double* __restrict__ X, const double* __restrict__ B,
                                         double* __restrict__ Y, bool store = true) {
  const int qb = rowptr[r0], m = rowptr[r0 + 1] - qb;  // every row of the run has m entries
  // B (Y for Y += A X) of the run's rows is requested with the first row loads of X, so that the
  // run waits for memory once rather than twice
  double pre[G];
  if (MODE != 0) {
    const double* src = MODE == 1 ? B : Y;
#pragma unroll
    for (int t = 0; t < G; ++t) pre[t] = src[(int64_t)(r0 + t) * R + c];
  }
  double acc[G];
#pragma unroll
  for (int t = 0; t < G; ++t) acc[t] = 0.0;
  int q = 0;
  for (; q + 8 <= m; q += 8) {
    int cc[8];
    double xx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) cc[u] = col[qb + q + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) xx[u] = X[(int64_t)cc[u] * R + c];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      double vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) vv[u] = val[qb + t * m + q + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[t] += vv[u] * xx[u];
    }
  }
  if (q < m) {
    // the last partial batch is padded with its final entry, whose value is multiplied by zero:
    // the padded terms add zeros (X is finite), so the sums keep the ascending order
    int cc[8];
    double xx[8], msk[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      cc[u] = col[qb + min(q + u, m - 1)];
      msk[u] = q + u < m ? 1.0 : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) xx[u] = X[(int64_t)cc[u] * R + c];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      double vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) vv[u] = val[qb + t * m + min(q + u, m - 1)] * msk[u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[t] += vv[u] * xx[u];
    }
  }
  if (!store) return;
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const int64_t o = (int64_t)(r0 + t) * R + c;
    if (MODE == 0) Y[o] = acc[t];
    else if (MODE == 1) Y[o] = pre[t] - acc[t];
    else Y[o] = pre[t] + acc[t];
  }
}

// One run of G <= GMAX rows: the cases above GMAX (the longest run the matrix holds, passed by
// the host) are not compiled, so a matrix of short runs (velocity pairs, continuous pressure)
// keeps the registers of its kernel low.
template <int MODE, int GMAX>
__device__ __forceinline__ void spmm_run_any(int G, int r0, int c, int R, const int* __restrict__ rowptr,
                                             const int* __restrict__ col, const double* __restrict__ val,
                                             const double* __restrict__ X, const double* __restrict__ B,
                                             double* __restrict__ Y, bool store = true) {
  switch (G) {
    case 1: spmm_run<MODE, 1>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
    case 2: if constexpr (GMAX >= 2) spmm_run<MODE, 2>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
    case 3: if constexpr (GMAX >= 3) spmm_run<MODE, 3>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
    case 4: if constexpr (GMAX >= 4) spmm_run<MODE, 4>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
    case 5: if constexpr (GMAX >= 5) spmm_run<MODE, 5>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
    case 6: if constexpr (GMAX >= 6) spmm_run<MODE, 6>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
    case 7: if constexpr (GMAX >= 7) spmm_run<MODE, 7>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
    default: if constexpr (GMAX >= 8) spmm_run<MODE, 8>(r0, c, R, rowptr, col, val, X, B, Y, store); break;
  }
}

template <int MODE, int GMAX>
__global__ void __launch_bounds__(256) spmm_kernel(int ngroups, const int* __restrict__ grp, int R, int Rp,
                                                   const int* __restrict__ rowptr, const int* __restrict__ col,
                                                   const double* __restrict__ val, const double* __restrict__ X,
                                                   const double* __restrict__ B, double* __restrict__ Y) {
  const int gpb = 256 / Rp;
  const int g = blockIdx.x * gpb + threadIdx.x / Rp;
  const int c = threadIdx.x % Rp;
  if (g >= ngroups || c >= R) return;
  const int r0 = grp[g];
  spmm_run_any<MODE, GMAX>(grp[g + 1] - r0, r0, c, R, rowptr, col, val, X, B, Y);
}

// R > 32: one run per wave.  The run index is made wave-uniform (readfirstlane), so the row
// pointers, column indices and values, identical for all lanes, are fetched by scalar loads and
// only the accumulators and the X rows occupy vector registers.  Lanes c >= R follow the same
// control flow on a clamped column and store nothing.
template <int MODE, int GMAX>
__global__ void __launch_bounds__(256) spmm_wave_kernel(int ngroups, const int* __restrict__ grp, int R,
                                                        const int* __restrict__ rowptr,
                                                        const int* __restrict__ col, const double* __restrict__ val,
                                                        const double* __restrict__ X, const double* __restrict__ B,
                                                        double* __restrict__ Y) {
  const int g = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (g >= ngroups) return;
  const int c = threadIdx.x & 63;
  const int cl = c < R ? c : R - 1;
  const bool st = c < R;
  const int r0 = __builtin_amdgcn_readfirstlane(grp[g]);
  spmm_run_any<MODE, GMAX>(__builtin_amdgcn_readfirstlane(grp[g + 1]) - r0, r0, cl, R, rowptr, col, val, X, B, Y,
                           st);
}

// Over union groups (up to 16 rows sharing one column list, see union_groups), one group per
// wave, on the FP64 matrix cores: Y_g (G x R) = V_g (G x U) X[list, :] (U x R) in steps of 4
// listed columns, v_mfma_f64_16x16x4f64 per 16 right-hand sides (NB = ceil(R / 16) of them, so
// 1 <= R <= 64).  Lane l holds A[l % 16][l / 16] (value of row l % 16 at the step's column
// l / 16), B[l / 16][l % 16] (X at the step's column l / 16, right-hand side 16 nb + l % 16),
// and D[4 r + l / 16][l % 16] in element r; the
// instruction accumulates D = C + A B as FMAs in ascending k (measured on gfx950), so every row
// sums its entries in ascending column order as spmm_run does and the results are bitwise those
// of launch_spmm.  Each listed row of X is read once per group (one 128-byte piece per 16 lanes)
// and the values once; rows beyond G take zeros, and rows without an entry in a column multiply
// a stored zero (X finite).  Right-hand sides c >= R run on a clamped column and store nothing.
//
// The steps go through a ring of 4 stages: while step k runs, the X rows and values of step k + 3
// and this lane's column index of step k + 7 are in flight; the output rows are read at the
// start and B (Y for Y += A X) while the last four steps run.  With NT the values, B (Y) and the
// output go through the caches as streaming (non-temporal) accesses, leaving the L2 to the X rows
// that neighbouring groups share.  Every step issues the same loads
// (clamped to the last step near the end) in a fixed order, kept by scheduling barriers, so the
// in-order load counter lets step k wait for its own rows only: the index a step waits for was
// issued four steps earlier, after every X row still pending (a group's first indices all go
// out before its first rows, so the loop is entered in the same state); the zeroing of rows
// beyond G is applied at the product, not at the load, for the same reason.  Column lists are
// padded to a multiple of 16, so a round of 4 steps is never cut short.  Workgroup b runs on
// XCD b % 8 (round-robin dispatch), so the launch gives XCD x the contiguous range of `per_xcd`
// blocks starting at x per_xcd: groups come in patch order, and neighbouring groups share X rows
// in that XCD's L2.
typedef double dbl4_t __attribute__((ext_vector_type(4)));

#define VK_UNION_STEP(Q, QN)                                                                       \
  {                                                                                                \
    const int k = k0 + Q;                                                                          \
    load(k + 3, ix##QN, x##QN, a##QN);                                                             \
    ix##QN = cidx(k + 7);                                                                          \
    __builtin_amdgcn_sched_barrier(0);                                                             \
    mma(x##Q, a##Q);                                                                               \
    __builtin_amdgcn_sched_barrier(0);                                                             \
  }

template <int MODE, bool NT, int NB>
__global__ void __launch_bounds__(256, NB == 4 ? 4 : 1) spmm_union_kernel(int ngroups, int per_xcd,
                                                            const int* __restrict__ gptr,
                                                            const int* __restrict__ grow,
                                                            const int* __restrict__ uptr,
                                                            const int* __restrict__ ucol,
                                                            const int64_t* __restrict__ voff,
                                                            const double* __restrict__ gval, int R,
                                                            const double* __restrict__ X,
                                                            const double* __restrict__ B, double* __restrict__ Y) {
  const int m = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  const int g = __builtin_amdgcn_readfirstlane(m * 4 + (threadIdx.x >> 6));
  if (g >= ngroups) return;
  const int l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
  const int r0 = __builtin_amdgcn_readfirstlane(gptr[g]);
  const int G = __builtin_amdgcn_readfirstlane(gptr[g + 1]) - r0;
  const int u0 = __builtin_amdgcn_readfirstlane(uptr[g]);
  const int nsteps = (__builtin_amdgcn_readfirstlane(uptr[g + 1]) - u0) >> 2;  // a multiple of 4
  const int* uc = ucol + u0 + kq;  // this lane's column of step k: uc[4 k]
  const double* v = gval + voff[g];
  int cx[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) cx[nb] = min(nb * 16 + i, R - 1);
  const int ia = min(i, G - 1) * 4 + kq;  // this lane's value in a step's G x 4 block (clamped row)
  auto cidx = [&](int k) { return uc[4 * min(k, nsteps - 1)]; };
  auto load = [&](int k, int c, double* x, double& a) {
    const int64_t xr = (int64_t)c * R;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) x[nb] = X[xr + cx[nb]];
    const double* va = v + (int64_t)min(k, nsteps - 1) * G * 4 + ia;
    a = NT ? __builtin_nontemporal_load(va) : *va;
  };
  dbl4_t acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = dbl4_t{0.0, 0.0, 0.0, 0.0};
  const bool live = i < G;
  auto mma = [&](const double* x, double a) {
    const double az = live ? a : 0.0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(az, x[nb], acc[nb], 0, 0, 0);
  };
  double x0[NB], x1[NB], x2[NB], x3[NB], a0, a1, a2, a3;
  // every index load before the first row loads, so that on entering the loop each pending
  // index is as old (in loads issued after it) as in the loop's steady state
  const int c0 = cidx(0), c1 = cidx(1), c2 = cidx(2);
  int ix3 = cidx(3), ix0 = cidx(4), ix1 = cidx(5), ix2 = cidx(6);
  int rows[4];  // this lane's output rows 4 r + l / 16 (clamped), needed only at the end
#pragma unroll
  for (int r = 0; r < 4; ++r) rows[r] = grow[r0 + min(4 * r + kq, G - 1)];
  __builtin_amdgcn_sched_barrier(0);
  load(0, c0, x0, a0);
  load(1, c1, x1, a1);
  load(2, c2, x2, a2);
  __builtin_amdgcn_sched_barrier(0);
  for (int k0 = 0; k0 < nsteps - 4; k0 += 4) {
    VK_UNION_STEP(0, 3)
    VK_UNION_STEP(1, 0)
    VK_UNION_STEP(2, 1)
    VK_UNION_STEP(3, 2)
  }
  // the last round: its one remaining row load, then B (or Y) under the last four products
  load(nsteps - 1, ix3, x3, a3);
  double bv[4][NB];
  if (MODE != 0) {
    const double* src = MODE == 1 ? B : Y;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const double* sb = src + (int64_t)rows[r] * R + cx[nb];
        bv[r][nb] = NT ? __builtin_nontemporal_load(sb) : *sb;
      }
  }
  __builtin_amdgcn_sched_barrier(0);
  mma(x0, a0);
  mma(x1, a1);
  mma(x2, a2);
  mma(x3, a3);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (4 * r + kq >= G) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = nb * 16 + i;
      if (c >= R) continue;
      const int64_t o = (int64_t)rows[r] * R + c;
      const double y = MODE == 0 ? acc[nb][r] : MODE == 1 ? bv[r][nb] - acc[nb][r] : bv[r][nb] + acc[nb][r];
      if (NT) __builtin_nontemporal_store(y, Y + o);
      else Y[o] = y;
    }
  }
}
#undef VK_UNION_STEP

void launch_spmm_union(int mode, int ngroups, const int* gptr, const int* grow, const int* uptr, const int* ucol,
                       const int64_t* voff, const double* gval, int R, const double* X, const double* B, double* Y,
                       bool nontemporal, hipStream_t s) {
  if (ngroups <= 0) return;
  const int blocks = (ngroups + 3) / 4;
  const int per_xcd = (blocks + 7) / 8;
  const int grid = per_xcd * 8;  // block b covers range block (b % 8) per_xcd + b / 8; those past the end exit
  // NB tiles of 16 right-hand sides per wave
#define VK_UNION_LAUNCH(M, NT, NB) \
  spmm_union_kernel<M, NT, NB><<<grid, 256, 0, s>>>(ngroups, per_xcd, gptr, grow, uptr, ucol, voff, gval, R, X, B, Y)
#define VK_UNION_MODES(NT, NB)                      \
  {                                                 \
    if (mode == 0) VK_UNION_LAUNCH(0, NT, NB);      \
    else if (mode == 1) VK_UNION_LAUNCH(1, NT, NB); \
    else VK_UNION_LAUNCH(2, NT, NB);                \
  }
  if (R > 32) {
    if (nontemporal) VK_UNION_MODES(true, 4)
    else VK_UNION_MODES(false, 4)
  } else if (R > 16) {
    if (nontemporal) VK_UNION_MODES(true, 2)
    else VK_UNION_MODES(false, 2)
  } else {
    if (nontemporal) VK_UNION_MODES(true, 1)
    else VK_UNION_MODES(false, 1)
  }
#undef VK_UNION_MODES
#undef VK_UNION_LAUNCH
}

template <int GMAX>
static void spmm_dispatch(int mode, int ngroups, const int* grp, int R, const int* rp, const int* col,
                          const double* val, const double* X, const double* B, double* Y, hipStream_t s) {
  if (R > 32) {
    const int grid = (ngroups + 3) / 4;
    if (mode == 0) spmm_wave_kernel<0, GMAX><<<grid, 256, 0, s>>>(ngroups, grp, R, rp, col, val, X, B, Y);
    else if (mode == 1) spmm_wave_kernel<1, GMAX><<<grid, 256, 0, s>>>(ngroups, grp, R, rp, col, val, X, B, Y);
    else spmm_wave_kernel<2, GMAX><<<grid, 256, 0, s>>>(ngroups, grp, R, rp, col, val, X, B, Y);
    return;
  }
  const int Rp = pow2_at_least(R);
  const int gpb = 256 / Rp;
  const int grid = (ngroups + gpb - 1) / gpb;
  if (mode == 0) spmm_kernel<0, GMAX><<<grid, 256, 0, s>>>(ngroups, grp, R, Rp, rp, col, val, X, B, Y);
  else if (mode == 1) spmm_kernel<1, GMAX><<<grid, 256, 0, s>>>(ngroups, grp, R, Rp, rp, col, val, X, B, Y);
  else spmm_kernel<2, GMAX><<<grid, 256, 0, s>>>(ngroups, grp, R, Rp, rp, col, val, X, B, Y);
}

void launch_spmm(int mode, int gmax, int ngroups, const int* grp, int R, const int* rp, const int* col,
                 const double* val, const double* X, const double* B, double* Y, hipStream_t s) {
  if (ngroups <= 0) return;
  if (gmax <= 2) spmm_dispatch<2>(mode, ngroups, grp, R, rp, col, val, X, B, Y, s);
  else if (gmax <= 4) spmm_dispatch<4>(mode, ngroups, grp, R, rp, col, val, X, B, Y, s);
  else spmm_dispatch<8>(mode, ngroups, grp, R, rp, col, val, X, B, Y, s);
}

// ============================================================================
// Column-wise scatter: X[d][c] (+)= scale[d] * sum over the slots of d (ascending patch id).
// ============================================================================
template <typename TD, int MODE>
__global__ void __launch_bounds__(256) scatter_multi_kernel(int N, int R, int Rp, const int* __restrict__ dptr,
                                                            const int* __restrict__ dslot,
                                                            const TD* __restrict__ delta,
                                                            const double* __restrict__ scale, double c1, double c2,
                                                            double* __restrict__ DV, double* __restrict__ X) {
  const int rpb = 256 / Rp;
  const int d = blockIdx.x * rpb + threadIdx.x / Rp;
  const int c = threadIdx.x % Rp;
  if (d >= N || c >= R) return;
  const int q0 = dptr[d], q1 = dptr[d + 1];
  const int64_t o = (int64_t)d * R + c;
  // the epilogue's operands are requested with the first slots; 16 slot rows in flight, summed
  // in ascending slot order
  const double sc = scale[d];
  double xo, dvo;
  scatter_prev<MODE>(X, DV, o, xo, dvo);
  double s = 0.0;
  for (int q = q0; q < q1; q += 16) {
    int idx[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) idx[u] = dslot[min(q + u, q1 - 1)];
    TD v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = delta[(int64_t)idx[u] * R + c];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (q + u < q1) s += (double)v[u];
  }
  scatter_put<MODE>(sc * s, c1, c2, xo, dvo, X, DV, o);
}

// R > 32: four DoFs per wave, made wave-uniform so that the slot lists come by scalar loads; the
// first 8 slot rows of delta of all four DoFs are loaded together (32 loads in flight), further
// ones 8 at a time (a batch padded with its final slot times zero; delta is finite), each DoF
// summed in ascending slot order.
template <typename TD, int MODE>
__global__ void __launch_bounds__(256) scatter_wave_kernel(int N, int R, const int* __restrict__ dptr,
                                                           const int* __restrict__ dslot,
                                                           const TD* __restrict__ delta,
                                                           const double* __restrict__ scale, double c1, double c2,
                                                           double* __restrict__ DV, double* __restrict__ X) {
  constexpr int DPW = 4;  // DoFs per wave: the first 8 slot rows of all of them are in flight together
  const int d0 = __builtin_amdgcn_readfirstlane((blockIdx.x * 4 + (threadIdx.x >> 6)) * DPW);
  if (d0 >= N) return;
  const int c = threadIdx.x & 63;
  const int cl = c < R ? c : R - 1;
  int q0[DPW], q1[DPW];
#pragma unroll
  for (int j = 0; j < DPW; ++j) {
    const int d = min(d0 + j, N - 1);
    q0[j] = __builtin_amdgcn_readfirstlane(dptr[d]);
    q1[j] = __builtin_amdgcn_readfirstlane(dptr[d + 1]);
  }
  double v[DPW][8];
#pragma unroll
  for (int j = 0; j < DPW; ++j)
#pragma unroll
    for (int u = 0; u < 8; ++u)  // a DoF without slots (none in the patch constructions here) reads slot 0, masked
      v[j][u] = (double)delta[(int64_t)dslot[q1[j] > q0[j] ? min(q0[j] + u, q1[j] - 1) : 0] * R + cl];
  double s[DPW];
#pragma unroll
  for (int j = 0; j < DPW; ++j) {
    s[j] = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s[j] += v[j][u] * (q0[j] + u < q1[j] ? 1.0 : 0.0);
    for (int q = q0[j] + 8; q < q1[j]; q += 8) {  // DoFs in more than 8 patches
      double w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = (double)delta[(int64_t)dslot[min(q + u, q1[j] - 1)] * R + cl];
#pragma unroll
      for (int u = 0; u < 8; ++u) s[j] += w[u] * (q + u < q1[j] ? 1.0 : 0.0);
    }
  }
  if (c >= R) return;
#pragma unroll
  for (int j = 0; j < DPW; ++j)
    if (d0 + j < N) scatter_store<MODE>(scale[d0 + j] * s[j], c1, c2, X, DV, (int64_t)(d0 + j) * R + c);
}

template <typename TD, int MODE>
void scatter_multi_launch(int N, int R, const int* dptr, const int* dslot, const void* delta, const double* scale,
                          double c1, double c2, double* DV, double* X, hipStream_t s) {
  if (R > 32) {
    const int grid = (N + 15) / 16;  // 4 waves of 4 DoFs
    if (grid == 0) return;
    scatter_wave_kernel<TD, MODE><<<grid, 256, 0, s>>>(N, R, dptr, dslot, (const TD*)delta, scale, c1, c2, DV, X);
    return;
  }
  const int Rp = pow2_at_least(R);
  const int rpb = 256 / Rp;
  const int grid = (N + rpb - 1) / rpb;
  if (grid == 0) return;
  scatter_multi_kernel<TD, MODE><<<grid, 256, 0, s>>>(N, R, Rp, dptr, dslot, (const TD*)delta, scale, c1, c2, DV, X);
}

template <int MODE>
void scatter_multi_prec(bool fp32, int N, int R, const int* dptr, const int* dslot, const void* delta,
                        const double* scale, double c1, double c2, double* DV, double* X, hipStream_t s) {
  if (fp32) scatter_multi_launch<float, MODE>(N, R, dptr, dslot, delta, scale, c1, c2, DV, X, s);
  else scatter_multi_launch<double, MODE>(N, R, dptr, dslot, delta, scale, c1, c2, DV, X, s);
}

void launch_scatter_multi(bool fp32, bool set, int N, int R, const int* dptr, const int* dslot, const void* delta,
                          const double* scale, double* X, hipStream_t s) {
  launch_scatter_multi_mode(fp32, set ? kScatterSet : kScatterAdd, N, R, dptr, dslot, delta, scale, 0.0, 0.0,
                            nullptr, X, s);
}

void launch_scatter_multi_mode(bool fp32, int mode, int N, int R, const int* dptr, const int* dslot,
                               const void* delta, const double* scale, double c1, double c2, double* DV, double* X,
                               hipStream_t s) {
  switch (mode) {
    case kScatterAdd: scatter_multi_prec<kScatterAdd>(fp32, N, R, dptr, dslot, delta, scale, c1, c2, DV, X, s); break;
    case kScatterSet: scatter_multi_prec<kScatterSet>(fp32, N, R, dptr, dslot, delta, scale, c1, c2, DV, X, s); break;
    case kChebFirstSet:
      scatter_multi_prec<kChebFirstSet>(fp32, N, R, dptr, dslot, delta, scale, c1, c2, DV, X, s);
      break;
    case kChebFirstAdd:
      scatter_multi_prec<kChebFirstAdd>(fp32, N, R, dptr, dslot, delta, scale, c1, c2, DV, X, s);
      break;
    default: scatter_multi_prec<kChebNext>(fp32, N, R, dptr, dslot, delta, scale, c1, c2, DV, X, s); break;
  }
}

// ============================================================================
// Coarsest level: E = M Rv, M dense row-major N0 x N0.  One 256-thread block
// per row: wave w sums the columns j = w, w + 4, ... (8 in flight per lane,
// ascending within the wave), lane = right-hand side; the four wave partials
// are added in wave order.
// ============================================================================
__global__ void __launch_bounds__(256) dense_gemm_kernel(int N, int R, const double* __restrict__ M,
                                                         const double* __restrict__ Rv, double* __restrict__ E) {
  __shared__ double part[4][64];
  const int row = blockIdx.x, c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* m = M + (int64_t)row * N;
  const int cl = c < R ? c : R - 1;
  double acc = 0.0;
  int j = w;
  for (; j + 28 < N; j += 32) {
    double mm[8], xx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      mm[u] = m[j + 4 * u];
      xx[u] = Rv[(int64_t)(j + 4 * u) * R + cl];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += mm[u] * xx[u];
  }
  for (; j < N; j += 4) acc += m[j] * Rv[(int64_t)j * R + cl];
  part[w][c] = acc;
  __syncthreads();
  if (w == 0 && c < R) E[(int64_t)row * R + c] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
}

void launch_dense_gemm(int N, int R, const double* M, const double* Rv, double* E, hipStream_t s) {
  dense_gemm_kernel<<<N, 256, 0, s>>>(N, R, M, Rv, E);
}

// ============================================================================
// Column-wise Krylov helpers.  Reductions: each block sums a contiguous row
// chunk for every column (4 row lanes x 64 columns, fixed tree), then one
// final pass sums the block partials in block order.
// ============================================================================
constexpr int kDotGroup = 8;     // basis vectors per block of the column dot products

// Block (chunk b, group g): 4 row lanes x 64 columns; W is read once per row and multiplied with
// up to 8 basis vectors v = 8 g + t.  Each lane sums rows i0 + rl, i0 + rl + 4, ... in order; the
// four row lanes are combined in a fixed tree.
__global__ void __launch_bounds__(256) dots_partial_kernel(int n, int R, int nv, const double* __restrict__ V,
                                                           int64_t ldv, const double* __restrict__ W,
                                                           double* __restrict__ partial) {
  __shared__ double sh[kDotGroup][256];
  const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int v0 = blockIdx.y * kDotGroup;
  const int chunk = (n + kColBlocks - 1) / kColBlocks;
  const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  const int cl = c < R ? c : R - 1;
  double acc[kDotGroup];
#pragma unroll
  for (int t = 0; t < kDotGroup; ++t) acc[t] = 0.0;
  for (int i = i0 + rl; i < i1; i += 4) {
    const int64_t o = (int64_t)i * R + cl;
    const double w = W[o];
    double x[kDotGroup];
#pragma unroll
    for (int t = 0; t < kDotGroup; ++t) x[t] = V[(int64_t)min(v0 + t, nv - 1) * ldv + o];
#pragma unroll
    for (int t = 0; t < kDotGroup; ++t) acc[t] += x[t] * w;
  }
#pragma unroll
  for (int t = 0; t < kDotGroup; ++t) sh[t][threadIdx.x] = acc[t];
  __syncthreads();
  if (rl == 0 && c < R)
    for (int t = 0; t < kDotGroup && v0 + t < nv; ++t) {
      const double s = (sh[t][c] + sh[t][64 + c]) + (sh[t][128 + c] + sh[t][192 + c]);
      partial[((int64_t)(v0 + t) * kColBlocks + blockIdx.x) * 64 + c] = s;
    }
}

__global__ void __launch_bounds__(64) dots_final_kernel(int R, const double* __restrict__ partial,
                                                        double* __restrict__ out) {
  const int v = blockIdx.x, c = threadIdx.x;
  if (c >= R) return;
  double s = 0.0;
  for (int b = 0; b < kColBlocks; ++b) s += partial[((int64_t)v * kColBlocks + b) * 64 + c];
  out[(int64_t)v * R + c] = s;
}

void launch_dots_cols(int n, int R, int nv, const double* V, int64_t ldv, const double* W, double* partial,
                      double* out, hipStream_t s) {
  dots_partial_kernel<<<dim3(kColBlocks, (nv + kDotGroup - 1) / kDotGroup), 256, 0, s>>>(n, R, nv, V, ldv, W,
                                                                                         partial);
  dots_final_kernel<<<nv, 64, 0, s>>>(R, partial, out);
}

// W[i][c] += sign * sum_{v < nvc[c]} V_v[i][c] h[v][c]  (nvc == nullptr: nv for every column).  The
// basis vectors are loaded 8 at a time for every column up to nv (all finite), and terms with
// v >= nvc[c] are multiplied by zero, so the loads carry no per-lane branch.
__global__ void __launch_bounds__(256) axpy_cols_kernel(int n, int R, int Rp, int nv, const int* __restrict__ nvc,
                                                        double sign, const double* __restrict__ V, int64_t ldv,
                                                        const double* __restrict__ h, double* __restrict__ W) {
  const int rpb = 256 / Rp;
  const int i = blockIdx.x * rpb + threadIdx.x / Rp;
  const int c = threadIdx.x % Rp;
  if (i >= n || c >= R) return;
  const int m = nvc ? nvc[c] : nv;
  const int64_t o = (int64_t)i * R + c;
  double s = 0.0;
  for (int v0 = 0; v0 < nv; v0 += 8) {
    double x[8], hv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int v = min(v0 + t, nv - 1);
      x[t] = V[(int64_t)v * ldv + o];
      hv[t] = v0 + t < m ? h[(int64_t)v * R + c] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (v0 + t < nv) s += x[t] * hv[t];
  }
  W[o] += sign * s;
}

void launch_axpy_cols(int n, int R, int nv, const int* nvc, double sign, const double* V, int64_t ldv,
                      const double* h, double* W, hipStream_t s) {
  const int Rp = pow2_at_least(R);
  const int rpb = 256 / Rp;
  axpy_cols_kernel<<<(n + rpb - 1) / rpb, 256, 0, s>>>(n, R, Rp, nv, nvc, sign, V, ldv, h, W);
}

// Fused CGS2 pass: W[i][c] += sign * sum_{v < nv} V_v[i][c] h[v][c] (the arithmetic of
// axpy_cols_kernel), then the column dot products of the updated W with V_0..V_{nv-1}
// (SELF: with W itself), so one pass reads the basis once instead of twice.  Block b sums
// the rows of chunk b (the chunks of dots_partial_kernel) over 8 row lanes, lane rl taking
// rows i0 + rl, i0 + rl + 8, ... in order, and combines the lanes by the fixed tree
// ((0+1)+(2+3))+((4+5)+(6+7)); the chunk partials are summed in chunk order.  NV (8, 16 or
// 32 >= nv) sizes the register arrays.
template <bool SELF, int NV>
__global__ void __launch_bounds__(512) axpy_dots_kernel(int n, int R, int nv, const int* __restrict__ nvc,
                                                        double sign, const double* __restrict__ V, int64_t ldv,
                                                        const double* __restrict__ h, double* __restrict__ W,
                                                        double* __restrict__ partial) {
  constexpr int ND = SELF ? 1 : NV;
  __shared__ double sh[ND][512];
  const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int chunk = (n + kColBlocks - 1) / kColBlocks;
  const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  const int cl = c < R ? c : R - 1;
  const int mc = nvc ? nvc[cl] : nv;  // the column's own basis size (terms past it are multiplied by zero)
  double hv[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) hv[t] = (t < nv && t < mc) ? h[(int64_t)min(t, nv - 1) * R + cl] : 0.0;
  double acc[ND];
#pragma unroll
  for (int t = 0; t < ND; ++t) acc[t] = 0.0;
  for (int i = i0 + rl; i < i1; i += 8) {
    const int64_t o = (int64_t)i * R + cl;
    double x[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) x[t] = t < nv ? V[(int64_t)t * ldv + o] : 0.0;  // nv is uniform
    double sacc = 0.0;
#pragma unroll
    for (int t = 0; t < NV; ++t)
      if (t < nv) sacc += x[t] * hv[t];
    const double w = W[o] + sign * sacc;
    if (c < R) W[o] = w;
    if (SELF) {
      acc[0] += w * w;
    } else {
#pragma unroll
      for (int t = 0; t < ND; ++t) acc[t] += x[t] * w;
    }
  }
#pragma unroll
  for (int t = 0; t < ND; ++t) sh[t][threadIdx.x] = acc[t];
  __syncthreads();
  if (rl == 0 && c < R)
    for (int t = 0; t < ND && t < (SELF ? 1 : nv); ++t) {
      const double* q = sh[t];
      const double sv = ((q[c] + q[64 + c]) + (q[128 + c] + q[192 + c])) +
                        ((q[256 + c] + q[320 + c]) + (q[384 + c] + q[448 + c]));
      partial[((int64_t)t * kColBlocks + blockIdx.x) * 64 + c] = sv;
    }
}

template <bool SELF>
static void axpy_dots_launch(int n, int R, int nv, const int* nvc, double sign, const double* V, int64_t ldv,
                             const double* h, double* W, double* partial, hipStream_t s) {
  if (nv <= 8)
    axpy_dots_kernel<SELF, 8><<<kColBlocks, 512, 0, s>>>(n, R, nv, nvc, sign, V, ldv, h, W, partial);
  else if (nv <= 16)
    axpy_dots_kernel<SELF, 16><<<kColBlocks, 512, 0, s>>>(n, R, nv, nvc, sign, V, ldv, h, W, partial);
  else
    axpy_dots_kernel<SELF, 32><<<kColBlocks, 512, 0, s>>>(n, R, nv, nvc, sign, V, ldv, h, W, partial);
}

void launch_axpy_dots_cols(bool self, int n, int R, int nv, const int* nvc, double sign, const double* V,
                           int64_t ldv, const double* h, double* W, double* partial, double* out, hipStream_t s) {
  if (self) axpy_dots_launch<true>(n, R, nv, nvc, sign, V, ldv, h, W, partial, s);
  else axpy_dots_launch<false>(n, R, nv, nvc, sign, V, ldv, h, W, partial, s);
  dots_final_kernel<<<self ? 1 : nv, 64, 0, s>>>(R, partial, out);
}

// Y[i][c] = X[i][c] / sqrt(nn[c]) (nn[c] <= 0 gives 0: a finished or empty column)
__global__ void __launch_bounds__(256) div_sqrt_cols_kernel(int64_t total, int R, const double* X,
                                                            const double* __restrict__ nn, double* Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const double q = nn[e % R];
  Y[e] = q > 0.0 ? X[e] / sqrt(q) : 0.0;
}

void launch_div_sqrt_cols(int n, int R, const double* X, const double* nn, double* Y, hipStream_t s) {
  const int64_t total = (int64_t)n * R;
  div_sqrt_cols_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(total, R, X, nn, Y);
}

// per-column removal of the constant pressure, for columns with mask[c] != 0
__global__ void __launch_bounds__(256) project_cols_partial_kernel(int n, int p0, int R, double zv,
                                                                   const double* __restrict__ X,
                                                                   double* __restrict__ partial) {
  __shared__ double sh[256];
  const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int np = n - p0;
  const int chunk = (np + kColBlocks - 1) / kColBlocks;
  const int i0 = p0 + blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  double acc = 0.0;
  if (c < R)
    for (int i = i0 + rl; i < i1; i += 4) acc += X[(int64_t)i * R + c] * zv;
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (rl == 0) partial[(int64_t)blockIdx.x * 64 + c] = (sh[c] + sh[64 + c]) + (sh[128 + c] + sh[192 + c]);
}

__global__ void __launch_bounds__(256) project_cols_apply_kernel(int n, int p0, int R, int Rp, double zv,
                                                                 const double* __restrict__ zx,
                                                                 const int* __restrict__ mask, double* __restrict__ X) {
  const int rpb = 256 / Rp;
  const int i = p0 + blockIdx.x * rpb + threadIdx.x / Rp;
  const int c = threadIdx.x % Rp;
  if (i >= n || c >= R || !mask[c]) return;
  X[(int64_t)i * R + c] -= zx[c] * zv;
}

void launch_project_cols(int n, int p0, int R, double zv, const int* mask, double* X, double* partial,
                         hipStream_t s) {
  project_cols_partial_kernel<<<kColBlocks, 256, 0, s>>>(n, p0, R, zv, X, partial);
  dots_final_kernel<<<1, 64, 0, s>>>(R, partial, partial + kColBlocks * 64);
  const int Rp = pow2_at_least(R);
  const int rpb = 256 / Rp;
  project_cols_apply_kernel<<<(n - p0 + rpb - 1) / rpb, 256, 0, s>>>(n, p0, R, Rp, zv, partial + kColBlocks * 64,
                                                                      mask, X);
}

// ============================================================================
// Serving helpers: per-column slices of a multivector stack V[slot][N][R]
// (slot index per column), per-column diagonal scalings of the velocity
// (rows < nvel) and pressure rows, single-column copies.
// ============================================================================
// out[i][c] = V[jc[c]][i][c] * (i < nvel ? sv[c] : sp[c]); 0 where jc[c] < 0
__global__ void __launch_bounds__(256) gather_slice_kernel(int n, int R, int Rp, int nvel,
                                                           const double* __restrict__ V, int64_t slice,
                                                           const int* __restrict__ jc, const double* __restrict__ sv,
                                                           const double* __restrict__ sp, double* __restrict__ out) {
  const int rpb = 256 / Rp;
  const int i = blockIdx.x * rpb + threadIdx.x / Rp;
  const int c = threadIdx.x % Rp;
  if (i >= n || c >= R) return;
  const int j = jc[c];
  const int64_t o = (int64_t)i * R + c;
  out[o] = j >= 0 ? V[(int64_t)j * slice + o] * (i < nvel ? sv[c] : sp[c]) : 0.0;
}

void launch_gather_slice(int n, int R, int nvel, const double* V, int64_t slice, const int* jc, const double* sv,
                         const double* sp, double* out, hipStream_t s) {
  const int Rp = pow2_at_least(R);
  const int rpb = 256 / Rp;
  gather_slice_kernel<<<(n + rpb - 1) / rpb, 256, 0, s>>>(n, R, Rp, nvel, V, slice, jc, sv, sp, out);
}

// V[jc[c]][i][c] = in[i][c] * (i < nvel ? sv[c] : sp[c]) where jc[c] >= 0
__global__ void __launch_bounds__(256) scatter_slice_kernel(int n, int R, int Rp, int nvel,
                                                            const double* __restrict__ in,
                                                            const double* __restrict__ sv,
                                                            const double* __restrict__ sp, const int* __restrict__ jc,
                                                            double* __restrict__ V, int64_t slice) {
  const int rpb = 256 / Rp;
  const int i = blockIdx.x * rpb + threadIdx.x / Rp;
  const int c = threadIdx.x % Rp;
  if (i >= n || c >= R) return;
  const int j = jc[c];
  if (j < 0) return;
  const int64_t o = (int64_t)i * R + c;
  V[(int64_t)j * slice + o] = in[o] * (i < nvel ? sv[c] : sp[c]);
}

void launch_scatter_slice(int n, int R, int nvel, const double* in, const double* sv, const double* sp,
                          const int* jc, double* V, int64_t slice, hipStream_t s) {
  const int Rp = pow2_at_least(R);
  const int rpb = 256 / Rp;
  scatter_slice_kernel<<<(n + rpb - 1) / rpb, 256, 0, s>>>(n, R, Rp, nvel, in, sv, sp, jc, V, slice);
}

// r[i][c] = bb[i][c] - (i < nvel ? sv[c] : 1) t[i][c]
__global__ void __launch_bounds__(256) residual_scaled_kernel(int n, int R, int Rp, int nvel,
                                                              const double* __restrict__ bb,
                                                              const double* __restrict__ t,
                                                              const double* __restrict__ sv, double* __restrict__ r) {
  const int rpb = 256 / Rp;
  const int i = blockIdx.x * rpb + threadIdx.x / Rp;
  const int c = threadIdx.x % Rp;
  if (i >= n || c >= R) return;
  const int64_t o = (int64_t)i * R + c;
  r[o] = bb[o] - (i < nvel ? sv[c] * t[o] : t[o]);
}

void launch_residual_scaled(int n, int R, int nvel, const double* bb, const double* t, const double* sv, double* r,
                            hipStream_t s) {
  const int Rp = pow2_at_least(R);
  const int rpb = 256 / Rp;
  residual_scaled_kernel<<<(n + rpb - 1) / rpb, 256, 0, s>>>(n, R, Rp, nvel, bb, t, sv, r);
}

// column c of X[n][R] <-> contiguous x[n]
__global__ void __launch_bounds__(256) column_io_kernel(int n, int R, int c, int put, double* __restrict__ X,
                                                        double* __restrict__ x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (put) X[(int64_t)i * R + c] = x ? x[i] : 0.0;
  else x[i] = X[(int64_t)i * R + c];
}

void launch_column_put(int n, int R, int c, const double* x, double* X, hipStream_t s) {
  column_io_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, R, c, 1, X, const_cast<double*>(x));
}
void launch_column_get(int n, int R, int c, const double* X, double* x, hipStream_t s) {
  column_io_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, R, c, 0, const_cast<double*>(X), x);
}

}  // namespace vk
