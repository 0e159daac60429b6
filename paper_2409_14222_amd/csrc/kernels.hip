// gfx950 kernels of the matrix-full additive Vanka multigrid path.
//
// Wavefronts are 64 lanes.  Every reduction has a fixed order (no floating
// point atomics), so results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <climits>
#include <cstdint>

#include "kernels.hpp"

namespace vk {

// ============================================================================
// CSR products: y = A x, y = b - A x, y += A x.  A group of LANES lanes owns
// one row.  The summation order is canonical and independent of LANES: the
// row's entries are dealt to 64 virtual positions p = (q - rowstart) mod 64,
// each position accumulates its entries in ascending order (a position past the
// row's end in the last chunk adds an exact zero), and the 64
// partial sums are combined by the xor tree with offsets 32, 16, ..., 1.  A
// lane holds 64/LANES positions, performs the tree levels with offsets
// >= LANES in registers and the rest with cross-lane shuffles, so every
// launch shape returns bitwise identical results.
// ============================================================================
template <int LANES, int MODE>
__global__ void __launch_bounds__(256) csr_kernel(int nrows, const int* __restrict__ rowptr,
                                                  const int* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ x, const double* __restrict__ b,
                                                  double* __restrict__ y) {
  constexpr int V = 64 / LANES;
  const int row = (int)((blockIdx.x * 256u + threadIdx.x) / LANES);
  const int lane = threadIdx.x & (LANES - 1);
  if (row >= nrows) return;  // uniform over the LANES-group
  const int s = rowptr[row], e = rowptr[row + 1];
  double a[V];
#pragma unroll
  for (int v = 0; v < V; ++v) a[v] = 0.0;
  // loads are unconditional at clamped positions and masked by a multiply (a guarded load would
  // become a branch of its own with a wait): the V column/value pairs, then the V entries of x
  for (int base = s; base < e; base += 64) {
    int cc[V];
    double vv[V], xx[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int q = base + lane + v * LANES;
      const int qc = min(q, e - 1);
      cc[v] = col[qc];
      vv[v] = val[qc] * (q < e ? 1.0 : 0.0);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) xx[v] = x[cc[v]];
#pragma unroll
    for (int v = 0; v < V; ++v) a[v] += vv[v] * xx[v];
  }
#pragma unroll
  for (int o = 32; o >= LANES; o >>= 1) {
    const int vo = o / LANES;
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (!(v & vo)) a[v] = a[v] + a[v | vo];
  }
  double acc = a[0];
#pragma unroll
  for (int off = LANES / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LANES);
  if (lane == 0) {
    if (MODE == 0) y[row] = acc;
    else if (MODE == 1) y[row] = b[row] - acc;
    else y[row] += acc;
  }
}

template <int LANES>
static void csr_dispatch(int mode, int nrows, const int* rp, const int* c, const double* v, const double* x,
                         const double* b, double* y, hipStream_t s) {
  const int64_t threads = (int64_t)nrows * LANES;
  const int grid = (int)((threads + 255) / 256);
  if (grid == 0) return;
  if (mode == 0) csr_kernel<LANES, 0><<<grid, 256, 0, s>>>(nrows, rp, c, v, x, b, y);
  else if (mode == 1) csr_kernel<LANES, 1><<<grid, 256, 0, s>>>(nrows, rp, c, v, x, b, y);
  else csr_kernel<LANES, 2><<<grid, 256, 0, s>>>(nrows, rp, c, v, x, b, y);
}

int csr_default_lanes(double mean_row) {
  if (mean_row <= 6) return 4;
  if (mean_row <= 12) return 8;
  if (mean_row <= 28) return 16;
  if (mean_row <= 80) return 32;
  return 64;
}

void launch_csr(int mode, int nrows, int lanes, const int* rp, const int* c, const double* v, const double* x,
                const double* b, double* y, hipStream_t s) {
  switch (lanes) {
    case 4: csr_dispatch<4>(mode, nrows, rp, c, v, x, b, y, s); break;
    case 8: csr_dispatch<8>(mode, nrows, rp, c, v, x, b, y, s); break;
    case 16: csr_dispatch<16>(mode, nrows, rp, c, v, x, b, y, s); break;
    case 32: csr_dispatch<32>(mode, nrows, rp, c, v, x, b, y, s); break;
    default: csr_dispatch<64>(mode, nrows, rp, c, v, x, b, y, s); break;
  }
}

// ============================================================================
// Patch gather: K_i[l, m] = K[I_i[l], I_i[m]] into an LDS tile (column-major,
// leading dimension n).  Each wave walks whole CSR rows of the patch's DoFs;
// the column of every entry is located in the (ascending) DoF list by binary
// search, entries outside the patch are skipped.
// ============================================================================
__device__ inline void gather_tile(int n, const int* __restrict__ Ii, const int* __restrict__ rowptr,
                                   const int* __restrict__ col, const double* __restrict__ val, double* T) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
  for (int l = wave; l < n; l += nwaves) {
    const int g = Ii[l];
    const int s = rowptr[g], e = rowptr[g + 1];
    for (int q = s + lane; q < e; q += 64) {
      const int c = col[q];
      int lo = 0, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (Ii[mid] < c) lo = mid + 1;
        else hi = mid;
      }
      if (lo < n && Ii[lo] == c) T[lo * n + l] = val[q];
    }
  }
}

// ============================================================================
// Batched Gauss-Jordan inversion with partial pivoting, one 256-thread
// workgroup per patch, tile resident in LDS (NMAX = 128: 128 KiB of the
// 160 KiB LDS of a gfx950 CU).  The pivot is the largest |a| in the column
// (ties -> lowest row), found by a wave-wide xor butterfly.  Row swaps are
// undone as column swaps at the end.
// ============================================================================
// Symmetric tiled storage of a patch inverse (bound for one right-hand side):
// the 8 x 8 tiles (I, J) with I >= J, tile I (I + 1) / 2 + J, and inside a tile
// element (row k, column c) at ((k / E) * 8 + c) * E + k % E, E = 16 / sizeof
// (2 doubles or 4 floats): lane c of a tile loads its column in 16-byte
// pieces while one load instruction across 8 lanes reads 128 contiguous bytes.
// The tiles of the last block row keep only the chunks (E rows) that hold
// rows below n: nvr = ceil(rem / E) chunks, rem = n - 8 (nb - 1), 8 E nvr
// elements each.  Padding rows and columns (beyond n) of stored chunks hold zeros.
template <typename TS>
__device__ __forceinline__ int64_t tri_pos(int i, int j, int n) {
  constexpr int E = 16 / sizeof(TS);
  const int I = i >> 3, J = j >> 3, k = i & 7, c = j & 7;
  const int nb = (n + 7) >> 3, nvr = (n - 8 * (nb - 1) + E - 1) / E;
  const int64_t inner = ((k / E) * 8 + c) * E + k % E;
  if (I < nb - 1) return ((int64_t)(I * (I + 1) / 2 + J) << 6) + inner;
  if (k / E >= nvr) return -1;
  return ((int64_t)((nb - 1) * nb / 2) << 6) + (int64_t)J * 8 * E * nvr + inner;
}

template <int NMAX, typename TS>
__global__ void __launch_bounds__(256) gather_invert_kernel(const int* __restrict__ list, const int* __restrict__ pptr,
                                                            const int* __restrict__ pdofs,
                                                            const int* __restrict__ rowptr,
                                                            const int* __restrict__ col,
                                                            const double* __restrict__ val,
                                                            const int64_t* __restrict__ inv_off, TS* __restrict__ inv,
                                                            int* __restrict__ singular, bool tri) {
  __shared__ double T[NMAX * NMAX];
  __shared__ int Ii[NMAX];
  __shared__ double colk[NMAX];
  __shared__ int perm[NMAX];
  __shared__ int piv_s, sing_s;
  const int p = list[blockIdx.x];
  const int base = pptr[p];
  const int n = pptr[p + 1] - base;
  const int tid = threadIdx.x;
  const int nn = n * n;
  if (n > NMAX || n <= 0) return;  // the host sorts patches into size classes; never taken
  for (int i = tid; i < n; i += 256) Ii[i] = pdofs[base + i];
  for (int e = tid; e < nn; e += 256) T[e] = 0.0;
  if (tid == 0) sing_s = 0;
  __syncthreads();
  gather_tile(n, Ii, rowptr, col, val, T);
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  // (i, j) walk of the flattened tile e = tid + 256 t, column-major
  const int dj = 256 / n, di = 256 - dj * n;
  for (int k = 0; k < n; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bi = n;
      for (int i = k + lane; i < n; i += 64) {
        const double v = fabs(T[k * n + i]);
        if (v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        piv_s = bi;
        if (!(best > 0.0) || bi >= n) sing_s = 1;
      }
    }
    __syncthreads();
    if (sing_s) break;
    const int pr = piv_s;
    if (pr != k)
      for (int j = tid; j < n; j += 256) {
        const double a = T[j * n + k];
        T[j * n + k] = T[j * n + pr];
        T[j * n + pr] = a;
      }
    if (tid == 0) perm[k] = pr;
    __syncthreads();
    const double piv = T[k * n + k];
    for (int i = tid; i < n; i += 256) colk[i] = T[k * n + i];
    __syncthreads();
    for (int j = tid; j < n; j += 256) T[j * n + k] = (j == k ? 1.0 : T[j * n + k]) / piv;
    __syncthreads();
    int i = tid % n, j = tid / n;
    for (int e = tid; e < nn; e += 256) {
      if (i != k) {
        const double a = (j == k) ? 0.0 : T[e];
        T[e] = a - colk[i] * T[j * n + k];
      }
      i += di;
      j += dj;
      if (i >= n) { i -= n; j += 1; }
    }
    __syncthreads();
  }
  if (sing_s) {
    if (tid == 0) atomicMin(singular, p);
    return;
  }
  for (int k = n - 1; k >= 0; --k) {
    const int pr = perm[k];
    if (pr != k)
      for (int i = tid; i < n; i += 256) {
        const double a = T[k * n + i];
        T[k * n + i] = T[pr * n + i];
        T[pr * n + i] = a;
      }
    __syncthreads();
  }
  TS* out = inv + inv_off[p];
  if (tri) {
    const int m = (n + 7) & ~7;
    for (int e = tid; e < m * m; e += 256) {
      const int jj = e / m, ii = e - jj * m;
      if ((ii >> 3) >= (jj >> 3)) {
        const int64_t q = tri_pos<TS>(ii, jj, n);
        if (q >= 0) out[q] = (ii < n && jj < n) ? (TS)T[jj * n + ii] : (TS)0;
      }
    }
    return;
  }
  constexpr int RPL = 16 / sizeof(TS);
  const int ld = (n + RPL - 1) / RPL * RPL;
  for (int e = tid; e < ld * n; e += 256) {
    const int jj = e / ld, ii = e - jj * ld;
    out[e] = ii < n ? (TS)T[jj * n + ii] : (TS)0;
  }
}

// ============================================================================
// Gauss-Jordan for patches with 128 < n <= 224 (3D vertex stars reach 196):
// the FP64 tile (up to 392 KiB) does not fit in LDS, so it lives in registers.
// 1024 threads form a 32 x 32 grid; thread (ti, tj) owns the elements
// (ti + 32 x, tj + 32 y), x < 7, y < 7, of the tile padded with the identity
// to 224 x 224 (the padding never pivots and stays the identity).  Per step
// only the pivot column and the normalised pivot row pass through LDS.  The
// tile is gathered from the CSR matrix in slabs of 32 rows.
// ============================================================================
template <typename TS>
__global__ void __launch_bounds__(1024) gather_invert_big_kernel(const int* __restrict__ list,
                                                                const int* __restrict__ pptr,
                                                                const int* __restrict__ pdofs,
                                                                const int* __restrict__ rowptr,
                                                                const int* __restrict__ col,
                                                                const double* __restrict__ val,
                                                                const int64_t* __restrict__ inv_off,
                                                                TS* __restrict__ inv, int* __restrict__ singular,
                                                                bool tri) {
  constexpr int TX = 32, TY = 32, NX = 7, NY = 7, T = 224, NT = 1024;
  __shared__ double slab[TX * T];
  __shared__ int Ii[T];
  __shared__ double colk[T], prow[T], qrow[T], nrow[T];
  __shared__ int perm[T];
  __shared__ int piv_s, sing_s;
  const int tid = threadIdx.x, ti = tid & (TX - 1), tj = tid >> 5;
  const int p = list[blockIdx.x];
  const int base = pptr[p];
  const int n = pptr[p + 1] - base;
  if (n > T || n <= 0) return;  // the host sorts patches into size classes; never taken
  for (int i = tid; i < n; i += NT) Ii[i] = pdofs[base + i];
  if (tid == 0) sing_s = 0;
  double a[NX][NY];
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll 1
  for (int x = 0; x < NX; ++x) {
    __syncthreads();
    for (int e = tid; e < TX * T; e += NT) slab[e] = 0.0;
    __syncthreads();
    for (int r = wave; r < TX; r += NT / 64) {
      const int l = TX * x + r;
      if (l >= n) continue;
      const int g = Ii[l];
      for (int q = rowptr[g] + lane; q < rowptr[g + 1]; q += 64) {
        const int c = col[q];
        int lo = 0, hi = n;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (Ii[mid] < c) lo = mid + 1;
          else hi = mid;
        }
        if (lo < n && Ii[lo] == c) slab[r * T + lo] = val[q];
      }
    }
    __syncthreads();
    const int i = ti + TX * x;
#pragma unroll
    for (int xx = 0; xx < NX; ++xx)
      if (xx == x)
#pragma unroll
        for (int y = 0; y < NY; ++y) {
          const int j = tj + TY * y;
          a[xx][y] = (i < n && j < n) ? slab[ti * T + j] : (i == j ? 1.0 : 0.0);
        }
  }
  __syncthreads();

  // k = 32 kb + kr with the block index kb unrolled, so that row block and
  // column block of k (TX == TY) are compile-time register indices
  static_assert(TX == TY && NX == NY, "square thread grid");
#pragma unroll
  for (int kb = 0; kb < NX; ++kb) {
    for (int kr = 0; kr < TX; ++kr) {
      const int k = TX * kb + kr;
      if (k >= n) break;
      if (tj == kr) {  // the 32 owners of column k: one half-wave
        double best = -1.0;
        int bi = T;
#pragma unroll
        for (int x = 0; x < NX; ++x) {
          const int i = ti + TX * x;
          const double v = fabs(a[x][kb]);
          if (i >= k && i < n && v > best) { best = v; bi = i; }
        }
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 32);
          const int oi = __shfl_xor(bi, off, 32);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (ti == 0) {
          piv_s = bi;
          if (!(best > 0.0) || bi >= n) sing_s = 1;
        }
      }
      __syncthreads();
      if (sing_s) break;
      const int pr = piv_s, px = pr / TX, prr = pr % TX;
      // rows pr (the new row k) and k to LDS
      if (ti == prr) {
#pragma unroll
        for (int x = 0; x < NX; ++x)
          if (x == px)
#pragma unroll
            for (int y = 0; y < NY; ++y) prow[tj + TY * y] = a[x][y];
      }
      if (pr != k && ti == kr) {
#pragma unroll
        for (int y = 0; y < NY; ++y) qrow[tj + TY * y] = a[kb][y];
      }
      if (tid == 0) perm[k] = pr;
      __syncthreads();
      if (pr != k) {
        if (ti == kr) {
#pragma unroll
          for (int y = 0; y < NY; ++y) a[kb][y] = prow[tj + TY * y];
        }
        if (ti == prr) {
#pragma unroll
          for (int x = 0; x < NX; ++x)
            if (x == px)
#pragma unroll
              for (int y = 0; y < NY; ++y) a[x][y] = qrow[tj + TY * y];
        }
      }
      // post-swap column k and the normalised pivot row
      if (tj == kr) {
#pragma unroll
        for (int x = 0; x < NX; ++x) colk[ti + TX * x] = a[x][kb];
      }
      const double piv = prow[k];
      for (int j = tid; j < T; j += NT) nrow[j] = (j == k ? 1.0 : prow[j]) / piv;
      __syncthreads();
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        const int i = ti + TX * x;
        const double ci = colk[i];
#pragma unroll
        for (int y = 0; y < NY; ++y) {
          const int j = tj + TY * y;
          if (i == k) a[x][y] = nrow[j];
          else a[x][y] = (j == k ? 0.0 : a[x][y]) - ci * nrow[j];
        }
      }
      __syncthreads();
    }
    if (sing_s) break;
  }
  if (sing_s) {
    if (tid == 0) atomicMin(singular, p);
    return;
  }
  // undo the row interchanges as column interchanges, last first
#pragma unroll
  for (int kb = NX - 1; kb >= 0; --kb) {
    for (int kr = TX - 1; kr >= 0; --kr) {
      const int k = TX * kb + kr;
      if (k >= n) continue;
      const int pr = perm[k];
      if (pr == k) continue;  // uniform: perm is in LDS
      const int py = pr / TY, pc = pr % TY;
      if (tj == kr) {
#pragma unroll
        for (int x = 0; x < NX; ++x) colk[ti + TX * x] = a[x][kb];
      }
      if (tj == pc) {
#pragma unroll
        for (int y = 0; y < NY; ++y)
          if (y == py)
#pragma unroll
            for (int x = 0; x < NX; ++x) qrow[ti + TX * x] = a[x][y];
      }
      __syncthreads();
      if (tj == kr) {
#pragma unroll
        for (int x = 0; x < NX; ++x) a[x][kb] = qrow[ti + TX * x];
      }
      if (tj == pc) {
#pragma unroll
        for (int y = 0; y < NY; ++y)
          if (y == py)
#pragma unroll
            for (int x = 0; x < NX; ++x) a[x][y] = colk[ti + TX * x];
      }
      __syncthreads();
    }
  }
  constexpr int RPL = 16 / sizeof(TS);
  const int ld = (n + RPL - 1) / RPL * RPL;
  TS* out = inv + inv_off[p];
#pragma unroll
  for (int y = 0; y < NY; ++y) {
    const int j = tj + TY * y;
    if (j >= n) continue;
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      const int i = ti + TX * x;
      if (tri) {
        // padding of the stored tiles was zeroed before the launch
        if (i < n && (i >> 3) >= (j >> 3)) out[tri_pos<TS>(i, j, n)] = (TS)a[x][y];
      } else if (i < ld) {
        out[(int64_t)j * ld + i] = (TS)a[x][y];
      }
    }
  }
}

// ============================================================================
// Patches with 224 < n <= 768 (vertex stars of P6 .. P8, Q7 and Q8): the FP64
// matrix (up to 4.5 MiB) lives in a global scratch slot of the workgroup and is
// inverted in place by blocked Gauss-Jordan without pivoting (blocks of BS = 16
// columns up to 512 DoFs, of 8 above, where two 16 x NMAXG LDS panels would
// not fit).  The patch's DoFs are
// ascending with the velocity before the pressure, so the pivots run through
// the symmetric positive definite velocity block and then through the negative
// definite Schur complement of the pressure; a pivot of magnitude at most
// n eps max|K_i|, or a non-finite one, reports the patch as singular.  One step on the pivot block K (BS columns):
//   D = M[K,K] -> D^{-1},  M[K,j] -> D^{-1} M[K,j],  M[i,K] -> -M[i,K] D^{-1},
//   M[i,j] -> M[i,j] - M[i,K] D^{-1} M[K,j]        (i, j outside K)
// with the block row and column of the step in LDS.  Every sum runs in a fixed
// order.  A grid of `slots` workgroups walks the patch list (each its own slot).
// ============================================================================
template <typename TS, int NMAXG, int BS>
__global__ void __launch_bounds__(1024) gather_invert_global_kernel(
    const int* __restrict__ list, int count, const int* __restrict__ pptr, const int* __restrict__ pdofs,
    const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ val,
    const int64_t* __restrict__ inv_off, TS* __restrict__ inv, int* __restrict__ singular, double* __restrict__ scratch,
    int64_t slot_elems, bool tri) {
  constexpr int NT = 1024;
  __shared__ int Ii[NMAXG];
  __shared__ double Dl[BS * BS];
  __shared__ double Rl[BS * NMAXG];  // block row  [s][j]
  __shared__ double Cl[BS * NMAXG];  // block column [s][i]
  __shared__ int sing_s;
  __shared__ double wmax_s[NT / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* M = scratch + (int64_t)blockIdx.x * slot_elems;  // column-major, ld n
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int p = list[q];
    const int base = pptr[p];
    const int n = pptr[p + 1] - base;
    if (n > NMAXG || n <= 0 || (int64_t)n * n > slot_elems) continue;  // the host sizes both; never taken
    __syncthreads();  // the previous patch's readers of Ii / M are done
    for (int i = tid; i < n; i += NT) Ii[i] = pdofs[base + i];
    if (tid == 0) sing_s = 0;
    for (int64_t e = tid; e < (int64_t)n * n; e += NT) M[e] = 0.0;
    __syncthreads();
    // gather: row l of K_i from CSR row Ii[l]; columns located by binary search
    for (int l = wave; l < n; l += NT / 64) {
      const int g = Ii[l];
      for (int qq = rowptr[g] + lane; qq < rowptr[g + 1]; qq += 64) {
        const int c = col[qq];
        int lo = 0, hi = n;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (Ii[mid] < c) lo = mid + 1;
          else hi = mid;
        }
        if (lo < n && Ii[lo] == c) M[(int64_t)lo * n + l] = val[qq];
      }
    }
    __syncthreads();
    // singularity floor without pivoting: a pivot of magnitude <= n eps max|K_i| (or not finite)
    // reports the patch as singular
    double amax = 0.0;
    for (int64_t e = tid; e < (int64_t)n * n; e += NT) amax = fmax(amax, fabs(M[e]));
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
    if (lane == 0) wmax_s[wave] = amax;
    __syncthreads();
    amax = 0.0;
    for (int w = 0; w < NT / 64; ++w) amax = fmax(amax, wmax_s[w]);
    const double piv_floor = (double)n * 2.220446049250313e-16 * amax;
    for (int k0 = 0; k0 < n; k0 += BS) {
      const int kb = min(BS, n - k0);
      if (tid < BS * BS) {
        const int r = tid % BS, c = tid / BS;
        Dl[c * BS + r] = (r < kb && c < kb) ? M[(int64_t)(k0 + c) * n + k0 + r] : (r == c ? 1.0 : 0.0);
      }
      for (int e = tid; e < BS * n; e += NT) {
        const int sidx = e / n, j = e - sidx * n;
        Rl[e] = sidx < kb ? M[(int64_t)j * n + k0 + sidx] : 0.0;
        Cl[e] = sidx < kb ? M[(int64_t)(k0 + sidx) * n + j] : 0.0;
      }
      __syncthreads();
      // D -> D^{-1}: unpivoted scalar Gauss-Jordan on the BS x BS block (identity padding)
      for (int j = 0; j < kb; ++j) {
        const double piv = Dl[j * BS + j];
        double nv = 0.0;
        const int r = tid % BS, c = tid / BS;
        if (tid < BS * BS) {
          const double arc = Dl[c * BS + r], arj = Dl[j * BS + r], ajc = Dl[c * BS + j];
          if (r == j && c == j) nv = 1.0 / piv;
          else if (r == j) nv = ajc / piv;
          else if (c == j) nv = -arj / piv;
          else nv = arc - arj * (ajc / piv);
        }
        if (tid == 0 && (!(fabs(piv) > piv_floor) || !isfinite(piv))) sing_s = 1;
        __syncthreads();
        if (tid < BS * BS) Dl[c * BS + r] = nv;
        __syncthreads();
      }
      if (sing_s) break;
      // block row D^{-1} M[K, j] and block column -M[i, K] D^{-1}, written to M (old values stay in LDS)
      for (int j = tid; j < n; j += NT) {
        if (j >= k0 && j < k0 + kb) continue;
        double x[BS];
#pragma unroll
        for (int sidx = 0; sidx < BS; ++sidx) x[sidx] = Rl[sidx * n + j];
        // column j of Rl belongs to this thread alone: the new values replace the old ones held in x
#pragma unroll 1
        for (int r = 0; r < kb; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int sidx = 0; sidx < BS; ++sidx) acc += Dl[sidx * BS + r] * x[sidx];
          Rl[r * n + j] = acc;
          M[(int64_t)j * n + k0 + r] = acc;
        }
        // the block column of row i = j
#pragma unroll
        for (int sidx = 0; sidx < BS; ++sidx) x[sidx] = Cl[sidx * n + j];
#pragma unroll 1
        for (int c = 0; c < kb; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int sidx = 0; sidx < BS; ++sidx) acc += x[sidx] * Dl[c * BS + sidx];
          M[(int64_t)(k0 + c) * n + j] = -acc;
        }
      }
      if (tid < BS * BS) {
        const int r = tid % BS, c = tid / BS;
        if (r < kb && c < kb) M[(int64_t)(k0 + c) * n + k0 + r] = Dl[c * BS + r];
      }
      __syncthreads();
      // trailing update outside the block row and column: wave-strided columns, lane-strided rows
      for (int j = wave; j < n; j += NT / 64) {
        if (j >= k0 && j < k0 + kb) continue;
        double rj[BS];
#pragma unroll
        for (int sidx = 0; sidx < BS; ++sidx) rj[sidx] = Rl[sidx * n + j];
        for (int i = lane; i < n; i += 64) {
          if (i >= k0 && i < k0 + kb) continue;
          double acc = M[(int64_t)j * n + i];
#pragma unroll
          for (int sidx = 0; sidx < BS; ++sidx) acc -= Cl[sidx * n + i] * rj[sidx];
          M[(int64_t)j * n + i] = acc;
        }
      }
      __syncthreads();
    }
    if (sing_s) {
      if (tid == 0) atomicMin(singular, p);
      continue;
    }
    constexpr int RPL = 16 / sizeof(TS);
    const int ld = (n + RPL - 1) / RPL * RPL;
    TS* out = inv + inv_off[p];
    for (int j = wave; j < n; j += NT / 64)
      for (int i = lane; i < n; i += 64) {
        const double v = M[(int64_t)j * n + i];
        if (tri) {
          if ((i >> 3) >= (j >> 3)) out[tri_pos<TS>(i, j, n)] = (TS)v;
        } else {
          out[(int64_t)j * ld + i] = (TS)v;
        }
      }
  }
}

template <int NMAX>
static void gather_invert_dispatch(bool fp32, bool tri, int count, const int* list, const int* pptr,
                                   const int* pdofs, const int* rowptr, const int* col, const double* val,
                                   const int64_t* inv_off, void* inv, int* singular, hipStream_t s) {
  if (fp32)
    gather_invert_kernel<NMAX, float><<<count, 256, 0, s>>>(list, pptr, pdofs, rowptr, col, val, inv_off,
                                                            (float*)inv, singular, tri);
  else
    gather_invert_kernel<NMAX, double><<<count, 256, 0, s>>>(list, pptr, pdofs, rowptr, col, val, inv_off,
                                                             (double*)inv, singular, tri);
}

void launch_gather_invert(int nmax, bool fp32, bool tri, int count, const int* list, const int* pptr,
                          const int* pdofs, const int* rowptr, const int* col, const double* val,
                          const int64_t* inv_off, void* inv, int* singular, double* scratch, int64_t slot_elems,
                          int slots, hipStream_t s) {
  if (count <= 0) return;
  if (nmax > 224) {
    const int grid = std::min(count, slots);
    if (nmax > 512) {
      if (fp32)
        gather_invert_global_kernel<float, 768, 8><<<grid, 1024, 0, s>>>(
            list, count, pptr, pdofs, rowptr, col, val, inv_off, (float*)inv, singular, scratch, slot_elems, tri);
      else
        gather_invert_global_kernel<double, 768, 8><<<grid, 1024, 0, s>>>(
            list, count, pptr, pdofs, rowptr, col, val, inv_off, (double*)inv, singular, scratch, slot_elems, tri);
    } else if (fp32) {
      gather_invert_global_kernel<float, 512, 16><<<grid, 1024, 0, s>>>(
          list, count, pptr, pdofs, rowptr, col, val, inv_off, (float*)inv, singular, scratch, slot_elems, tri);
    } else {
      gather_invert_global_kernel<double, 512, 16><<<grid, 1024, 0, s>>>(
          list, count, pptr, pdofs, rowptr, col, val, inv_off, (double*)inv, singular, scratch, slot_elems, tri);
    }
    return;
  }
  if (nmax <= 32)
    gather_invert_dispatch<32>(fp32, tri, count, list, pptr, pdofs, rowptr, col, val, inv_off, inv, singular, s);
  else if (nmax <= 64)
    gather_invert_dispatch<64>(fp32, tri, count, list, pptr, pdofs, rowptr, col, val, inv_off, inv, singular, s);
  else if (nmax <= 128)
    gather_invert_dispatch<128>(fp32, tri, count, list, pptr, pdofs, rowptr, col, val, inv_off, inv, singular, s);
  else if (fp32)
    gather_invert_big_kernel<float><<<count, 1024, 0, s>>>(list, pptr, pdofs, rowptr, col, val, inv_off, (float*)inv,
                                                          singular, tri);
  else
    gather_invert_big_kernel<double><<<count, 1024, 0, s>>>(list, pptr, pdofs, rowptr, col, val, inv_off,
                                                           (double*)inv, singular, tri);
}

template <int NMAX>
__global__ void __launch_bounds__(256) gather_dense_kernel(int first, const int* __restrict__ pptr,
                                                           const int* __restrict__ pdofs,
                                                           const int* __restrict__ rowptr,
                                                           const int* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const int64_t* __restrict__ out_off,
                                                           double* __restrict__ out) {
  __shared__ double T[NMAX * NMAX];
  __shared__ int Ii[NMAX];
  const int p = first + blockIdx.x;
  const int base = pptr[p], n = pptr[p + 1] - base;
  if (n > NMAX) return;  // the host picks NMAX >= every size in the range; never taken
  for (int i = threadIdx.x; i < n; i += 256) Ii[i] = pdofs[base + i];
  for (int e = threadIdx.x; e < n * n; e += 256) T[e] = 0.0;
  __syncthreads();
  gather_tile(n, Ii, rowptr, col, val, T);
  __syncthreads();
  double* o = out + out_off[blockIdx.x];
  for (int e = threadIdx.x; e < n * n; e += 256) o[e] = T[e];
}

// Big patches: the dense tile is zeroed and filled directly in the output.
__global__ void __launch_bounds__(256) gather_dense_global_kernel(int first, const int* __restrict__ pptr,
                                                                  const int* __restrict__ pdofs,
                                                                  const int* __restrict__ rowptr,
                                                                  const int* __restrict__ col,
                                                                  const double* __restrict__ val,
                                                                  const int64_t* __restrict__ out_off,
                                                                  double* __restrict__ out) {
  const int p = first + blockIdx.x;
  const int base = pptr[p], n = pptr[p + 1] - base;
  const int* Ii = pdofs + base;
  double* o = out + out_off[blockIdx.x];
  for (int e = threadIdx.x; e < n * n; e += 256) o[e] = 0.0;
  __syncthreads();
  gather_tile(n, Ii, rowptr, col, val, o);
}

void launch_gather_dense(int nmax, int first, int count, const int* pptr, const int* pdofs, const int* rowptr,
                         const int* col, const double* val, const int64_t* out_off, double* out, hipStream_t s) {
  if (count <= 0) return;
  if (nmax > 128) {
    gather_dense_global_kernel<<<count, 256, 0, s>>>(first, pptr, pdofs, rowptr, col, val, out_off, out);
    return;
  }
  if (nmax <= 32) gather_dense_kernel<32><<<count, 256, 0, s>>>(first, pptr, pdofs, rowptr, col, val, out_off, out);
  else if (nmax <= 64) gather_dense_kernel<64><<<count, 256, 0, s>>>(first, pptr, pdofs, rowptr, col, val, out_off, out);
  else gather_dense_kernel<128><<<count, 256, 0, s>>>(first, pptr, pdofs, rowptr, col, val, out_off, out);
}

template <typename TS>
__global__ void copy_inverse_kernel(int n, const TS* __restrict__ inv, int64_t off, double* __restrict__ out,
                                    bool tri) {
  constexpr int RPL = 16 / sizeof(TS);
  const int ld = (n + RPL - 1) / RPL * RPL;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n * n; e += gridDim.x * 256) {
    const int j = e / n, i = e - j * n;
    if (tri) out[e] = (double)inv[off + ((i >> 3) >= (j >> 3) ? tri_pos<TS>(i, j, n) : tri_pos<TS>(j, i, n))];
    else out[e] = (double)inv[off + (int64_t)j * ld + i];
  }
}

void launch_copy_inverse(bool fp32, bool tri, int n, const void* inv, int64_t off, double* out, hipStream_t s) {
  const int grid = (n * n + 255) / 256;
  if (fp32) copy_inverse_kernel<float><<<grid, 256, 0, s>>>(n, (const float*)inv, off, out, tri);
  else copy_inverse_kernel<double><<<grid, 256, 0, s>>>(n, (const double*)inv, off, out, tri);
}

// ============================================================================
// Deterministic segmented scatter-add of the weighted corrections:
// x[d] (+)= scale[d] * sum over the slots of d (ascending patch id).  The
// slot indices of a chunk of 8 are loaded first and the corrections after,
// so the dependent loads overlap; the sum stays in ascending slot order.
// ============================================================================
template <typename TD, int MODE>
__global__ void __launch_bounds__(256) scatter_kernel(int N, const int* __restrict__ dptr,
                                                      const int* __restrict__ dslot, const TD* __restrict__ delta,
                                                      const double* __restrict__ scale, double c1, double c2,
                                                      double* __restrict__ dv, double* __restrict__ x) {
  const int d = blockIdx.x * 256 + threadIdx.x;
  if (d >= N) return;
  const int q0 = dptr[d], q1 = dptr[d + 1];
  // the epilogue's operands are requested with the first slots
  const double sc = scale[d];
  double xo, dvo;
  scatter_prev<MODE>(x, dv, d, xo, dvo);
  double s = 0.0;
  for (int q = q0; q < q1; q += 16) {
    int idx[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) idx[u] = q + u < q1 ? dslot[q + u] : -1;
    TD v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = idx[u] >= 0 ? delta[idx[u]] : (TD)0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (q + u < q1) s += (double)v[u];
  }
  scatter_put<MODE>(sc * s, c1, c2, xo, dvo, x, dv, d);
}

template <int MODE>
void scatter_launch(bool fp32, int N, const int* dptr, const int* dslot, const void* delta, const double* scale,
                    double c1, double c2, double* dv, double* x, hipStream_t s) {
  const int grid = (N + 255) / 256;
  if (grid == 0) return;
  if (fp32)
    scatter_kernel<float, MODE><<<grid, 256, 0, s>>>(N, dptr, dslot, (const float*)delta, scale, c1, c2, dv, x);
  else
    scatter_kernel<double, MODE><<<grid, 256, 0, s>>>(N, dptr, dslot, (const double*)delta, scale, c1, c2, dv, x);
}

void launch_scatter(bool fp32, int N, const int* dptr, const int* dslot, const void* delta, const double* scale,
                    double* x, hipStream_t s) {
  scatter_launch<kScatterAdd>(fp32, N, dptr, dslot, delta, scale, 0.0, 0.0, nullptr, x, s);
}

void launch_scatter_set(bool fp32, int N, const int* dptr, const int* dslot, const void* delta,
                        const double* scale, double* x, hipStream_t s) {
  scatter_launch<kScatterSet>(fp32, N, dptr, dslot, delta, scale, 0.0, 0.0, nullptr, x, s);
}

void launch_scatter_mode(bool fp32, int mode, int N, const int* dptr, const int* dslot, const void* delta,
                         const double* scale, double c1, double c2, double* dv, double* x, hipStream_t s) {
  switch (mode) {
    case kScatterAdd: scatter_launch<kScatterAdd>(fp32, N, dptr, dslot, delta, scale, c1, c2, dv, x, s); break;
    case kScatterSet: scatter_launch<kScatterSet>(fp32, N, dptr, dslot, delta, scale, c1, c2, dv, x, s); break;
    case kChebFirstSet: scatter_launch<kChebFirstSet>(fp32, N, dptr, dslot, delta, scale, c1, c2, dv, x, s); break;
    case kChebFirstAdd: scatter_launch<kChebFirstAdd>(fp32, N, dptr, dslot, delta, scale, c1, c2, dv, x, s); break;
    default: scatter_launch<kChebNext>(fp32, N, dptr, dslot, delta, scale, c1, c2, dv, x, s); break;
  }
}

// ============================================================================
// Counter-based start vector of the eigenvalue estimate: SplitMix64's output
// function of seed + level * 0xD1B54A32D192ED03 + (i + 1) * 0x9E3779B97F4A7C15
// (64-bit wrap-around), top 53 bits as a uniform u in [0, 1), entry 2 u - 1
// (exact in FP64).
// ============================================================================
__global__ void __launch_bounds__(256) splitmix_vector_kernel(int n, uint64_t base, double* __restrict__ v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint64_t z = base + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * 0x1.0p-53;
  v[i] = 2.0 * u - 1.0;
}

void launch_splitmix_vector(int n, uint64_t seed, int level, double* v, hipStream_t s) {
  const int grid = (n + 255) / 256;
  if (grid == 0) return;
  const uint64_t base = seed + (uint64_t)level * 0xD1B54A32D192ED03ull;
  splitmix_vector_kernel<<<grid, 256, 0, s>>>(n, base, v);
}

// ============================================================================
// Coarsest level: e = M r with the pre-inverted bordered system; one wave per row.
// ============================================================================
__global__ void __launch_bounds__(256) dense_gemv_kernel(int N, const double* __restrict__ M,
                                                         const double* __restrict__ r, double* __restrict__ e) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  const double* m = M + (int64_t)row * N;
  double acc = 0.0;
  for (int j = lane; j < N; j += 64) acc += m[j] * r[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) e[row] = acc;
}

void launch_dense_gemv(int N, const double* M, const double* r, double* e, hipStream_t s) {
  dense_gemv_kernel<<<(N + 3) / 4, 256, 0, s>>>(N, M, r, e);
}

// ============================================================================
// Krylov helpers with fixed-order two-stage reductions.
// ============================================================================
__device__ inline double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256) multidot_partial_kernel(int n, const double* __restrict__ V, int64_t ldv,
                                                               const double* __restrict__ w,
                                                               double* __restrict__ partial) {
  __shared__ double sh[256];
  const int v = blockIdx.y;
  const double* x = V + (int64_t)v * ldv;
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kReduceBlocks * 256) acc += x[i] * w[i];
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) partial[v * kReduceBlocks + blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) reduce_final_kernel(const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double sh[256];
  const double s = block_sum256(partial[blockIdx.x * kReduceBlocks + threadIdx.x], sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

void launch_multidot(int n, int nv, const double* V, int64_t ldv, const double* w, double* partial, double* out,
                     hipStream_t s) {
  static_assert(kReduceBlocks == 256, "final stage sums one partial per thread");
  multidot_partial_kernel<<<dim3(kReduceBlocks, nv), 256, 0, s>>>(n, V, ldv, w, partial);
  reduce_final_kernel<<<nv, 256, 0, s>>>(partial, out);
}

__global__ void __launch_bounds__(256) multiaxpy_kernel(int n, int nv, double sign, const double* __restrict__ V,
                                                        int64_t ldv, const double* __restrict__ h,
                                                        double* __restrict__ w) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < nv; ++v) s += V[(int64_t)v * ldv + i] * h[v];
  w[i] += sign * s;
}

void launch_multiaxpy(int n, int nv, double sign, const double* V, int64_t ldv, const double* h, double* w,
                      hipStream_t s) {
  multiaxpy_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, nv, sign, V, ldv, h, w);
}

// w[i] += sign * sum_v V[v*ldv + i] * h[v] (the terms in v order, as multiaxpy_kernel), then the
// block partials of the dots V_v . w (or of w . w for SELF) with the updated w, in the row order and
// tree of multidot_partial_kernel: the fused pass gives bitwise the values of the two separate ones
// and reads V once.  NV (8, 16 or 32 >= nv) sizes the register arrays.
template <bool SELF, int NV>
__global__ void __launch_bounds__(256) axpy_multidot_kernel(int n, int nv, double sign, const double* __restrict__ V,
                                                            int64_t ldv, const double* __restrict__ h,
                                                            double* __restrict__ w, double* __restrict__ partial) {
  constexpr int ND = SELF ? 1 : NV;
  __shared__ double sh[256];
  double hv[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) hv[t] = t < nv ? h[t] : 0.0;
  double acc[ND];
#pragma unroll
  for (int t = 0; t < ND; ++t) acc[t] = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kReduceBlocks * 256) {
    double x[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) x[t] = t < nv ? V[(int64_t)t * ldv + i] : 0.0;
    double sacc = 0.0;
#pragma unroll
    for (int t = 0; t < NV; ++t)
      if (t < nv) sacc += x[t] * hv[t];
    const double wi = w[i] + sign * sacc;
    w[i] = wi;
    if (SELF) {
      acc[0] += wi * wi;
    } else {
#pragma unroll
      for (int t = 0; t < ND; ++t) acc[t] += x[t] * wi;
    }
  }
  const int nd = SELF ? 1 : nv;
#pragma unroll
  for (int t = 0; t < ND; ++t) {
    if (t >= nd) break;  // uniform across the block
    const double r = block_sum256(acc[t], sh);
    if (threadIdx.x == 0) partial[t * kReduceBlocks + blockIdx.x] = r;
  }
}

template <bool SELF>
static void axpy_multidot_launch(int n, int nv, double sign, const double* V, int64_t ldv, const double* h,
                                 double* w, double* partial, hipStream_t s) {
  if (nv <= 8)
    axpy_multidot_kernel<SELF, 8><<<kReduceBlocks, 256, 0, s>>>(n, nv, sign, V, ldv, h, w, partial);
  else if (nv <= 16)
    axpy_multidot_kernel<SELF, 16><<<kReduceBlocks, 256, 0, s>>>(n, nv, sign, V, ldv, h, w, partial);
  else
    axpy_multidot_kernel<SELF, 32><<<kReduceBlocks, 256, 0, s>>>(n, nv, sign, V, ldv, h, w, partial);
}

void launch_axpy_multidot(bool self, int n, int nv, double sign, const double* V, int64_t ldv, const double* h,
                          double* w, double* partial, double* out, hipStream_t s) {
  if (self) axpy_multidot_launch<true>(n, nv, sign, V, ldv, h, w, partial, s);
  else axpy_multidot_launch<false>(n, nv, sign, V, ldv, h, w, partial, s);
  reduce_final_kernel<<<self ? 1 : nv, 256, 0, s>>>(partial, out);
}

__global__ void __launch_bounds__(256) div_kernel(int n, const double* x, double a, double* y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = x[i] / a;
}
__global__ void __launch_bounds__(256) copy_kernel(int n, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = x[i];
}
__global__ void __launch_bounds__(256) fill_kernel(int n, double v, double* __restrict__ y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = v;
}

__global__ void __launch_bounds__(256) div_norm_kernel(int n, double* y, const double* __restrict__ nn) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = y[i] / sqrt(nn[0]);
}

void launch_div_norm(int n, double* y, const double* nn, hipStream_t s) {
  div_norm_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, y, nn);
}

void launch_div(int n, const double* x, double alpha, double* y, hipStream_t s) {
  div_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, x, alpha, y);
}
void launch_copy(int n, const double* x, double* y, hipStream_t s) {
  copy_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, x, y);
}
void launch_fill(int n, double v, double* y, hipStream_t s) {
  fill_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, v, y);
}

__global__ void __launch_bounds__(256) project_partial_kernel(int n, int p0, double zv, const double* __restrict__ x,
                                                              double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = p0 + blockIdx.x * 256 + threadIdx.x; i < n; i += kReduceBlocks * 256) acc += x[i] * zv;
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) project_apply_kernel(int n, int p0, double zv, const double* __restrict__ zx,
                                                            double* __restrict__ x) {
  const int i = p0 + blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] -= zx[0] * zv;
}

void launch_project(int n, int p0, double zv, double* x, double* partial, hipStream_t s) {
  project_partial_kernel<<<kReduceBlocks, 256, 0, s>>>(n, p0, zv, x, partial);
  reduce_final_kernel<<<1, 256, 0, s>>>(partial, partial + kReduceBlocks);
  project_apply_kernel<<<(n - p0 + 255) / 256, 256, 0, s>>>(n, p0, zv, partial + kReduceBlocks, x);
}

}  // namespace vk
