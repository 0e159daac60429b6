// gfx950 patch GEMMs of many right-hand sides: Delta_i = K_i^{-1} T[I_i, 0:R]
// for every patch, FP32 inverses on the matrix cores and FP64 inverses on
// vector FMAs (the dominant kernels of the many-right-hand-side smoother).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels_multi.hpp"

namespace vk {
// ============================================================================
// Patch GEMM on the matrix cores: Delta_i = K_i^{-1} T[I_i, 0:R] with FP32
// inverses, FP32 inputs and FP32 accumulation (v_mfma_f32_16x16x4_f32).  One
// workgroup per patch.  The residual block T[I_i, :] is gathered once into LDS
// as FP32 (zero-padded to 64 columns and to a multiple of 4 rows); the inverse
// streams from HBM as the A operand.  Each 16-row tile of the result is taken
// against the four 16-column tiles.
// Operand layout of the instruction (lane l): A[l % 16][l / 16],
// B[l / 16][l % 16], result rows 4 (l / 16) + i, column l % 16.
// ============================================================================
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// NW waves per patch (nmax <= 64 NW); wave w computes the 16-row tiles w,
// w + NW, ...  The residual block R_i T (FP64 rows of T, converted to FP32)
// is staged in dynamic LDS sized by the launch's largest patch, with the
// column index XOR-swizzled by bit 0 of the row so that the four k-groups of
// one MFMA read disjoint banks.  Latency hiding: the patch's DoF indices sit
// in registers (read back with readlane), each lane keeps 16 row loads in
// flight during the gather, and the A operand of a tile (16 MFMA steps = 64
// columns of K_i^{-1}) is loaded in one batch, the first one before the
// gather and each next one before the current tile's stores.
__device__ __forceinline__ int bs_index(int j, int c) { return j * 64 + (c ^ ((j & 1) << 4)); }

// FULL: all four 16-column tiles hold right-hand sides (R > 48), so the MFMA
// sequence carries no per-tile test.  KP > 0: patches of at most 64 KP DoFs on
// NW = 4 KP waves, one 16-row tile each in at most KP passes of 64 columns; the
// compiler then keeps a wave in about 52 VGPRs (KP = 1), and the workgroup's waves
// share the LDS block that a workgroup of KP waves per patch held alone, so 8 waves
// per SIMD fit instead of 3 (SV P3-dP2 macro patches of 56 DoFs, 64 right-hand
// sides: 126.5 -> 78.0 us per 8,192 patches; the same tiles in the same order, so
// the same bits).
template <int NW, bool FULL, int KP = 0>
__global__ void __launch_bounds__(64 * NW, KP > 0 ? 16 / NW : 1) patch_gemm_mfma_kernel(const int4* __restrict__ meta,
                                                                  const int* __restrict__ pdofs,
                                                                  const float* __restrict__ inv,
                                                                  const double* __restrict__ T, int R, int nmax,
                                                                  float* __restrict__ delta) {
  extern __shared__ float Bs[];  // [nk][64], swizzled
  const int4 m4 = meta[blockIdx.x];
  const int base = m4.x, n = m4.y;
  const int64_t off = (int64_t)(uint32_t)m4.z | ((int64_t)m4.w << 32);
  if (n > nmax || n <= 0 || n > (KP > 0 ? 64 * KP : 64 * NW)) return;  // the launch sizes LDS and waves for every n; never taken
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ld = (n + 3) / 4 * 4;  // FP32 inverses: leading dimension rounded to 4
  const int nk = ld;               // depth padded to the MFMA depth 4
  // uniform bases with 32-bit element offsets (the host keeps N R and sum(n) R below 2^31), so each
  // load needs one offset register
  const float* A = inv + off;
  float* D = delta + (int64_t)base * R;
  const int lr = lane & 15, lk = lane >> 4;
  const int ntiles = (n + 15) / 16;
  const int nct = FULL ? 4 : (R + 15) >> 4;  // 16-column tiles that hold right-hand sides

  // loads are unconditional at clamped (in-bounds) addresses and masked afterwards by a multiply
  // (a select lets the compiler sink each load into a branch of its own, one wait per load)
  float a[16];
  auto load_a = [&](int rt, int k0) {
    const int row = rt * 16 + lr;
    const int rowc = min(row, ld - 1);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + 4 * u + lk;
      const float x = A[(uint32_t)(min(k, n - 1) * ld + rowc)];
      a[u] = x * ((row < ld && k < n) ? 1.f : 0.f);  // finite entries: exact 0 or x
    }
  };
  int rt = wave;
  if (rt < ntiles) load_a(rt, 0);

  int pd[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) pd[q] = lane + 64 * q < n ? pdofs[base + lane + 64 * q] : 0;
  const int lc = min(lane, R - 1);
  for (int j0 = wave; j0 < nk; j0 += 8 * NW) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * NW;
      const int jj = j < n ? j : 0;
      int dof = pd[0];
#pragma unroll
      for (int t = 1; t < NW; ++t) dof = (jj >> 6) == t ? pd[t] : dof;
      dof = __builtin_amdgcn_readlane(dof, jj & 63);
      v[u] = T[(uint32_t)(dof * R + lc)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] *= (j0 + u * NW < n && lane < R) ? 1.0 : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * NW;
      if (j < nk) Bs[bs_index(j, lane)] = (float)v[u];
    }
  }
  __syncthreads();

  for (; rt < ntiles; rt += NW) {
    floatx4_t acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = (floatx4_t){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < (KP > 0 ? min(nk, 64 * KP) : nk); k0 += 64) {
      if (k0 > 0) load_a(rt, k0);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (k0 + 4 * u < nk) {
          const int k = k0 + 4 * u + lk;
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            if (!FULL && ct >= nct) break;  // column tiles past R hold zeros: skipped (wave-uniform)
            const float b = Bs[bs_index(k, ct * 16 + lr)];
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b, acc[ct], 0, 0, 0);
          }
        }
      }
    }
    if (KP == 0 && rt + NW < ntiles) load_a(rt + NW, 0);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int c = ct * 16 + lr;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rt * 16 + 4 * lk + i;
        if (r < n && c < R) D[(uint32_t)(r * R + c)] = acc[ct][i];
      }
    }
    if (KP > 0) break;  // at most NW tiles
  }
}

// FP64 inverses: vector FMAs.  The residual block T[I_i, 0:R] sits in LDS as
// [n][W] doubles, W = 16 ceil(R / 16); wave g computes the 16 columns
// 16 g .. 16 g + 15 (waves past ceil(R / 16) leave after the gather) for rows
// r, r + 64, ...  The columns of the inverse stream from HBM 16 at a time;
// every column sums in ascending j.
__global__ void __launch_bounds__(256) patch_gemm_f64_kernel(const int4* __restrict__ meta,
                                                             const int* __restrict__ pdofs,
                                                             const double* __restrict__ inv,
                                                             const double* __restrict__ T, int R,
                                                             double* __restrict__ delta) {
  extern __shared__ double Bd[];
  const int4 m4 = meta[blockIdx.x];
  const int base = m4.x, n = m4.y;
  const int64_t off = (int64_t)(uint32_t)m4.z | ((int64_t)m4.w << 32);
  if (n > 128 || n <= 0) return;  // the host limits FP64 multi-RHS patches to 128 DoFs; never taken
  const int tid = threadIdx.x;
  const int G = (R + 15) >> 4, W = 16 * G;
  for (int e = tid; e < n * W; e += 256) {
    const int j = e / W, c = e - j * W;
    Bd[e] = c < R ? T[(int64_t)pdofs[base + j] * R + c] : 0.0;
  }
  __syncthreads();
  const int g = tid >> 6, r0 = tid & 63;
  if (g >= G) return;  // wave-uniform, after the only barrier
  const int ld = (n + 1) / 2 * 2;
  const double* A = inv + off;
  for (int r = r0; r < n; r += 64) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    // whole batches of 16 columns without a test (a test per column let the compiler sink each
    // load next to its use, one load in flight), then the last partial batch with clamped loads
    // and the terms past n dropped by a select
    int j0 = 0;
    for (; j0 + 16 <= n; j0 += 16) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = A[(int64_t)(j0 + u) * ld + r];
      __builtin_amdgcn_sched_barrier(0);  // all 16 loads go out before the first product
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const double* b = Bd + (j0 + u) * W + 16 * g;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] += a[u] * b[v];
      }
    }
    if (j0 < n) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = A[(int64_t)min(j0 + u, n - 1) * ld + r];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const bool on = j0 + u < n;
        const double* b = Bd + min(j0 + u, n - 1) * W + 16 * g;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const double t = acc[v] + a[u] * b[v];
          acc[v] = on ? t : acc[v];
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c = 16 * g + v;
      if (c < R) delta[(int64_t)(base + r) * R + c] = acc[v];
    }
  }
}

template <bool FULL>
static void mfma_launch(int count, int nmax, size_t lds, const int4* meta, const int* pdofs, const float* inv,
                        const double* T, int R, float* delta, hipStream_t s) {
  if (nmax > 256)
    patch_gemm_mfma_kernel<8, FULL><<<count, 512, lds, s>>>(meta, pdofs, inv, T, R, nmax, delta);
  else if (nmax > 128)
    patch_gemm_mfma_kernel<4, FULL><<<count, 256, lds, s>>>(meta, pdofs, inv, T, R, nmax, delta);
  else if (nmax > 64)
    patch_gemm_mfma_kernel<8, FULL, 2><<<count, 512, lds, s>>>(meta, pdofs, inv, T, R, nmax, delta);
  else
    patch_gemm_mfma_kernel<4, FULL, 1><<<count, 256, lds, s>>>(meta, pdofs, inv, T, R, nmax, delta);
}

void launch_patch_gemm(bool fp32, int count, int nmax, const int4* meta, const int* pdofs, const void* inv,
                       const double* T, int R, void* delta, hipStream_t s) {
  if (count <= 0) return;
  if (fp32) {
    const int nk = (nmax + 3) / 4 * 4;
    const size_t lds = (size_t)nk * 64 * sizeof(float);
    if (R > 48) mfma_launch<true>(count, nmax, lds, meta, pdofs, (const float*)inv, T, R, (float*)delta, s);
    else mfma_launch<false>(count, nmax, lds, meta, pdofs, (const float*)inv, T, R, (float*)delta, s);
  } else {
    const size_t lds = (size_t)std::min(nmax, 128) * 16 * ((R + 15) / 16) * sizeof(double);
    patch_gemm_f64_kernel<<<count, 256, lds, s>>>(meta, pdofs, (const double*)inv, T, R, (double*)delta);
  }
}

}  // namespace vk
