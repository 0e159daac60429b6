// gfx950 additive patch apply of one right-hand side: delta_i = K_i^{-1} t[I_i]
// for every patch (the dominant kernel of the smoother), from the column-major
// or the symmetric tiled inverse storage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"

namespace vk {
// ============================================================================
// Additive patch apply: delta_i = K_i^{-1} t[I_i].  One workgroup of W waves
// per patch.  The gathered residual sits in LDS; the inverse (column-major,
// ld rounded to RPL rows) streams from HBM in 16-byte non-temporal loads.
//
// Lane layout: R = ld / RPL lanes cover the rows (RPL rows each), C column
// slots (a power of two <= 8) cover the columns.  The summation order of
// every output row is canonical: column j belongs to group j mod 8, each
// group sums its columns in ascending order, and the 8 group sums are
// combined by the xor tree with offsets 4, 2, 1.  A slot c owns groups
// c, c + C, ... and performs the tree levels with offsets >= C in
// registers; the remaining levels run over LDS.  Results are therefore
// bitwise independent of W (the autotuned launch shape).
// ============================================================================
typedef double dbl2_t __attribute__((ext_vector_type(2)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
template <typename T> struct vec16;
template <> struct vec16<double> { using type = dbl2_t; };
template <> struct vec16<float> { using type = flt4_t; };

template <typename TS, bool NT>
__device__ inline typename vec16<TS>::type load16(const TS* p) {
  using V = typename vec16<TS>::type;
  if (NT) return __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return *reinterpret_cast<const V*>(p);
}

// One row pass of the apply with C column slots (compile-time, so every
// accumulator index is static).  Slot c owns the columns c, c + C, ... whose
// canonical groups are c, c + C, ... (ng = 8 / C of them).
template <typename TS, int NTH, bool NT, int C>
__device__ inline void apply_pass(const TS* __restrict__ A, int n, int ld, int r0, int rows, bool gather,
                                  const int* __restrict__ dofs, const double* __restrict__ t, TS* xs, TS* red,
                                  TS* __restrict__ dout) {  // dout: the patch's first slot
  constexpr int RPL = 16 / sizeof(TS);
  constexpr int U = 16;       // column loads in flight per lane
  constexpr int ng = 8 / C;   // canonical groups per slot
  using V = typename vec16<TS>::type;
  const int tid = threadIdx.x;
  const int R = rows / RPL;
  const int r = tid % R, c = tid / R;
  const bool active = c < C;
  const int mcount = active ? (n - c + C - 1) / C : 0;
  const TS* Ap = A + r0 + r * RPL + (int64_t)c * ld;
  const int64_t cstride = (int64_t)C * ld;
  V a[U];
  // the first batch of column loads goes out before the residual gather completes
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (u < mcount) a[u] = load16<TS, NT>(Ap + u * cstride);
  if (gather) {
    for (int j = tid; j < n; j += NTH) xs[j] = (TS)t[dofs[j]];
    __syncthreads();
  }
  TS acc[ng][RPL];
#pragma unroll
  for (int g = 0; g < ng; ++g)
#pragma unroll
    for (int q = 0; q < RPL; ++q) acc[g][q] = (TS)0;
  for (int m = 0; m < mcount; m += U) {
    if (m > 0) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (m + u < mcount) a[u] = load16<TS, NT>(Ap + (int64_t)(m + u) * cstride);
    }
    // column c + C (m + u) is in local group (m + u) mod ng = u mod ng (U is a multiple of 8)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (m + u < mcount) {
        const TS xj = xs[c + C * (m + u)];
#pragma unroll
        for (int q = 0; q < RPL; ++q) acc[u % ng][q] += a[u][q] * xj;
      }
    }
  }
  if (active) {
    // in-register tree levels: global group c + C g; xor offset o >= C is local xor o / C
#pragma unroll
    for (int o = 4; o >= C; o >>= 1) {
      const int lo = o / C;
#pragma unroll
      for (int g = 0; g < ng; ++g)
        if (!(g & lo))
#pragma unroll
          for (int q = 0; q < RPL; ++q) acc[g][q] = acc[g][q] + acc[g | lo][q];
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) red[c * rows + r * RPL + q] = acc[0][q];
  }
  __syncthreads();
  // cross-slot tree levels (offsets C/2 .. 1) and the store
  for (int el = tid; el < rows; el += NTH) {
    const int row = r0 + el;
    TS w[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) w[cc] = red[cc * rows + el];
#pragma unroll
    for (int o = C / 2; o >= 1; o >>= 1)
#pragma unroll
      for (int cc = 0; cc < C; ++cc)
        if (!(cc & o)) w[cc] = w[cc] + w[cc | o];
    if (row < n) dout[row] = w[0];
  }
  __syncthreads();
}

// meta[i] = {first slot, n, inverse offset (low, high 32 bits)} of the i-th
// patch in processing order.
template <typename TS, int W, bool NT>
__global__ void __launch_bounds__(64 * W) patch_apply_kernel(const int4* __restrict__ meta,
                                                             const int* __restrict__ pdofs,
                                                             const TS* __restrict__ inv,
                                                             const double* __restrict__ t,
                                                             TS* __restrict__ delta) {
  constexpr int RPL = 16 / sizeof(TS);
  constexpr int NTH = 64 * W;
  __shared__ TS xs[768];
  __shared__ TS red[8 * 64 * RPL];
  const int4 m4 = meta[blockIdx.x];
  const int base = m4.x, n = m4.y;
  const int64_t off = (int64_t)(uint32_t)m4.z | ((int64_t)m4.w << 32);
  if (n > 768 || n <= 0) return;  // the host rejects patches above 768 DoFs; never taken
  const int ld = (n + RPL - 1) / RPL * RPL;
  const TS* A = inv + off;
  for (int r0 = 0; r0 < ld; r0 += 64 * RPL) {
    const int rows = min(ld - r0, 64 * RPL);
    const int R = rows / RPL;
    const int Cm = NTH / R;
    const bool g = r0 == 0;
    const int* dofs = pdofs + base;
    TS* dout = delta + base;
    if (Cm >= 8) apply_pass<TS, NTH, NT, 8>(A, n, ld, r0, rows, g, dofs, t, xs, red, dout);
    else if (Cm >= 4) apply_pass<TS, NTH, NT, 4>(A, n, ld, r0, rows, g, dofs, t, xs, red, dout);
    else if (Cm >= 2) apply_pass<TS, NTH, NT, 2>(A, n, ld, r0, rows, g, dofs, t, xs, red, dout);
    else apply_pass<TS, NTH, NT, 1>(A, n, ld, r0, rows, g, dofs, t, xs, red, dout);
  }
}


// Exchange with a partner lane through the DPP lane crossbar (a VALU move): CTRL 0xB1
// (quad_perm [1,0,3,2]: lane xor 1), 0x4E (quad_perm [2,3,0,1]: lane xor 2), 0x141 (half-row
// mirror: lane c <-> 7 - c within each group of 8 lanes).
template <int CTRL>
__device__ __forceinline__ double dpp_x(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_x(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// Symmetric tiled apply (storage described at tri_pos): y = S x with S the
// symmetric inverse, from the tiles on and below the diagonal only.  Tile
// (I, J) adds S_IJ x_J to rows 8 I.. and, when I > J, S_IJ^T x_I to rows 8 J...
// Eight lanes take one tile, lane c its column c (8 rows, 16-byte loads); a
// wave takes 8 tiles per step and keeps U steps of loads in flight.  Inside a
// tile the row sums combine the 8 columns by a fixed transposing tree (partners
// 7 - c, then c xor 2, then c xor 1; lane c ends with row c), the column sums are
// lane-local in row order.  Every tile
// writes its partial vectors to Q[I][J][.] (and Q[J][I][.]); row i then sums
// Q[I][0..nb)[i % 8] in ascending J.  Which wave takes which tile changes
// nothing, so the result depends on neither waves nor the cache policy.
template <typename TS, int W, bool NT, int U>
__global__ void __launch_bounds__(64 * W) patch_apply_tri_kernel(const int4* __restrict__ meta,
                                                                 const int* __restrict__ pdofs,
                                                                 const TS* __restrict__ inv,
                                                                 const double* __restrict__ t,
                                                                 TS* __restrict__ delta) {
  constexpr int E = 16 / sizeof(TS);  // rows per 16-byte load
  constexpr int NV = 8 / E;           // loads per tile column
  constexpr int NTH = 64 * W;
  using V = typename vec16<TS>::type;
  extern __shared__ char smem[];
  const int4 m4 = meta[blockIdx.x];
  const int base = m4.x, n = m4.y;
  const int64_t off = (int64_t)(uint32_t)m4.z | ((int64_t)m4.w << 32);
  if (n > 224 || n <= 0) return;  // the launch sizes LDS for every n of the launch; never taken
  const int nb = (n + 7) >> 3;
  const int T = nb * (nb + 1) / 2;
  const int T0 = (nb - 1) * nb / 2;               // first tile of the last block row
  const int nvr = (n - 8 * (nb - 1) + E - 1) / E;  // chunks its tiles keep
  TS* xs = (TS*)smem;   // 8 nb gathered residual entries (zero padding)
  TS* Q = xs + 8 * nb;  // nb x nb x 8 partial vectors
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ts = lane >> 3, c = lane & 7;
  const TS* A = inv + off;
  const int t0 = wave * 8 + ts;
  const int nsteps = T > wave * 8 ? (T - wave * 8 + 8 * W - 1) / (8 * W) : 0;  // wave-uniform
  V a[U][NV];
  auto load_step = [&](int s, V* dst) {
    const int tt = min(t0 + s * 8 * W, T - 1);
    const bool lastrow = tt >= T0;
    const int64_t tile = lastrow ? ((int64_t)T0 << 6) + (int64_t)(tt - T0) * (8 * E * nvr) : ((int64_t)tt << 6);
    const TS* tp = A + tile + c * E;
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[v] = (!lastrow || v < nvr) ? load16<TS, NT>(tp + v * 8 * E) : V{};
  };
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (u < nsteps) load_step(u, a[u]);
  for (int j = tid; j < 8 * nb; j += NTH) xs[j] = j < n ? (TS)t[pdofs[base + j]] : (TS)0;
  __syncthreads();
  for (int s0 = 0; s0 < nsteps; s0 += U) {
    if (s0 > 0) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (s0 + u < nsteps) load_step(s0 + u, a[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (s0 + u >= nsteps) break;
      const int tt = t0 + (s0 + u) * 8 * W;
      const int tc = min(tt, T - 1);  // lanes past the last tile repeat it and write nothing
      int I = (int)((sqrtf(8.f * (float)tc + 1.f) - 1.f) * 0.5f);
      while ((I + 1) * (I + 2) / 2 <= tc) ++I;
      while (I * (I + 1) / 2 > tc) --I;
      const int J = tc - I * (I + 1) / 2;
      TS col[8];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < E; ++e) col[v * E + e] = a[u][v][e];
      // row part: p_k = S[k][c] x_J[c], summed over the 8 columns (lanes)
      const TS xj = xs[8 * J + c];
      TS p[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = col[k] * xj;
      TS q4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {  // keep rows 4 (c & 4) .. + 3, take the same rows of lane 7 - c
        const TS keep = (c & 4) ? p[4 + k] : p[k];
        const TS send = (c & 4) ? p[k] : p[4 + k];
        q4[k] = keep + dpp_x<0x141>(send);  // half-row mirror: lane c <-> 7 - c
      }
      TS q2[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {  // xor 2: keep rows 4 (c & 4) + 2 (c & 2) / 2 ..
        const TS keep = (c & 2) ? q4[2 + k] : q4[k];
        const TS send = (c & 2) ? q4[k] : q4[2 + k];
        q2[k] = keep + dpp_x<0x4E>(send);  // quad_perm [2,3,0,1]: xor 2
      }
      const TS keep = (c & 1) ? q2[1] : q2[0];
      const TS send = (c & 1) ? q2[0] : q2[1];
      const TS rowsum = keep + dpp_x<0xB1>(send);  // quad_perm [1,0,3,2]: xor 1; row c of the tile
      // column part: sum_k S[k][c] x_I[k] in row order
      TS colsum = (TS)0;
#pragma unroll
      for (int k = 0; k < 8; ++k) colsum += col[k] * xs[8 * I + k];
      if (tt < T) {
        Q[(I * nb + J) * 8 + c] = rowsum;
        if (I > J) Q[(J * nb + I) * 8 + c] = colsum;
      }
    }
  }
  __syncthreads();
  TS* dout = delta + base;
  for (int i = tid; i < n; i += NTH) {
    const TS* q = Q + (i >> 3) * nb * 8 + (i & 7);
    TS y = q[0];
    for (int J = 1; J < nb; ++J) y += q[J * 8];
    dout[i] = y;
  }
}

template <typename TS, bool NT, int U>
static void apply_tri_waves(int waves, int count, size_t lds, const int4* meta, const int* pdofs, const TS* inv,
                            const double* t, TS* delta, hipStream_t s) {
  switch (waves) {
    case 1: patch_apply_tri_kernel<TS, 1, NT, U><<<count, 64, lds, s>>>(meta, pdofs, inv, t, delta); break;
    case 2: patch_apply_tri_kernel<TS, 2, NT, U><<<count, 128, lds, s>>>(meta, pdofs, inv, t, delta); break;
    // 8 and 16 waves: fewer tile steps per patch, for latency-bound small levels
    case 8: patch_apply_tri_kernel<TS, 8, NT, U><<<count, 512, lds, s>>>(meta, pdofs, inv, t, delta); break;
    case 16: patch_apply_tri_kernel<TS, 16, NT, U><<<count, 1024, lds, s>>>(meta, pdofs, inv, t, delta); break;
    default: patch_apply_tri_kernel<TS, 4, NT, U><<<count, 256, lds, s>>>(meta, pdofs, inv, t, delta); break;
  }
}

template <typename TS, bool NT>
static void apply_tri_dispatch(int waves, int depth, int nmax, int count, const int4* meta, const int* pdofs,
                               const TS* inv, const double* t, TS* delta, hipStream_t s) {
  if (count <= 0) return;
  const int nb = (std::min(nmax, 224) + 7) / 8;
  const size_t lds = (size_t)(8 * nb + 8 * nb * nb) * sizeof(TS);
  // the load depth (tile steps in flight per lane) trades occupancy against latency hiding
  if (depth >= 4) apply_tri_waves<TS, NT, 4>(waves, count, lds, meta, pdofs, inv, t, delta, s);
  else apply_tri_waves<TS, NT, 2>(waves, count, lds, meta, pdofs, inv, t, delta, s);
}

template <typename TS, bool NT>
static void apply_dispatch(int waves, int count, const int4* meta, const int* pdofs, const TS* inv, const double* t,
                           TS* delta, hipStream_t s) {
  if (count <= 0) return;
  switch (waves) {
    case 1: patch_apply_kernel<TS, 1, NT><<<count, 64, 0, s>>>(meta, pdofs, inv, t, delta); break;
    case 2: patch_apply_kernel<TS, 2, NT><<<count, 128, 0, s>>>(meta, pdofs, inv, t, delta); break;
    default: patch_apply_kernel<TS, 4, NT><<<count, 256, 0, s>>>(meta, pdofs, inv, t, delta); break;
  }
}

void launch_patch_apply(bool fp32, bool tri, int nmax, int waves, bool nontemporal, int depth, int count,
                        const int4* meta, const int* pdofs, const void* inv, const double* t, void* delta,
                        hipStream_t s) {
  if (tri) {
    if (fp32) {
      if (nontemporal)
        apply_tri_dispatch<float, true>(waves, depth, nmax, count, meta, pdofs, (const float*)inv, t, (float*)delta, s);
      else
        apply_tri_dispatch<float, false>(waves, depth, nmax, count, meta, pdofs, (const float*)inv, t, (float*)delta, s);
    } else {
      if (nontemporal)
        apply_tri_dispatch<double, true>(waves, depth, nmax, count, meta, pdofs, (const double*)inv, t, (double*)delta,
                                         s);
      else
        apply_tri_dispatch<double, false>(waves, depth, nmax, count, meta, pdofs, (const double*)inv, t,
                                          (double*)delta, s);
    }
    return;
  }
  if (fp32) {
    if (nontemporal) apply_dispatch<float, true>(waves, count, meta, pdofs, (const float*)inv, t, (float*)delta, s);
    else apply_dispatch<float, false>(waves, count, meta, pdofs, (const float*)inv, t, (float*)delta, s);
  } else {
    if (nontemporal) apply_dispatch<double, true>(waves, count, meta, pdofs, (const double*)inv, t, (double*)delta, s);
    else apply_dispatch<double, false>(waves, count, meta, pdofs, (const double*)inv, t, (double*)delta, s);
  }
}

}  // namespace vk
