// Device-side hierarchy: workspace carving, upload, the additive Vanka
// smoother, the V-cycle and FGMRES (Sec. 3 and Sec. 4 of the paper), and the
// C ABI declared in include/vk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "kernels_multi.hpp"
#include "vk_internal.hpp"

using namespace vk;

#include "hierarchy_internal.hpp"

namespace {

// the longest run of a row-group start list (runs of identical column lists hold at most 8 rows)
int longest_run(const std::vector<int>& grp) {
  int m = 1;
  for (size_t i = 0; i + 1 < grp.size(); ++i) m = std::max(m, grp[i + 1] - grp[i]);
  require(m <= 8, VK_EINVAL, "a run of identical rows longer than 8");
  return m;
}

thread_local std::string g_err;

// K's union groups of a level with patches, runs taken in patch order (built once)
const vk::UnionGroups& k_unions(const vk::LevelHost& lh) {
  if (!lh.kunion_built) {
    lh.kunion = vk::union_groups(lh.K, lh.kgrp, vk::runs_in_patch_order(lh.kgrp, lh.pptr, lh.pdofs));
    lh.kunion_built = true;
  }
  return lh.kunion;
}

// Lays out every device array of the hierarchy `Hs` in the carver; pointers go
// to `h` (a scratch object when only sizing).
// The FGMRES basis also holds the Arnoldi vectors of the Chebyshev estimate
// (`est_steps` + 1 of them, 0 for the damped smoother).
void carve(const std::vector<LevelHost>& Hs, bool fp32, vk_hierarchy* h, Carver& cv, int max_restart, int R,
           int est_steps) {
  const int L = (int)Hs.size();
  const bool cheb = est_steps > 0;
  max_restart = std::max(max_restart, est_steps);
  h->D.assign(L, DevLevel());
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  for (int l = 0; l < L; ++l) {
    const LevelHost& lh = Hs[l];
    DevLevel& d = h->D[l];
    d.N = lh.N;
    d.nvel = lh.nvel;
    d.mean_row = (double)lh.K.nnz() / lh.N;
    d.k_lanes = csr_default_lanes(d.mean_row);
    d.rowptr = cv.take<int>(lh.N + 1);
    d.col = cv.take<int>(lh.K.col.size());
    d.val = cv.take<double>(lh.K.val.size());
    d.nkg = (int)lh.kgrp.size() - 1;
    d.kg_max = longest_run(lh.kgrp);
    d.kgrp = cv.take<int>(lh.kgrp.size());
    d.b = cv.take<double>((size_t)lh.N * R);
    d.x = cv.take<double>((size_t)lh.N * R);
    d.t = cv.take<double>((size_t)lh.N * R);
    if (l == 0) {
      d.M = cv.take<double>((size_t)lh.N * lh.N);
      continue;
    }
    if (R > kUnionMinRhs) {
      const UnionGroups& ug = k_unions(lh);
      d.nug = ug.ngroups();
      d.ug_nval = ug.nval;
      d.ug_ptr = cv.take<int>(ug.gptr.size());
      d.ug_row = cv.take<int>(ug.grow.size());
      d.ug_uptr = cv.take<int>(ug.uptr.size());
      d.ug_col = cv.take<int>(ug.ucol.size());
      d.ug_voff = cv.take<int64_t>(ug.voff.size());
      d.ug_val = cv.take<double>((size_t)ug.nval);
    }
    d.prow = cv.take<int>(lh.P.rowptr.size());
    d.pcol = cv.take<int>(lh.P.col.size());
    d.pval = cv.take<double>(lh.P.val.size());
    d.ptrow = cv.take<int>(lh.PT.rowptr.size());
    d.ptcol = cv.take<int>(lh.PT.col.size());
    d.ptval = cv.take<double>(lh.PT.val.size());
    d.npg = (int)lh.pgrp.size() - 1;
    d.pg_max = longest_run(lh.pgrp);
    d.pgrp = cv.take<int>(lh.pgrp.size());
    d.nptg = (int)lh.ptgrp.size() - 1;
    d.ptg_max = longest_run(lh.ptgrp);
    d.ptgrp = cv.take<int>(lh.ptgrp.size());
    d.p_mean = (double)lh.P.nnz() / std::max(1, lh.P.nrows);
    d.pt_mean = (double)lh.PT.nnz() / std::max(1, lh.PT.nrows);
    d.p_lanes = csr_default_lanes(d.p_mean);
    d.pt_lanes = csr_default_lanes(d.pt_mean);
    for (int i = 0; i + 1 < (int)lh.pptr.size(); ++i)
      if (lh.pptr[i + 1] - lh.pptr[i] > 64) d.n_large++;
    d.max_n = lh.max_n;
    d.J = (int)lh.pptr.size() - 1;
    d.pptr = cv.take<int>(lh.pptr.size());
    d.pdofs = cv.take<int>(lh.pdofs.size());
    d.dptr = cv.take<int>(lh.dptr.size());
    d.dslot = cv.take<int>(lh.dslot.size());
    d.order = cv.take<int>(lh.order.size());
    d.classes = cv.take<int>(lh.order.size());
    d.tri = R == 1 && lh.max_n <= kTiledMaxN;
    d.inv_off = cv.take<int64_t>(lh.inv_off.size());
    d.meta = cv.take<int4>(lh.order.size());
    d.scale = cv.take<double>(lh.scale.size());
    d.inv = cv.take<char>((size_t)(d.tri ? lh.inv_elems_tri : lh.inv_elems) * es);
    d.delta = cv.take<char>(lh.pdofs.size() * es * R);
    if (cheb) d.cd = cv.take<double>((size_t)lh.N * R);
  }
  // scratch of the global-memory inversion (patches above 224 DoFs), shared by the levels
  int64_t big_n = 0;
  int big_count = 0;
  for (int l = 1; l < L; ++l) {
    const LevelHost& lh = Hs[l];
    if (lh.max_n <= kClassLimit[3]) continue;
    big_n = std::max<int64_t>(big_n, lh.max_n);
    int cnt = 0;
    for (int i = 0; i + 1 < (int)lh.pptr.size(); ++i) cnt += lh.pptr[i + 1] - lh.pptr[i] > kClassLimit[3];
    big_count = std::max(big_count, cnt);
  }
  h->big_slots = std::min(big_count, kBigSlots);
  h->big_slot_elems = big_n * big_n;
  h->big_scratch = h->big_slots ? cv.take<double>((size_t)h->big_slots * h->big_slot_elems) : nullptr;
  const int N = Hs.back().N;
  h->V = cv.take<double>((size_t)(max_restart + 1) * N * R);
  h->Z = cv.take<double>((size_t)max_restart * N * R);
  h->bb = cv.take<double>((size_t)N * R);
  h->r = cv.take<double>((size_t)N * R);
  h->partial = cv.take<double>(std::max<size_t>((size_t)kReduceBlocks * 2 * (max_restart + 2) + 512,
                                                (size_t)(max_restart + 2) * kColBlocks * 64 + kColBlocks * 64 + 64));
  h->small = cv.take<double>((size_t)4 * (max_restart + 2) * R + 16);
  h->ydev = cv.take<double>((size_t)(max_restart + 2) * R);
  h->singular = cv.take<int>(64);
  h->nvc = cv.take<int>(64);
  h->mask = cv.take<int>(64);
}

int cheb_steps(const vk_hierarchy* h) { return h->cheb() ? h->opts.est_steps : 0; }

template <typename T>
void up(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (!src.empty()) HIPCHECK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

}  // namespace

void vk::check_launch() { HIPCHECK(hipGetLastError()); }

void vk::spmm_k(const DevLevel& d, int mode, int R, const double* X, const double* B, double* Y, hipStream_t s) {
  if (R > kUnionMinRhs && d.nug > 0) {
    // values, X, Y and (modes 1, 2) B: beyond the last-level cache nothing survives to the next
    // launch, so the single-use operands stream and the L2 keeps the shared X rows
    const double bytes = 8.0 * ((double)d.ug_nval + (mode == 0 ? 2.0 : 3.0) * d.N * R);
    launch_spmm_union(mode, d.nug, d.ug_ptr, d.ug_row, d.ug_uptr, d.ug_col, d.ug_voff, d.ug_val, R, X, B, Y,
                      bytes > kLastLevelCacheBytes, s);
  } else {
    launch_spmm(mode, d.kg_max, d.nkg, d.kgrp, R, d.rowptr, d.col, d.val, X, B, Y, s);
  }
}

namespace {

void require_ready(const vk_hierarchy* h) {
  require(h != nullptr, VK_EINVAL, "null hierarchy");
  require(h->bound, VK_ESTATE, "hierarchy is not bound to a workspace");
  require(h->ready, VK_ESTATE, "vk_patches_setup has not run");
}

void require_level(const vk_hierarchy* h, int level, int lo) {
  require(level >= lo && level < h->L(), VK_EINVAL, "level out of range");
}

// ---------------------------------------------------------------- smoother
void drop_graphs(vk_hierarchy* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
  h->graphs.clear();
}

// An event pair from the hierarchy's pool, its first event recorded on the stream.
std::pair<hipEvent_t, hipEvent_t> timer_start(vk_hierarchy* h) {
  if (h->ev_free.empty()) {
    hipEvent_t a, b;
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    h->ev_free.push_back({a, b});
  }
  auto ev = h->ev_free.back();
  h->ev_free.pop_back();
  HIPCHECK(hipEventRecord(ev.first, h->stream));
  return ev;
}

bool sweep_timed(const vk_hierarchy* h, int l) { return h->sweep_timing && !h->capturing && l == h->L() - 1; }

void sweep_timer_stop(vk_hierarchy* h, std::pair<hipEvent_t, hipEvent_t> ev) {
  HIPCHECK(hipEventRecord(ev.second, h->stream));
  h->sw_pending.push_back(ev);
}

void patch_apply(vk_hierarchy* h, int l, const double* t) {
  DevLevel& d = h->D[l];
  const bool timed = h->timing && !h->capturing && l == h->L() - 1;
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (timed) ev = timer_start(h);
  launch_patch_apply(h->fp32(), d.tri, d.max_n, d.waves_large, d.nt_large != 0, d.depth_large,
                     d.merged ? d.J : d.n_large, d.meta, d.pdofs, d.inv, t, d.delta, h->stream);
  if (!d.merged)
    launch_patch_apply(h->fp32(), d.tri, std::min(d.max_n, 64), d.waves_small, d.nt_small != 0, d.depth_small,
                       d.J - d.n_large, d.meta + d.n_large, d.pdofs, d.inv, t, d.delta, h->stream);
  check_launch();
  if (timed) {
    HIPCHECK(hipEventRecord(ev.second, h->stream));
    h->ev_pending.push_back(ev);
  }
}

// Scatter mode and coefficients of smoothing step `it` of a sequence: the
// damped sweep (scale = omega W), or the Chebyshev iteration on [lambda / 4,
// 1.1 lambda] (scale = W): step 0 sets the direction to W B r / theta, step
// it > 0 to rho' rho d + (2 rho' / delta) W B r with rho' = 1 / (2 sigma - rho).
struct SmoothStep {
  int mode;
  double c1, c2;
};

struct SmoothSchedule {
  bool cheb;
  double sigma = 0, rho = 0, theta = 1, delta = 1;
  SmoothSchedule(const vk_hierarchy* h, const DevLevel& d) : cheb(h->cheb()) {
    if (cheb) {
      theta = d.cheb_theta;
      delta = d.cheb_delta;
      sigma = theta / delta;
      rho = 1.0 / sigma;
    }
  }
  SmoothStep next(int it, bool first_zero) {
    if (!cheb) return {first_zero ? kScatterSet : kScatterAdd, 0.0, 0.0};
    if (it == 0) return {first_zero ? kChebFirstSet : kChebFirstAdd, 0.0, 1.0 / theta};
    const double rn = 1.0 / (2.0 * sigma - rho);
    const SmoothStep st{kChebNext, rn * rho, 2.0 * rn / delta};
    rho = rn;
    return st;
  }
};

// nsweeps smoothing steps on K x = b: x <- x + omega W sum_i R_i^T K_i^{-1} R_i (b - K x)
// (damped), or the Chebyshev steps of SmoothSchedule; if x_zero the first
// residual is b itself (x = 0) and the first update overwrites x.
void smooth(vk_hierarchy* h, int l, const double* b, double* x, int nsweeps, bool x_zero) {
  DevLevel& d = h->D[l];
  const hipStream_t s = h->stream;
  SmoothSchedule sch(h, d);
  for (int it = 0; it < nsweeps; ++it) {
    const bool first_zero = x_zero && it == 0;
    const bool stimed = sweep_timed(h, l);
    std::pair<hipEvent_t, hipEvent_t> sev;
    if (stimed) sev = timer_start(h);
    const double* t = b;
    if (!first_zero) {
      launch_csr(1, d.N, d.k_lanes, d.rowptr, d.col, d.val, x, b, d.t, s);
      t = d.t;
    }
    patch_apply(h, l, t);
    const SmoothStep st = sch.next(it, first_zero);
    launch_scatter_mode(h->fp32(), st.mode, d.N, d.dptr, d.dslot, d.delta, d.scale, st.c1, st.c2, d.cd, x, s);
    check_launch();
    if (stimed) sweep_timer_stop(h, sev);
  }
  if (x_zero && nsweeps == 0) launch_fill(d.N, 0.0, x, s);
}

// e = V-cycle(level l) applied to r, zero initial guess
void vcycle(vk_hierarchy* h, int l, const double* r, double* e, int nu_pre, int nu_post) {
  DevLevel& d = h->D[l];
  const hipStream_t s = h->stream;
  if (l == 0) {
    launch_dense_gemv(d.N, d.M, r, e, s);
    check_launch();
    return;
  }
  DevLevel& c = h->D[l - 1];
  smooth(h, l, r, e, nu_pre, true);
  launch_csr(1, d.N, d.k_lanes, d.rowptr, d.col, d.val, e, r, d.t, s);           // t = r - K e
  launch_csr(0, c.N, d.pt_lanes, d.ptrow, d.ptcol, d.ptval, d.t, nullptr, c.b, s);  // r_c = P^T t
  check_launch();
  vcycle(h, l - 1, c.b, c.x, nu_pre, nu_post);
  launch_csr(2, d.N, d.p_lanes, d.prow, d.pcol, d.pval, c.x, nullptr, e, s);     // e += P e_c
  check_launch();
  smooth(h, l, r, e, nu_post, false);
}

double dot_host(vk_hierarchy* h, int n, const double* a, const double* b) {
  launch_multidot(n, 1, a, 0, b, h->partial, h->small, h->stream);
  check_launch();
  double v;
  HIPCHECK(hipMemcpyAsync(&v, h->small, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return v;
}

// Interval of the Chebyshev smoother on level l (Sec. 3): lambda = the largest
// real part of the Ritz values of est_steps Arnoldi steps on W B K, the vectors
// in the FGMRES basis (carved with room for them), two classical Gram-Schmidt
// passes per step as in FGMRES; the step stops early when the new vector's norm
// is at most 1e-14 times the largest coefficient of its column (an invariant
// subspace: the Ritz values are then exact eigenvalues).
void estimate_lambda(vk_hierarchy* h, int l) {
  DevLevel& d = h->D[l];
  const hipStream_t s = h->stream;
  const int N = d.N, k = h->opts.est_steps;
  const int m = std::max(h->max_restart, k);
  double* V = h->V;
  const bool timing = h->timing;
  h->timing = false;
  launch_splitmix_vector(N, h->opts.est_seed, l, V, s);
  check_launch();
  const double n0 = std::sqrt(dot_host(h, N, V, V));
  require(std::isfinite(n0) && n0 > 0.0, VK_ENAN, "zero start vector of the eigenvalue estimate");
  launch_div(N, V, n0, V, s);
  std::vector<double> H((size_t)k * k, 0.0), hh(3 * (m + 2));
  int steps = k;
  for (int j = 0; j < k; ++j) {
    const double* vj = V + (size_t)j * N;
    double* w = V + (size_t)(j + 1) * N;
    launch_csr(0, N, d.k_lanes, d.rowptr, d.col, d.val, vj, nullptr, d.t, s);  // t = K v_j
    patch_apply(h, l, d.t);
    launch_scatter_mode(h->fp32(), kScatterSet, N, d.dptr, d.dslot, d.delta, d.scale, 0.0, 0.0, nullptr, w, s);
    launch_multidot(N, j + 1, V, N, w, h->partial, h->small, s);
    launch_multiaxpy(N, j + 1, -1.0, V, N, h->small, w, s);
    launch_multidot(N, j + 1, V, N, w, h->partial, h->small + (m + 2), s);
    launch_multiaxpy(N, j + 1, -1.0, V, N, h->small + (m + 2), w, s);
    launch_multidot(N, 1, w, 0, w, h->partial, h->small + 2 * (m + 2), s);
    check_launch();
    HIPCHECK(hipMemcpyAsync(hh.data(), h->small, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    double big = 0.0;
    for (int i = 0; i <= j; ++i) {
      H[(size_t)i * k + j] = hh[i] + hh[(m + 2) + i];
      big = std::max(big, std::fabs(H[(size_t)i * k + j]));
    }
    const double hn = std::sqrt(hh[2 * (m + 2)]);
    require(std::isfinite(hn) && std::isfinite(big), VK_ENAN, "eigenvalue estimate: non-finite Arnoldi vector");
    if (hn <= 1e-14 * big) {
      steps = j + 1;
      break;
    }
    if (j + 1 < k) H[(size_t)(j + 1) * k + j] = hn;
    launch_div_norm(N, w, h->small + 2 * (m + 2), s);
  }
  h->timing = timing;
  std::vector<double> Hs((size_t)steps * steps);
  for (int i = 0; i < steps; ++i)
    for (int j = 0; j < steps; ++j) Hs[(size_t)i * steps + j] = H[(size_t)i * k + j];
  std::vector<std::complex<double>> ev;
  require(hessenberg_eigs(steps, Hs.data(), ev), VK_ENAN, "eigenvalue estimate: QR iteration failed");
  double lam = -INFINITY;
  for (const auto& e : ev) lam = std::max(lam, e.real());
  require(std::isfinite(lam) && lam > 0.0, VK_ENAN,
          "eigenvalue estimate on level " + std::to_string(l) + " is not positive");
  const double a = lam / 4.0, c = 1.1 * lam;
  d.cheb_lambda = lam;
  d.cheb_steps = steps;
  d.cheb_theta = (a + c) / 2.0;
  d.cheb_delta = (c - a) / 2.0;
}

void collect_timing(vk_hierarchy* h) {
  for (auto& ev : h->ev_pending) {
    float ms = 0.f;
    HIPCHECK(hipEventSynchronize(ev.second));
    HIPCHECK(hipEventElapsedTime(&ms, ev.first, ev.second));
    h->t_ms += ms;
    h->t_launches += 1;
    h->ev_free.push_back(ev);
  }
  h->ev_pending.clear();
  for (auto& ev : h->sw_pending) {
    float ms = 0.f;
    HIPCHECK(hipEventSynchronize(ev.second));
    HIPCHECK(hipEventElapsedTime(&ms, ev.first, ev.second));
    h->s_ms += ms;
    h->s_sweeps += 1;
    h->ev_free.push_back(ev);
  }
  h->sw_pending.clear();
}

// One Arnoldi step of FGMRES: z_j = V-cycle(v_j), w = K z_j, two classical
// Gram-Schmidt passes against v_0..v_j (coefficients and |w|^2 left in
// `small`), v_{j+1} = w / |w|.  Everything stays on the device.
void arnoldi_step(vk_hierarchy* h, int j, const vk_solve_opts& o) {
  const int N = h->H.back().N;
  const int m = o.restart;
  const hipStream_t s = h->stream;
  DevLevel& F = h->D[h->L() - 1];
  double* vj = h->V + (size_t)j * N;
  double* zj = h->Z + (size_t)j * N;
  double* w = h->V + (size_t)(j + 1) * N;
  vcycle(h, h->L() - 1, vj, zj, o.nu_pre, o.nu_post);
  launch_csr(0, N, F.k_lanes, F.rowptr, F.col, F.val, zj, nullptr, w, s);
  launch_multidot(N, j + 1, h->V, N, w, h->partial, h->small, s);
  if (j + 1 <= kFusedMaxNv1) {
    // CGS2 with each update fused into the following reduction (bitwise the unfused values)
    launch_axpy_multidot(false, N, j + 1, -1.0, h->V, N, h->small, w, h->partial, h->small + (m + 2), s);
    launch_axpy_multidot(true, N, j + 1, -1.0, h->V, N, h->small + (m + 2), w, h->partial, h->small + 2 * (m + 2), s);
  } else {
    launch_multiaxpy(N, j + 1, -1.0, h->V, N, h->small, w, s);
    launch_multidot(N, j + 1, h->V, N, w, h->partial, h->small + (m + 2), s);
    launch_multiaxpy(N, j + 1, -1.0, h->V, N, h->small + (m + 2), w, s);
    launch_multidot(N, 1, w, 0, w, h->partial, h->small + 2 * (m + 2), s);
  }
  launch_div_norm(N, w, h->small + 2 * (m + 2), s);
  check_launch();
}

// The same step replayed from a HIP graph captured on first use (one graph
// per (j, restart, nu_pre, nu_post); dropped when launch shapes change).
// Replays `step` from the graph cached under `key`, capturing it on first use.
template <typename Step>
void replay_graph(vk_hierarchy* h, const std::tuple<int, int, int, int, int>& key, Step&& step) {
  auto it = h->graphs.find(key);
  if (it == h->graphs.end()) {
    const hipStream_t s = h->stream;
    require(s != nullptr, VK_EINVAL, "graph capture needs a non-default stream");
    hipGraph_t g = nullptr;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    h->capturing = true;
    try {
      step();
    } catch (...) {
      h->capturing = false;
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    h->capturing = false;
    HIPCHECK(hipStreamEndCapture(s, &g));
    hipGraphExec_t ge = nullptr;
    const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHECK(e);
    it = h->graphs.emplace(key, ge).first;
  }
  HIPCHECK(hipGraphLaunch(it->second, h->stream));
}

void arnoldi_step_graph(vk_hierarchy* h, int j, const vk_solve_opts& o) {
  replay_graph(h, std::make_tuple(j, o.restart, o.nu_pre, o.nu_post, 0), [&] { arnoldi_step(h, j, o); });
}

// FGMRES(m) preconditioned by one V-cycle (right preconditioning, stored Z).
vk_status fgmres(vk_hierarchy* h, const double* b_in, double* x, const vk_solve_opts& o, vk_solve_info* info) {
  const int N = h->H.back().N;
  const int Lf = h->L() - 1;
  const int nvel = h->H.back().nvel;
  const double zv = 1.0 / std::sqrt((double)h->H.back().npres);
  const hipStream_t s = h->stream;
  DevLevel& F = h->D[Lf];
  const int m = o.restart;
  // consistent right-hand side: remove the constant-pressure component
  launch_copy(N, b_in, h->bb, s);
  launch_project(N, nvel, zv, h->bb, h->partial, s);
  check_launch();
  const double bnorm = std::sqrt(dot_host(h, N, h->bb, h->bb));
  require(std::isfinite(bnorm), VK_ENAN, "right-hand side is not finite");
  launch_fill(N, 0.0, x, s);
  int its = 0;
  bool converged = false;
  if (info && info->h_history) info->h_history[0] = bnorm;
  if (bnorm == 0.0) {
    if (info) { info->iterations = 0; info->converged = 1; info->rel_residual = 0.0; }
    return VK_OK;
  }
  launch_copy(N, h->bb, h->r, s);
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  // pinned slots for the Hessenberg read-back (allocated once, grown with the restart length)
  const size_t col_elems = 3 * (size_t)(m + 2);
  if (h->hh_pin_elems < 2 * col_elems) {
    if (h->hh_pin) HIPCHECK(hipHostFree(h->hh_pin));
    h->hh_pin = nullptr;
    h->hh_pin_elems = 0;
    HIPCHECK(hipHostMalloc((void**)&h->hh_pin, 2 * col_elems * sizeof(double)));
    h->hh_pin_elems = 2 * col_elems;
  }
  for (auto& e : h->ev_copy)
    if (!e) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  auto step = [&](int j) {
    if (o.use_graphs) arnoldi_step_graph(h, j, o);
    else arnoldi_step(h, j, o);
  };
  double beta = bnorm;
  while (true) {
    beta = std::sqrt(dot_host(h, N, h->r, h->r));
    require(std::isfinite(beta), VK_ENAN, "residual is not finite");
    if (beta <= o.rtol * bnorm) { converged = true; break; }
    if (its >= o.maxit) break;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    launch_div(N, h->r, beta, h->V, s);
    int jlast = -1;
    step(0);
    for (int j = 0; j < m; ++j) {
      // step j is enqueued; copy its Hessenberg column out, then (while the residual estimate is
      // still far from the tolerance) enqueue step j + 1 before waiting for the copy.  Step j + 1
      // depends only on device data, so the result is the same whether or not it runs ahead; if
      // the cycle ends at j, its output (V[j + 2], Z[j + 1]) is simply not used.
      double* hh = h->hh_pin + (size_t)(j & 1) * col_elems;
      HIPCHECK(hipMemcpyAsync(hh, h->small, col_elems * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipEventRecord(h->ev_copy[j & 1], s));
      const bool ahead = j + 1 < m && its + 1 < o.maxit && std::fabs(g[j]) > 100.0 * o.rtol * bnorm;
      if (ahead) step(j + 1);
      HIPCHECK(hipEventSynchronize(h->ev_copy[j & 1]));
      const double hn = std::sqrt(hh[2 * (m + 2)]);
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + hh[(m + 2) + i];
      H[(size_t)(j + 1) * m + j] = hn;
      require(std::isfinite(hn), VK_ENAN, "Arnoldi breakdown to a non-finite value");
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], c2 = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
      }
      const double a = H[(size_t)j * m + j], c2 = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(a, c2);
      cs[j] = a / den;
      sn[j] = c2 / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      jlast = j;
      if (info && info->h_history) info->h_history[its] = std::fabs(g[j + 1]);
      if (std::fabs(g[j + 1]) <= o.rtol * bnorm || its >= o.maxit || hn == 0.0) break;
      if (!ahead && j + 1 < m) step(j + 1);
    }
    const int nk = jlast + 1;
    h->ybuf.assign(nk, 0.0);
    for (int i = nk - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int q = i + 1; q < nk; ++q) sacc -= H[(size_t)i * m + q] * h->ybuf[q];
      h->ybuf[i] = sacc / H[(size_t)i * m + i];
    }
    HIPCHECK(hipMemcpyAsync(h->ydev, h->ybuf.data(), nk * sizeof(double), hipMemcpyHostToDevice, s));
    launch_multiaxpy(N, nk, 1.0, h->Z, N, h->ydev, x, s);
    launch_project(N, nvel, zv, x, h->partial, s);
    launch_csr(1, N, F.k_lanes, F.rowptr, F.col, F.val, x, h->bb, h->r, s);
    check_launch();
  }
  if (info) {
    info->iterations = its;
    info->converged = converged ? 1 : 0;
    info->rel_residual = beta / bnorm;
  }
  if (h->timing || h->sweep_timing) collect_timing(h);
  return converged ? VK_OK : VK_NOT_CONVERGED;
}

// Times `fn` (enqueued on the stream) `reps` times after one warm-up; returns the mean in ms.
template <typename Fn>
float time_ms(hipStream_t s, int reps, Fn&& fn) {
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  fn();
  HIPCHECK(hipEventRecord(a, s));
  for (int i = 0; i < reps; ++i) fn();
  HIPCHECK(hipEventRecord(b, s));
  HIPCHECK(hipEventSynchronize(b));
  float ms = 0.f;
  HIPCHECK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

// Autotuner: for every level, the lanes per CSR row of K, P and P^T and the
// waves per patch of the two apply launches are chosen by timing each
// candidate on the level's own data.  Launch shapes never change results.
void autotune(vk_hierarchy* h, int reps) {
  const hipStream_t s = h->stream;
  const int lanes[5] = {4, 8, 16, 32, 64};
  const int waves[5] = {1, 2, 4, 8, 16};
  // 8 and 16 waves per patch: tiled apply only, and only tried on levels of few patches (they
  // shorten the tile loop where the launch is latency-bound; a full chip gains nothing from them).
  // 16 waves at depth 4 exceed the 64 VGPRs a lane has at 1024 threads and spill: not tried.
  auto wide_ok = [&](const DevLevel& d, int w, int depth, int count) {
    return w <= 4 || (d.tri && count <= kWideApplyMaxPatches && !(w == 16 && depth == 4));
  };
  for (int l = 0; l < h->L(); ++l) {
    DevLevel& d = h->D[l];
    launch_fill(d.N, 1.0, d.b, s);
    launch_fill(d.N, 1.0, d.x, s);
    auto best_lanes = [&](auto&& run) {
      int best = 64;
      float bt = 1e30f;
      for (int ln : lanes) {
        const float t = time_ms(s, reps, [&] { run(ln); });
        if (t < bt * 0.98f) { bt = t; best = ln; }
      }
      return best;
    };
    d.k_lanes = best_lanes([&](int ln) { launch_csr(1, d.N, ln, d.rowptr, d.col, d.val, d.x, d.b, d.t, s); });
    if (l == 0) continue;
    DevLevel& c = h->D[l - 1];
    launch_fill(c.N, 1.0, c.x, s);
    d.p_lanes = best_lanes([&](int ln) { launch_csr(2, d.N, ln, d.prow, d.pcol, d.pval, c.x, nullptr, d.t, s); });
    d.pt_lanes = best_lanes([&](int ln) { launch_csr(0, c.N, ln, d.ptrow, d.ptcol, d.ptval, d.x, nullptr, c.b, s); });
    for (int part = 0; part < 2; ++part) {
      const int first = part == 0 ? 0 : d.n_large;
      const int count = part == 0 ? d.n_large : d.J - d.n_large;
      if (count == 0) continue;
      int best = 1, best_nt = 1, best_depth = 2;
      float bt = 1e30f;
      for (int depth : {2, 4}) {
        if (!d.tri && depth != 2) continue;  // the column-major apply has a fixed depth
        for (int nt = 1; nt >= 0; --nt)
          for (int w : waves) {
            if (!wide_ok(d, w, depth, count)) continue;
            const float t = time_ms(s, reps, [&] {
              launch_patch_apply(h->fp32(), d.tri, part == 0 ? d.max_n : std::min(d.max_n, 64), w, nt != 0, depth,
                                 count, d.meta + first, d.pdofs, d.inv, d.b, d.delta, s);
            });
            if (t < bt * 0.98f) { bt = t; best = w; best_nt = nt; best_depth = depth; }
          }
      }
      (part == 0 ? d.waves_large : d.waves_small) = best;
      (part == 0 ? d.nt_large : d.nt_small) = best_nt;
      (part == 0 ? d.depth_large : d.depth_small) = best_depth;
    }
    // one launch over all patches instead of two (saves a launch where the level is latency-bound)
    d.merged = 0;
    if (d.n_large > 0 && d.n_large < d.J) {
      const float split = time_ms(s, reps, [&] {
        launch_patch_apply(h->fp32(), d.tri, d.max_n, d.waves_large, d.nt_large != 0, d.depth_large, d.n_large,
                           d.meta, d.pdofs, d.inv, d.b, d.delta, s);
        launch_patch_apply(h->fp32(), d.tri, std::min(d.max_n, 64), d.waves_small, d.nt_small != 0, d.depth_small,
                           d.J - d.n_large, d.meta + d.n_large, d.pdofs, d.inv, d.b, d.delta, s);
      });
      float bm = 1e30f;
      int mw = 1, mnt = 1, mdepth = 2;
      for (int depth : {2, 4}) {
        if (!d.tri && depth != 2) continue;
        for (int nt = 1; nt >= 0; --nt)
          for (int w : waves) {
            if (!wide_ok(d, w, depth, d.J)) continue;
            const float t = time_ms(s, reps, [&] {
              launch_patch_apply(h->fp32(), d.tri, d.max_n, w, nt != 0, depth, d.J, d.meta, d.pdofs, d.inv, d.b,
                                 d.delta, s);
            });
            if (t < bm) { bm = t; mw = w; mnt = nt; mdepth = depth; }
          }
      }
      if (bm < split * 0.97f) {
        d.merged = 1;
        d.waves_large = mw;
        d.nt_large = mnt;
        d.depth_large = mdepth;
      }
    }
  }
  check_launch();
}

// ============================================================================ many right-hand sides
// The same smoother, V-cycle and FGMRES as above on multivectors [N][R]; each
// column follows the single-vector algorithm, columns never interact.
void smooth_multi(vk_hierarchy* h, int l, int R, const double* B, double* X, int nsweeps, bool x_zero) {
  DevLevel& d = h->D[l];
  const hipStream_t s = h->stream;
  SmoothSchedule sch(h, d);
  for (int it = 0; it < nsweeps; ++it) {
    const bool first_zero = x_zero && it == 0;
    const bool stimed = sweep_timed(h, l);
    std::pair<hipEvent_t, hipEvent_t> sev;
    if (stimed) sev = timer_start(h);
    const double* T = B;
    if (!first_zero) {
      spmm_k(d, 1, R, X, B, d.t, s);
      T = d.t;
    }
    const bool timed = h->timing && !h->capturing && l == h->L() - 1;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (timed) ev = timer_start(h);
    if (d.tri) {
      // bound for one right-hand side: [N][1] multivectors are plain vectors
      launch_patch_apply(h->fp32(), true, d.max_n, d.waves_large, d.nt_large != 0, d.depth_large,
                         d.merged ? d.J : d.n_large, d.meta, d.pdofs, d.inv, T, d.delta, s);
      if (!d.merged)
        launch_patch_apply(h->fp32(), true, std::min(d.max_n, 64), d.waves_small, d.nt_small != 0, d.depth_small,
                           d.J - d.n_large, d.meta + d.n_large, d.pdofs, d.inv, T, d.delta, s);
    } else {
      launch_patch_gemm(h->fp32(), d.n_large, d.max_n, d.meta, d.pdofs, d.inv, T, R, d.delta, s);
      launch_patch_gemm(h->fp32(), d.J - d.n_large, std::min(d.max_n, 64), d.meta + d.n_large, d.pdofs, d.inv, T, R,
                        d.delta, s);
    }
    if (timed) {
      HIPCHECK(hipEventRecord(ev.second, s));
      h->ev_pending.push_back(ev);
    }
    const SmoothStep st = sch.next(it, first_zero);
    launch_scatter_multi_mode(h->fp32(), st.mode, d.N, R, d.dptr, d.dslot, d.delta, d.scale, st.c1, st.c2, d.cd, X,
                              s);
    check_launch();
    if (stimed) sweep_timer_stop(h, sev);
  }
  if (x_zero && nsweeps == 0) launch_fill(d.N * R, 0.0, X, s);
}

}  // namespace

void vk::vcycle_multi(vk_hierarchy* h, int l, int R, const double* Rv, double* E, int nu_pre, int nu_post) {
  DevLevel& d = h->D[l];
  const hipStream_t s = h->stream;
  if (l == 0) {
    launch_dense_gemm(d.N, R, d.M, Rv, E, s);
    check_launch();
    return;
  }
  DevLevel& c = h->D[l - 1];
  smooth_multi(h, l, R, Rv, E, nu_pre, true);
  spmm_k(d, 1, R, E, Rv, d.t, s);
  launch_spmm(0, d.ptg_max, d.nptg, d.ptgrp, R, d.ptrow, d.ptcol, d.ptval, d.t, nullptr, c.b, s);
  check_launch();
  vcycle_multi(h, l - 1, R, c.b, c.x, nu_pre, nu_post);
  launch_spmm(2, d.pg_max, d.npg, d.pgrp, R, d.prow, d.pcol, d.pval, c.x, nullptr, E, s);
  check_launch();
  smooth_multi(h, l, R, Rv, E, nu_post, false);
}

namespace {

void require_multi(const vk_hierarchy* h, int R) {
  require(R >= 1 && R <= h->max_rhs, VK_EINVAL, "nrhs exceeds the max_rhs the workspace was bound for");
  for (int l = 1; l < h->L(); ++l) {
    if (!h->fp32())
      require(h->H[l].max_n <= 128, VK_EINVAL, "FP64 inverses with many right-hand sides need patches <= 128 DoFs");
    require(h->H[l].max_n <= 512, VK_EINVAL, "many right-hand sides need patches <= 512 DoFs");
  }
}

// sqrt of the column dot products <A_c, B_c> on the host
std::vector<double> col_norms(vk_hierarchy* h, int n, int R, const double* A, const double* B) {
  launch_dots_cols(n, R, 1, A, 0, B, h->partial, h->small, h->stream);
  check_launch();
  std::vector<double> v(R);
  HIPCHECK(hipMemcpyAsync(v.data(), h->small, R * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  for (double& x : v) x = std::sqrt(x);
  return v;
}

vk_status fgmres_multi(vk_hierarchy* h, int R, const double* B, double* X, const vk_solve_opts& o,
                       vk_solve_info* info) {
  const int N = h->H.back().N;
  const int Lf = h->L() - 1;
  const int nvel = h->H.back().nvel;
  const double zv = 1.0 / std::sqrt((double)h->H.back().npres);
  const hipStream_t s = h->stream;
  DevLevel& F = h->D[Lf];
  const int m = o.restart;
  std::vector<int> ones(R, 1);
  HIPCHECK(hipMemcpyAsync(h->mask, ones.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
  launch_copy(N * R, B, h->bb, s);
  launch_project_cols(N, nvel, R, zv, h->mask, h->bb, h->partial, s);
  check_launch();
  const std::vector<double> bnorm = col_norms(h, N, R, h->bb, h->bb);
  for (double v : bnorm) require(std::isfinite(v), VK_ENAN, "right-hand side is not finite");
  launch_fill(N * R, 0.0, X, s);
  launch_copy(N * R, h->bb, h->r, s);
  std::vector<int> conv(R, 0), its_c(R, 0);
  for (int c = 0; c < R; ++c) {
    conv[c] = bnorm[c] == 0.0;
    if (info && info[c].h_history) info[c].h_history[0] = bnorm[c];
  }
  std::vector<double> beta(R, 0.0);
  std::vector<double> Hs((size_t)R * (m + 1) * m), cs((size_t)R * m), sn((size_t)R * m), g((size_t)R * (m + 1));
  std::vector<double> hh((size_t)3 * (m + 2) * R), ybuf((size_t)(m + 2) * R), nn(R);
  std::vector<int> nk(R), running(R), mask(R);
  while (true) {
    beta = col_norms(h, N, R, h->r, h->r);
    // a column takes part in the next cycle if it has not converged and has
    // iterations left (its own count, so a batch never changes its course)
    bool any = false;
    std::vector<int> go(R, 0);
    for (int c = 0; c < R; ++c) {
      require(std::isfinite(beta[c]), VK_ENAN, "residual is not finite");
      if (!conv[c] && beta[c] <= o.rtol * bnorm[c]) conv[c] = 1;
      go[c] = !conv[c] && its_c[c] < o.maxit;
      any = any || go[c];
    }
    if (!any) break;
    for (int c = 0; c < R; ++c) nn[c] = go[c] ? beta[c] * beta[c] : 0.0;
    HIPCHECK(hipMemcpyAsync(h->small, nn.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
    launch_div_sqrt_cols(N, R, h->r, h->small, h->V, s);
    std::fill(Hs.begin(), Hs.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    for (int c = 0; c < R; ++c) {
      g[(size_t)c * (m + 1)] = beta[c];
      running[c] = go[c];
      nk[c] = 0;
    }
    for (int j = 0; j < m; ++j) {
      auto step = [&] {
        const size_t NR = (size_t)N * R;
        double* vj = h->V + j * NR;
        double* zj = h->Z + j * NR;
        double* w = h->V + (j + 1) * NR;
        vk::vcycle_multi(h, Lf, R, vj, zj, o.nu_pre, o.nu_post);
        spmm_k(F, 0, R, zj, nullptr, w, s);
        double* h1 = h->small;
        double* h2 = h->small + (size_t)(m + 2) * R;
        double* nn = h->small + (size_t)2 * (m + 2) * R;
        launch_dots_cols(N, R, j + 1, h->V, NR, w, h->partial, h1, s);
        if (j + 1 <= kFusedMaxNv) {
          // CGS2 with each update fused into the next reduction (one read of the basis fewer)
          launch_axpy_dots_cols(false, N, R, j + 1, nullptr, -1.0, h->V, NR, h1, w, h->partial, h2, s);
          launch_axpy_dots_cols(true, N, R, j + 1, nullptr, -1.0, h->V, NR, h2, w, h->partial, nn, s);
        } else {
          launch_axpy_cols(N, R, j + 1, nullptr, -1.0, h->V, NR, h1, w, s);
          launch_dots_cols(N, R, j + 1, h->V, NR, w, h->partial, h2, s);
          launch_axpy_cols(N, R, j + 1, nullptr, -1.0, h->V, NR, h2, w, s);
          launch_dots_cols(N, R, 1, w, 0, w, h->partial, nn, s);
        }
        launch_div_sqrt_cols(N, R, w, nn, w, s);
        check_launch();
      };
      // every step processes all R columns (finished ones too), so its kernel sequence depends on
      // (j, R, nu) only and can be replayed
      if (o.use_graphs) replay_graph(h, std::make_tuple(j, o.restart, o.nu_pre, o.nu_post, R), step);
      else step();
      HIPCHECK(hipMemcpyAsync(hh.data(), h->small, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      bool still = false;
      for (int c = 0; c < R; ++c) {
        if (!running[c]) continue;
        double* Hc = &Hs[(size_t)c * (m + 1) * m];
        double* gc = &g[(size_t)c * (m + 1)];
        double* csc = &cs[(size_t)c * m];
        double* snc = &sn[(size_t)c * m];
        const double hn = std::sqrt(hh[(size_t)2 * (m + 2) * R + c]);
        require(std::isfinite(hn), VK_ENAN, "Arnoldi breakdown to a non-finite value");
        for (int i = 0; i <= j; ++i) Hc[(size_t)i * m + j] = hh[(size_t)i * R + c] + hh[(size_t)(m + 2) * R + (size_t)i * R + c];
        Hc[(size_t)(j + 1) * m + j] = hn;
        for (int i = 0; i < j; ++i) {
          const double a = Hc[(size_t)i * m + j], b2 = Hc[(size_t)(i + 1) * m + j];
          Hc[(size_t)i * m + j] = csc[i] * a + snc[i] * b2;
          Hc[(size_t)(i + 1) * m + j] = -snc[i] * a + csc[i] * b2;
        }
        const double a = Hc[(size_t)j * m + j], b2 = Hc[(size_t)(j + 1) * m + j];
        const double den = std::hypot(a, b2);
        csc[j] = a / den;
        snc[j] = b2 / den;
        Hc[(size_t)j * m + j] = den;
        Hc[(size_t)(j + 1) * m + j] = 0.0;
        gc[j + 1] = -snc[j] * gc[j];
        gc[j] = csc[j] * gc[j];
        its_c[c] += 1;
        nk[c] = j + 1;
        if (info && info[c].h_history) info[c].h_history[its_c[c]] = std::fabs(gc[j + 1]);
        if (std::fabs(gc[j + 1]) <= o.rtol * bnorm[c] || hn == 0.0 || its_c[c] >= o.maxit) running[c] = 0;
        still = still || running[c];
      }
      if (!still) break;
    }
    std::fill(ybuf.begin(), ybuf.end(), 0.0);
    for (int c = 0; c < R; ++c) {
      mask[c] = go[c];
      if (!go[c]) { nk[c] = 0; continue; }
      const double* Hc = &Hs[(size_t)c * (m + 1) * m];
      const double* gc = &g[(size_t)c * (m + 1)];
      std::vector<double> y(nk[c]);
      for (int i = nk[c] - 1; i >= 0; --i) {
        double acc = gc[i];
        for (int q = i + 1; q < nk[c]; ++q) acc -= Hc[(size_t)i * m + q] * y[q];
        y[i] = acc / Hc[(size_t)i * m + i];
      }
      for (int i = 0; i < nk[c]; ++i) ybuf[(size_t)i * R + c] = y[i];
    }
    HIPCHECK(hipMemcpyAsync(h->ydev, ybuf.data(), (size_t)(m + 2) * R * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(h->nvc, nk.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(h->mask, mask.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
    launch_axpy_cols(N, R, m, h->nvc, 1.0, h->Z, (int64_t)N * R, h->ydev, X, s);
    launch_project_cols(N, nvel, R, zv, h->mask, X, h->partial, s);
    spmm_k(F, 1, R, X, h->bb, h->r, s);
    check_launch();
  }
  if (h->timing || h->sweep_timing) collect_timing(h);
  bool all = true;
  for (int c = 0; c < R; ++c) {
    all = all && conv[c];
    if (info) {
      info[c].iterations = its_c[c];
      info[c].converged = conv[c];
      info[c].rel_residual = bnorm[c] > 0 ? beta[c] / bnorm[c] : 0.0;
    }
  }
  return all ? VK_OK : VK_NOT_CONVERGED;
}

template <typename F>
vk_status guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return VK_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return VK_EINVAL;
  }
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

const char* vk_last_error(void) { return g_err.c_str(); }

vk_status vk_hierarchy_create(const vk_problem* prob, const vk_patch_opts* opts, vk_hierarchy** out) {
  return guarded([&]() -> vk_status {
    require(prob && opts && out, VK_EINVAL, "null argument");
    const vk_problem& p = *prob;
    require(p.dim == 2 || p.dim == 3, VK_EINVAL, "dim must be 2 or 3");
    require(p.family == VK_TH ||
                ((p.family == VK_SV || p.family == VK_TH_QUAD || p.family == VK_BDM) && p.dim == 2),
            VK_EINVAL, "unsupported family");
    if (p.family == VK_SV) require(p.k >= 2 && p.k <= 4, VK_EINVAL, "Scott-Vogelius supports 2 <= k <= 4");
    if (p.family == VK_TH_QUAD)
      require(p.k >= 2 && p.k <= 8, VK_EINVAL, "quadrilateral Taylor-Hood supports 2 <= k <= 8");
    if (p.family == VK_BDM) {
      require(p.k >= 1 && p.k <= 8, VK_EINVAL, "BDM supports 1 <= k <= 8");
      require(p.forcing == VK_F_PAPER_MMS, VK_EINVAL, "BDM levels take the paper's field (VK_F_PAPER_MMS)");
      require(p.penalty >= 0 && std::isfinite(p.penalty), VK_EINVAL, "penalty must be >= 0 (0: default)");
    } else {
      require(p.k >= 2 && p.k <= (p.dim == 2 ? 8 : 2), VK_EINVAL, "unsupported order k");
    }
    require(p.n_coarse >= 1 && p.n_levels >= 2 && p.n_levels <= 12, VK_EINVAL, "bad hierarchy size");
    require(p.viscosity > 0 && std::isfinite(p.viscosity), VK_EINVAL, "viscosity must be positive");
    require(opts->omega > 0 && std::isfinite(opts->omega), VK_EINVAL, "omega must be positive");
    require(opts->store == VK_STORE_FP64 || opts->store == VK_STORE_FP32, VK_EINVAL, "bad store");
    require(opts->smoother == VK_SMOOTH_DAMPED || opts->smoother == VK_SMOOTH_CHEBYSHEV, VK_EINVAL, "bad smoother");
    require(opts->weighting == VK_WEIGHT_MULTIPLICITY || opts->weighting == VK_WEIGHT_NONE, VK_EINVAL,
            "bad weighting");
    require(opts->est_steps >= 0 && opts->est_steps <= 200, VK_EINVAL, "est_steps must be in 0..200");
    if (p.family == VK_SV)
      require(opts->construct == VK_PATCH_MACRO, VK_EINVAL, "Scott-Vogelius levels use VK_PATCH_MACRO");
    else if (p.family == VK_BDM)
      require(opts->construct == VK_PATCH_EXTENDED, VK_EINVAL, "BDM levels use VK_PATCH_EXTENDED");
    else
      require(opts->construct == VK_PATCH_COMPOSITE || (opts->construct == VK_PATCH_STAR && p.dim == 2), VK_EINVAL,
              "bad patch construction");
    const int nf = p.n_coarse << (p.n_levels - 1);
    require((int64_t)nf * p.k * (p.family == VK_SV ? 3 : 1) <= (p.dim == 2 ? 4096 : 256), VK_EINVAL,
            "mesh too fine");
    if (p.dim == 3) require(p.forcing == VK_F_CUBE_MMS, VK_EINVAL, "3D supports the cube field only");
    else require(p.forcing == VK_F_BASELINE_MMS || p.forcing == VK_F_PAPER_MMS || p.forcing == VK_F_RANDOM,
                 VK_EINVAL, "bad forcing");
    auto h = std::make_unique<vk_hierarchy>();
    h->pr.p = p;
    if (p.forcing == VK_F_RANDOM) {
      require(p.n_modes >= 1 && p.n_modes <= 64 && p.h_forcing_coeffs, VK_EINVAL, "random forcing needs coefficients");
      h->pr.coeffs.assign(p.h_forcing_coeffs, p.h_forcing_coeffs + 2 * p.n_modes * p.n_modes);
    }
    h->pr.p.h_forcing_coeffs = nullptr;
    h->opts = *opts;
    if (h->opts.est_steps == 0) h->opts.est_steps = 10;
    h->H.resize(p.n_levels);
    for (int l = 0; l < p.n_levels; ++l) {
      LevelHost& L = h->H[l];
      L.dim = p.dim;
      L.k = p.k;
      L.n = p.n_coarse << l;
      L.family = p.family;
      build_level(L, h->pr, l == p.n_levels - 1);
      L.kgrp = row_groups(L.K, 8);
      if (l > 0) {
        build_prolongation(h->H[l - 1], L);
        L.pgrp = row_groups(L.P, 8);
        L.ptgrp = row_groups(L.PT, 8);
        build_patches(L, opts->construct, opts->omega, opts->store);
        require(L.max_n <= kClassLimit[kClasses - 1], VK_EINVAL, "patches above 768 DoFs are not supported");
        if (opts->smoother == VK_SMOOTH_CHEBYSHEV || opts->weighting == VK_WEIGHT_NONE) {
          // W (and omega for the damped sweep only)
          const double om = opts->smoother == VK_SMOOTH_CHEBYSHEV ? 1.0 : opts->omega;
          for (int dof = 0; dof < L.N; ++dof)
            L.scale[dof] = opts->weighting == VK_WEIGHT_NONE ? om : om / (L.dptr[dof + 1] - L.dptr[dof]);
        }
      }
    }
    h->coarse_M = bordered_inverse(h->H[0]);
    h->class_lists.assign(p.n_levels, {});
    for (int l = 1; l < p.n_levels; ++l) {
      const LevelHost& L = h->H[l];
      std::vector<int>& cl = h->class_lists[l];
      for (int c = 0; c < kClasses; ++c)
        for (int i = 0; i + 1 < (int)L.pptr.size(); ++i) {
          const int n = L.pptr[i + 1] - L.pptr[i];
          if (n <= kClassLimit[c] && (c == 0 || n > kClassLimit[c - 1])) cl.push_back(i);
        }
    }
    *out = h.release();
    return VK_OK;
  });
}

vk_status vk_hierarchy_destroy(vk_hierarchy* h) {
  return guarded([&]() -> vk_status {
    if (!h) return VK_OK;
    drop_graphs(h);
    for (auto& e : h->ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : h->ev_pending) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : h->sw_pending) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : h->ev_copy)
      if (e) (void)hipEventDestroy(e);
    if (h->hh_pin) (void)hipHostFree(h->hh_pin);
    delete h;
    return VK_OK;
  });
}

vk_status vk_hierarchy_workspace_bytes(const vk_hierarchy* h, int max_restart, int max_rhs, size_t* bytes) {
  return guarded([&]() -> vk_status {
    require(h && bytes, VK_EINVAL, "null argument");
    require(max_restart >= 1 && max_restart <= 200, VK_EINVAL, "max_restart out of range");
    require(max_rhs >= 1 && max_rhs <= 64, VK_EINVAL, "max_rhs must be in 1..64");
    vk_hierarchy tmp;  // sizing pass: pointers land in a scratch object
    Carver cv(nullptr);
    carve(h->H, h->fp32(), &tmp, cv, max_restart, max_rhs, cheb_steps(h));
    *bytes = cv.off + 256;
    return VK_OK;
  });
}

vk_status vk_hierarchy_bind(vk_hierarchy* h, void* d_ws, size_t bytes, int max_restart, int max_rhs,
                            void* stream) {
  return guarded([&]() -> vk_status {
    require(h && d_ws, VK_EINVAL, "null argument");
    require(((uintptr_t)d_ws & 255) == 0, VK_EINVAL, "workspace must be 256-byte aligned");
    require(max_restart >= 1 && max_restart <= 200, VK_EINVAL, "max_restart out of range");
    require(max_rhs >= 1 && max_rhs <= 64, VK_EINVAL, "max_rhs must be in 1..64");
    Carver dry(nullptr);
    {
      vk_hierarchy tmp;
      carve(h->H, h->fp32(), &tmp, dry, max_restart, max_rhs, cheb_steps(h));
    }
    require(bytes >= dry.off, VK_ENOMEM, "workspace too small");
    HIPCHECK(hipGetDevice(&h->device));
    h->stream = (hipStream_t)stream;
    h->max_restart = max_restart;
    h->max_rhs = max_rhs;
    drop_graphs(h);
    Carver cv(d_ws);
    carve(h->H, h->fp32(), h, cv, max_restart, max_rhs, cheb_steps(h));
    h->meta_host.clear();
    const hipStream_t s = h->stream;
    for (int l = 0; l < h->L(); ++l) {
      const LevelHost& L = h->H[l];
      DevLevel& d = h->D[l];
      up(d.rowptr, L.K.rowptr, s);
      up(d.col, L.K.col, s);
      up(d.val, L.K.val, s);
      up(d.kgrp, L.kgrp, s);
      if (l == 0) {
        up(d.M, h->coarse_M, s);
        continue;
      }
      up(d.prow, L.P.rowptr, s);
      up(d.pcol, L.P.col, s);
      up(d.pval, L.P.val, s);
      up(d.ptrow, L.PT.rowptr, s);
      up(d.ptcol, L.PT.col, s);
      up(d.ptval, L.PT.val, s);
      up(d.pgrp, L.pgrp, s);
      up(d.ptgrp, L.ptgrp, s);
      if (d.nug > 0) {
        const UnionGroups& ug = k_unions(L);
        up(d.ug_ptr, ug.gptr, s);
        up(d.ug_row, ug.grow, s);
        up(d.ug_uptr, ug.uptr, s);
        up(d.ug_col, ug.ucol, s);
        up(d.ug_voff, ug.voff, s);
        const std::vector<double> v = union_values(L.K, ug);
        up(d.ug_val, v, s);
        HIPCHECK(hipStreamSynchronize(s));  // v is released on return
      }
      up(d.pptr, L.pptr, s);
      up(d.pdofs, L.pdofs, s);
      up(d.dptr, L.dptr, s);
      up(d.dslot, L.dslot, s);
      up(d.order, L.order, s);
      up(d.classes, h->class_lists[l], s);
      const std::vector<int64_t>& ioff = d.tri ? L.inv_off_tri : L.inv_off;
      up(d.inv_off, ioff, s);
      {
        std::vector<int4> meta(L.order.size());
        for (size_t i = 0; i < L.order.size(); ++i) {
          const int p = L.order[i];
          const int64_t o = ioff[p];
          meta[i] = make_int4(L.pptr[p], L.pptr[p + 1] - L.pptr[p], (int)(uint32_t)(o & 0xffffffffLL),
                              (int)(o >> 32));
        }
        h->meta_host.push_back(std::move(meta));
        up(d.meta, h->meta_host.back(), s);
      }
      up(d.scale, L.scale, s);
      for (int c = 0; c < kClasses; ++c) {
        d.class_count[c] = 0;
        for (int i = 0; i + 1 < (int)L.pptr.size(); ++i) {
          const int n = L.pptr[i + 1] - L.pptr[i];
          if (n <= kClassLimit[c] && (c == 0 || n > kClassLimit[c - 1])) d.class_count[c]++;
        }
      }
    }
    HIPCHECK(hipStreamSynchronize(s));
    h->bound = true;
    h->ready = false;
    return VK_OK;
  });
}

vk_status vk_patches_setup(vk_hierarchy* h) {
  return guarded([&]() -> vk_status {
    require(h && h->bound, VK_ESTATE, "hierarchy is not bound");
    const hipStream_t s = h->stream;
    drop_graphs(h);  // captured smoothing steps hold the Chebyshev coefficients
    h->ready = false;
    for (int l = 1; l < h->L(); ++l) {
      DevLevel& d = h->D[l];
      std::vector<int> init(1, INT_MAX);
      HIPCHECK(hipMemcpyAsync(h->singular, init.data(), sizeof(int), hipMemcpyHostToDevice, s));
      int first = 0;
      const LevelHost& lh = h->H[l];
      // tile padding beyond n must read as zero (the register-resident inversion writes only n x n)
      HIPCHECK(hipMemsetAsync(d.inv, 0,
                              (size_t)(d.tri ? lh.inv_elems_tri : lh.inv_elems) * (h->fp32() ? 4 : 8), s));
      for (int c = 0; c < kClasses; ++c) {
        launch_gather_invert(kClassLimit[c], h->fp32(), d.tri, d.class_count[c], d.classes + first, d.pptr,
                             d.pdofs, d.rowptr, d.col, d.val, d.inv_off, d.inv, h->singular, h->big_scratch,
                             h->big_slot_elems, h->big_slots, s);
        check_launch();
        first += d.class_count[c];
      }
      int sing = INT_MAX;
      HIPCHECK(hipMemcpyAsync(&sing, h->singular, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      require(sing == INT_MAX, VK_ESINGULAR,
              "zero pivot in patch " + std::to_string(sing) + " on level " + std::to_string(l));
    }
    if (h->cheb())
      for (int l = 1; l < h->L(); ++l) estimate_lambda(h, l);
    h->ready = true;
    return VK_OK;
  });
}

vk_status vk_level_info_get(const vk_hierarchy* h, int level, vk_level_info* info) {
  return guarded([&]() -> vk_status {
    require(h && info, VK_EINVAL, "null argument");
    require_level(h, level, 0);
    const LevelHost& L = h->H[level];
    info->n = L.n;
    info->n_free = L.N;
    info->n_velocity = L.nvel;
    info->nnz = L.K.nnz();
    info->n_patches = level == 0 ? 0 : (int)L.pptr.size() - 1;
    info->sum_n = level == 0 ? 0 : (int64_t)L.pdofs.size();
    info->sum_n2 = level == 0 ? 0 : L.sum_n2;
    info->max_n = level == 0 ? 0 : L.max_n;
    info->p_nnz = level == 0 ? 0 : L.P.nnz();
    info->inv_elems_full = level == 0 ? 0 : L.inv_elems;
    info->inv_elems_tri = level == 0 ? 0 : L.inv_elems_tri;
    const bool est = h->ready && h->cheb() && level > 0;
    info->cheb_lambda = est ? h->D[level].cheb_lambda : 0.0;
    info->cheb_steps = est ? h->D[level].cheb_steps : 0;
    return VK_OK;
  });
}

vk_status vk_level_csr(const vk_hierarchy* h, int level, int* rp, int* col, double* val) {
  return guarded([&]() -> vk_status {
    require(h && rp && col && val, VK_EINVAL, "null argument");
    require_level(h, level, 0);
    const Csr& K = h->H[level].K;
    std::copy(K.rowptr.begin(), K.rowptr.end(), rp);
    std::copy(K.col.begin(), K.col.end(), col);
    std::copy(K.val.begin(), K.val.end(), val);
    return VK_OK;
  });
}

vk_status vk_level_union_groups(const vk_hierarchy* h, int level, int64_t* sizes, int* gptr, int* grow, int* uptr,
                                int* ucol, int64_t* voff, double* val) {
  return guarded([&]() -> vk_status {
    require(h && sizes, VK_EINVAL, "null argument");
    require_level(h, level, 1);
    const bool all = gptr && grow && uptr && ucol && voff && val;
    require(all || !(gptr || grow || uptr || ucol || voff || val), VK_EINVAL,
            "union group arrays: give all of them or none");
    const LevelHost& L = h->H[level];
    const UnionGroups& g = k_unions(L);
    sizes[0] = g.ngroups();
    sizes[1] = (int64_t)g.grow.size();
    sizes[2] = (int64_t)g.ucol.size();
    sizes[3] = g.nval;
    if (!all) return VK_OK;
    std::copy(g.gptr.begin(), g.gptr.end(), gptr);
    std::copy(g.grow.begin(), g.grow.end(), grow);
    std::copy(g.uptr.begin(), g.uptr.end(), uptr);
    std::copy(g.ucol.begin(), g.ucol.end(), ucol);
    std::copy(g.voff.begin(), g.voff.end(), voff);
    const std::vector<double> v = union_values(L.K, g);
    std::copy(v.begin(), v.end(), val);
    return VK_OK;
  });
}

vk_status vk_level_prolongation(const vk_hierarchy* h, int level, int* rp, int* col, double* val) {
  return guarded([&]() -> vk_status {
    require(h && rp && col && val, VK_EINVAL, "null argument");
    require_level(h, level, 1);
    const Csr& P = h->H[level].P;
    std::copy(P.rowptr.begin(), P.rowptr.end(), rp);
    std::copy(P.col.begin(), P.col.end(), col);
    std::copy(P.val.begin(), P.val.end(), val);
    return VK_OK;
  });
}

vk_status vk_level_patches(const vk_hierarchy* h, int level, int* ptr, int* dofs) {
  return guarded([&]() -> vk_status {
    require(h && ptr && dofs, VK_EINVAL, "null argument");
    require_level(h, level, 1);
    const LevelHost& L = h->H[level];
    std::copy(L.pptr.begin(), L.pptr.end(), ptr);
    std::copy(L.pdofs.begin(), L.pdofs.end(), dofs);
    return VK_OK;
  });
}

vk_status vk_solution_errors(const vk_hierarchy* h, const double* x, double* err) {
  return guarded([&]() -> vk_status {
    require(h && x && err, VK_EINVAL, "null argument");
    require(h->pr.p.forcing != VK_F_RANDOM, VK_EINVAL, "the random forcing has no exact solution");
    solution_errors(h->H.back(), h->pr, x, &err[0], &err[1]);
    return VK_OK;
  });
}

vk_status vk_coarse_inverse(const vk_hierarchy* h, double* out) {
  return guarded([&]() -> vk_status {
    require(h && out, VK_EINVAL, "null argument");
    std::copy(h->coarse_M.begin(), h->coarse_M.end(), out);
    return VK_OK;
  });
}

vk_status vk_dof_coords(const vk_hierarchy* h, int level, double* xyz, int* kind) {
  return guarded([&]() -> vk_status {
    require(h && xyz && kind, VK_EINVAL, "null argument");
    require_level(h, level, 0);
    dof_coords(h->H[level], xyz, kind);
    return VK_OK;
  });
}

vk_status vk_rhs(const vk_hierarchy* h, double* hb) {
  return guarded([&]() -> vk_status {
    require(h && hb, VK_EINVAL, "null argument");
    const LevelHost& L = h->H.back();
    // consistent right-hand side: b - (z.b) z, z = constant pressure / sqrt(#pressure)
    const double zv = 1.0 / std::sqrt((double)L.npres);
    double zb = 0.0;
    for (int i = L.nvel; i < L.N; ++i) zb += L.b[i] * zv;
    for (int i = 0; i < L.N; ++i) hb[i] = i < L.nvel ? L.b[i] : L.b[i] - zb * zv;
    return VK_OK;
  });
}

vk_status vk_patch_gather(vk_hierarchy* h, int level, int first, int count, double* d_out) {
  return guarded([&]() -> vk_status {
    require(h && h->bound && d_out, VK_ESTATE, "hierarchy not bound or null output");
    require_level(h, level, 1);
    const LevelHost& L = h->H[level];
    const int J = (int)L.pptr.size() - 1;
    require(first >= 0 && count >= 0 && first + count <= J, VK_EINVAL, "patch range out of bounds");
    if (count == 0) return VK_OK;
    // the per-patch output offsets go to the FGMRES basis, unused outside a solve
    std::vector<int64_t> off(count);
    int64_t o = 0;
    int nmax = 0;
    for (int i = 0; i < count; ++i) {
      const int n = L.pptr[first + i + 1] - L.pptr[first + i];
      off[i] = o;
      o += (int64_t)n * n;
      nmax = std::max(nmax, n);
    }
    const size_t scratch_bytes = (size_t)(h->max_restart + 1) * h->H.back().N * sizeof(double);
    require(off.size() * sizeof(int64_t) <= scratch_bytes, VK_ENOMEM, "too many patches for one gather call");
    int64_t* d_off = (int64_t*)h->V;
    HIPCHECK(hipMemcpyAsync(d_off, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
    DevLevel& d = h->D[level];
    launch_gather_dense(nmax, first, count, d.pptr, d.pdofs, d.rowptr, d.col, d.val, d_off, d_out, h->stream);
    check_launch();
    HIPCHECK(hipStreamSynchronize(h->stream));
    return VK_OK;
  });
}

vk_status vk_patch_inverse(vk_hierarchy* h, int level, int patch, double* d_out) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(d_out, VK_EINVAL, "null output");
    require_level(h, level, 1);
    const LevelHost& L = h->H[level];
    require(patch >= 0 && patch + 1 < (int)L.pptr.size(), VK_EINVAL, "patch out of range");
    const int n = L.pptr[patch + 1] - L.pptr[patch];
    const DevLevel& dl = h->D[level];
    launch_copy_inverse(h->fp32(), dl.tri, n, dl.inv, dl.tri ? L.inv_off_tri[patch] : L.inv_off[patch], d_out,
                        h->stream);
    check_launch();
    return VK_OK;
  });
}

vk_status vk_spmv(vk_hierarchy* h, int level, const double* x, double* y) {
  return guarded([&]() -> vk_status {
    require(h && h->bound && x && y, VK_ESTATE, "hierarchy not bound or null vector");
    require_level(h, level, 0);
    DevLevel& d = h->D[level];
    launch_csr(0, d.N, d.k_lanes, d.rowptr, d.col, d.val, x, nullptr, y, h->stream);
    check_launch();
    return VK_OK;
  });
}

vk_status vk_spmv_multi(vk_hierarchy* h, int level, const double* X, double* Y, int nrhs) {
  return guarded([&]() -> vk_status {
    require(h && h->bound && X && Y, VK_ESTATE, "hierarchy not bound or null vector");
    require_level(h, level, 0);
    require(nrhs >= 1 && nrhs <= h->max_rhs, VK_EINVAL, "nrhs must be in 1..max_rhs of the bind");
    spmm_k(h->D[level], 0, nrhs, X, nullptr, Y, h->stream);
    check_launch();
    return VK_OK;
  });
}

vk_status vk_restrict(vk_hierarchy* h, int level, const double* rf, double* rc) {
  return guarded([&]() -> vk_status {
    require(h && h->bound && rf && rc, VK_ESTATE, "hierarchy not bound or null vector");
    require_level(h, level, 1);
    DevLevel& d = h->D[level];
    launch_csr(0, h->D[level - 1].N, d.pt_lanes, d.ptrow, d.ptcol, d.ptval, rf, nullptr, rc, h->stream);
    check_launch();
    return VK_OK;
  });
}

vk_status vk_prolong_add(vk_hierarchy* h, int level, const double* ec, double* ef) {
  return guarded([&]() -> vk_status {
    require(h && h->bound && ec && ef, VK_ESTATE, "hierarchy not bound or null vector");
    require_level(h, level, 1);
    DevLevel& d = h->D[level];
    launch_csr(2, d.N, d.p_lanes, d.prow, d.pcol, d.pval, ec, nullptr, ef, h->stream);
    check_launch();
    return VK_OK;
  });
}

vk_status vk_smooth(vk_hierarchy* h, int level, const double* b, double* x, int nsweeps) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(b && x && nsweeps >= 0, VK_EINVAL, "bad argument");
    require_level(h, level, 1);
    smooth(h, level, b, x, nsweeps, false);
    return VK_OK;
  });
}

vk_status vk_smooth_noalloc(vk_hierarchy* h, int level, const double* b, double* x, int nsweeps) {
  return guarded([&]() -> vk_status {
    require(h != nullptr, VK_EINVAL, "null hierarchy");
    require(b && x && nsweeps >= 0, VK_EINVAL, "bad argument");
    require_level(h, level, 1);
    // the sweep's scratch: residual t [N], patch corrections [sum n] (stored precision),
    // Chebyshev direction [N]; each piece 256-byte aligned
    const LevelHost& L = h->H[level];
    const size_t es = h->fp32() ? sizeof(float) : sizeof(double);
    auto up256 = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t t_bytes = up256((size_t)L.N * sizeof(double));
    const size_t d_bytes = up256(L.pdofs.size() * es);
    const size_t c_bytes = h->cheb() ? up256((size_t)L.N * sizeof(double)) : 0;
    require(t_bytes + d_bytes + c_bytes <= kNoAllocScratchBytes, VK_EINVAL,
            "level " + std::to_string(level) + " needs " + std::to_string(t_bytes + d_bytes + c_bytes) +
                " bytes of sweep scratch; vk_smooth_noalloc holds at most " + std::to_string(kNoAllocScratchBytes));
    require_ready(h);
    char* base = (char*)noalloc_scratch(h->device);
    DevLevel& d = h->D[level];
    // point the level's sweep buffers at the fixed scratch for this call (restored on every exit);
    // no timing events either (creating them would allocate)
    struct Swap {
      DevLevel& d;
      vk_hierarchy* h;
      double* t;
      void* delta;
      double* cd;
      bool timing, sweep_timing;
      ~Swap() {
        d.t = t;
        d.delta = delta;
        d.cd = cd;
        h->timing = timing;
        h->sweep_timing = sweep_timing;
      }
    } guard{d, h, d.t, d.delta, d.cd, h->timing, h->sweep_timing};
    h->timing = false;
    h->sweep_timing = false;
    d.t = (double*)base;
    d.delta = base + t_bytes;
    d.cd = h->cheb() ? (double*)(base + t_bytes + d_bytes) : nullptr;
    smooth(h, level, b, x, nsweeps, false);
    return VK_OK;
  });
}

vk_status vk_coarse_solve(vk_hierarchy* h, const double* r, double* e) {
  return guarded([&]() -> vk_status {
    require(h && h->bound && r && e, VK_ESTATE, "hierarchy not bound or null vector");
    launch_dense_gemv(h->D[0].N, h->D[0].M, r, e, h->stream);
    check_launch();
    return VK_OK;
  });
}

vk_status vk_vcycle(vk_hierarchy* h, const double* r, double* e, int nu_pre, int nu_post) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(r && e && nu_pre >= 0 && nu_post >= 0, VK_EINVAL, "bad argument");
    vcycle(h, h->L() - 1, r, e, nu_pre, nu_post);
    return VK_OK;
  });
}

vk_status vk_solve(vk_hierarchy* h, const double* b, double* x, const vk_solve_opts* opts, vk_solve_info* info) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(b && x && opts, VK_EINVAL, "null argument");
    require(opts->restart >= 1 && opts->restart <= h->max_restart, VK_EINVAL, "restart exceeds the bound basis");
    require(opts->maxit >= 0 && opts->rtol >= 0 && opts->nu_pre >= 0 && opts->nu_post >= 0, VK_EINVAL,
            "bad solve options");
    return fgmres(h, b, x, *opts, info);
  });
}


vk_status vk_smooth_multi(vk_hierarchy* h, int level, const double* B, double* X, int nrhs, int nsweeps) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(B && X && nsweeps >= 0, VK_EINVAL, "bad argument");
    require_level(h, level, 1);
    require_multi(h, nrhs);
    smooth_multi(h, level, nrhs, B, X, nsweeps, false);
    return VK_OK;
  });
}

vk_status vk_vcycle_multi(vk_hierarchy* h, const double* Rv, double* E, int nrhs, int nu_pre, int nu_post) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(Rv && E && nu_pre >= 0 && nu_post >= 0, VK_EINVAL, "bad argument");
    require_multi(h, nrhs);
    vcycle_multi(h, h->L() - 1, nrhs, Rv, E, nu_pre, nu_post);
    return VK_OK;
  });
}

vk_status vk_solve_multi(vk_hierarchy* h, const double* B, double* X, int nrhs, const vk_solve_opts* opts,
                         vk_solve_info* info) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(B && X && opts, VK_EINVAL, "null argument");
    require_multi(h, nrhs);
    require(opts->restart >= 1 && opts->restart <= h->max_restart, VK_EINVAL, "restart exceeds the bound basis");
    require(opts->maxit >= 0 && opts->rtol >= 0 && opts->nu_pre >= 0 && opts->nu_post >= 0, VK_EINVAL,
            "bad solve options");
    return fgmres_multi(h, nrhs, B, X, *opts, info);
  });
}

vk_status vk_rhs_random(const vk_hierarchy* h, int n_modes, const double* coeffs, double* hb) {
  return guarded([&]() -> vk_status {
    require(h && coeffs && hb, VK_EINVAL, "null argument");
    require(h->H.back().dim == 2, VK_EINVAL, "random forcing is defined on the unit square");
    require(h->H.back().family != VK_TH_QUAD, VK_EINVAL,
            "quadrilateral levels take the random forcing at create (VK_F_RANDOM)");
    require(h->H.back().family != VK_BDM, VK_EINVAL, "BDM levels take the paper's field only");
    require(n_modes >= 1 && n_modes <= 64, VK_EINVAL, "n_modes out of range");
    // zero boundary velocity: no lifting, pressure rows are zero, so the load is already
    // consistent (orthogonal to the constant pressure)
    const LevelHost& F = h->H.back();
    assemble_random_load(F.family, F.k, F.n, n_modes, coeffs, hb);
    return VK_OK;
  });
}

vk_status vk_autotune(vk_hierarchy* h, int reps) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(reps >= 1 && reps <= 1000, VK_EINVAL, "reps out of range");
    drop_graphs(h);
    autotune(h, reps);
    return VK_OK;
  });
}

}  // extern "C"

namespace {

// Key of a hierarchy in the tuning cache: what fixes the shapes the autotuner can pick and the
// data they run on (problem, patches, storage, right-hand sides) and the device they ran on.
std::string tuning_key(const vk_hierarchy* h) {
  hipDeviceProp_t prop{};
  HIPCHECK(hipGetDeviceProperties(&prop, h->device));
  std::string arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  const vk_problem& p = h->pr.p;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|dim%d|fam%d|k%d|n%d|L%d|pen%.17g|con%d|st%d|sm%d|w%d|rhs%d|cu%d", arch.c_str(),
                p.dim, p.family, p.k, p.n_coarse, p.n_levels, p.penalty, h->opts.construct, h->opts.store,
                h->opts.smoother, h->opts.weighting, h->max_rhs, prop.multiProcessorCount);
  return buf;
}

}  // namespace

extern "C" {

vk_status vk_autotune_cached(vk_hierarchy* h, int reps, const char* path, int* hit) {
  return guarded([&]() -> vk_status {
    require_ready(h);
    require(path && *path, VK_EINVAL, "empty tuning cache path");
    require(reps >= 1 && reps <= 1000, VK_EINVAL, "reps out of range");
    const std::string key = tuning_key(h);
    const int L = h->L();
    std::vector<vk_tuning> found(L);
    std::vector<char> have(L, 0);
    if (FILE* f = std::fopen(path, "r")) {
      char line[1024];
      while (std::fgets(line, sizeof line, f)) {
        char k[512];
        int lv = -1;
        vk_tuning t{};
        const int nread = std::sscanf(line, "%511s %d %d %d %d %d %d %d %d %d %d %d", k, &lv, &t.k_lanes, &t.p_lanes,
                                      &t.pt_lanes, &t.apply_waves_large, &t.apply_waves_small,
                                      &t.apply_nontemporal_large, &t.apply_nontemporal_small, &t.apply_depth_large,
                                      &t.apply_depth_small, &t.apply_merged);
        if (nread == 12 && key == k && lv >= 0 && lv < L) {  // later lines of a key replace earlier ones
          found[lv] = t;
          have[lv] = 1;
        }
      }
      std::fclose(f);
    }
    bool all = true;
    for (int l = 0; l < L; ++l) all = all && have[l];
    if (all) {
      for (int l = 0; l < L; ++l) {
        const vk_status st = vk_tuning_set(h, l, &found[l]);
        if (st != VK_OK) { all = false; break; }  // an entry this build does not accept: tune afresh
      }
    }
    if (hit) *hit = all ? 1 : 0;
    if (all) return VK_OK;
    drop_graphs(h);
    autotune(h, reps);
    FILE* f = std::fopen(path, "a");
    require(f != nullptr, VK_EINVAL, std::string("cannot append to the tuning cache ") + path);
    for (int l = 0; l < L; ++l) {
      vk_tuning t{};
      (void)vk_tuning_get(h, l, &t);
      std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d\n", key.c_str(), l, t.k_lanes, t.p_lanes, t.pt_lanes,
                   t.apply_waves_large, t.apply_waves_small, t.apply_nontemporal_large, t.apply_nontemporal_small,
                   t.apply_depth_large, t.apply_depth_small, t.apply_merged);
    }
    const bool ok = std::fclose(f) == 0;
    require(ok, VK_EINVAL, std::string("cannot write the tuning cache ") + path);
    return VK_OK;
  });
}

vk_status vk_tuning_get(const vk_hierarchy* h, int level, vk_tuning* t) {
  return guarded([&]() -> vk_status {
    require(h && t, VK_EINVAL, "null argument");
    require(h->bound, VK_ESTATE, "hierarchy is not bound");
    require_level(h, level, 0);
    const DevLevel& d = h->D[level];
    t->k_lanes = d.k_lanes;
    t->p_lanes = d.p_lanes;
    t->pt_lanes = d.pt_lanes;
    t->apply_waves_large = d.waves_large;
    t->apply_waves_small = d.waves_small;
    t->apply_nontemporal_large = d.nt_large;
    t->apply_nontemporal_small = d.nt_small;
    t->apply_depth_large = d.depth_large;
    t->apply_depth_small = d.depth_small;
    t->apply_merged = d.merged;
    return VK_OK;
  });
}

vk_status vk_tuning_set(vk_hierarchy* h, int level, const vk_tuning* t) {
  return guarded([&]() -> vk_status {
    require(h && t, VK_EINVAL, "null argument");
    require(h->bound, VK_ESTATE, "hierarchy is not bound");
    require_level(h, level, 0);
    auto okl = [](int v) { return v == 4 || v == 8 || v == 16 || v == 32 || v == 64; };
    const bool tiled = level > 0 && h->D[level].tri;
    auto okw = [tiled](int v) { return v == 1 || v == 2 || v == 4 || (tiled && (v == 8 || v == 16)); };
    require(okl(t->k_lanes) && okl(t->p_lanes) && okl(t->pt_lanes), VK_EINVAL, "lanes must be 4, 8, 16, 32 or 64");
    require(okw(t->apply_waves_large) && okw(t->apply_waves_small), VK_EINVAL,
            "waves must be 1, 2 or 4 (also 8 or 16 on levels with the tiled inverse storage)");
    auto okd = [](int v) { return v == 2 || v == 4; };
    require(okd(t->apply_depth_large) && okd(t->apply_depth_small), VK_EINVAL, "depth must be 2 or 4");
    drop_graphs(h);
    DevLevel& d = h->D[level];
    d.k_lanes = t->k_lanes;
    d.p_lanes = t->p_lanes;
    d.pt_lanes = t->pt_lanes;
    d.waves_large = t->apply_waves_large;
    d.waves_small = t->apply_waves_small;
    d.nt_large = t->apply_nontemporal_large != 0;
    d.nt_small = t->apply_nontemporal_small != 0;
    d.depth_large = t->apply_depth_large;
    d.depth_small = t->apply_depth_small;
    d.merged = t->apply_merged != 0;
    return VK_OK;
  });
}

vk_status vk_sweep_timing(vk_hierarchy* h, int enable, int reset, int64_t* sweeps, double* total_ms) {
  return guarded([&]() -> vk_status {
    require(h, VK_EINVAL, "null hierarchy");
    if (h->bound) {
      HIPCHECK(hipStreamSynchronize(h->stream));
      collect_timing(h);
    }
    if (sweeps) *sweeps = h->s_sweeps;
    if (total_ms) *total_ms = h->s_ms;
    if (reset) { h->s_sweeps = 0; h->s_ms = 0.0; }
    h->sweep_timing = enable != 0;
    return VK_OK;
  });
}

vk_status vk_kernel_timing(vk_hierarchy* h, int enable, int reset, int64_t* launches, double* total_ms) {
  return guarded([&]() -> vk_status {
    require(h, VK_EINVAL, "null hierarchy");
    if (h->bound) {
      HIPCHECK(hipStreamSynchronize(h->stream));
      collect_timing(h);
    }
    if (launches) *launches = h->t_launches;
    if (total_ms) *total_ms = h->t_ms;
    if (reset) { h->t_launches = 0; h->t_ms = 0.0; }
    h->timing = enable != 0;
    return VK_OK;
  });
}

}  // extern "C"
