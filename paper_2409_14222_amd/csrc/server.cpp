// Serving loop: continuous batching of Stokes solves on one GPU.
//
// Requests name a Taylor-Hood problem (mesh n x n, order k, viscosity nu) and
// bring their right-hand side.  One hierarchy per (n, k) is kept resident in
// a caller-owned device pool (first-fit allocator, admission by exact
// footprint, least-recently-used idle hierarchies evicted when a new one
// does not fit).  Each resident hierarchy serves up to `slots` requests as
// the columns of the many-right-hand-side kernels; every column carries its
// own FGMRES state (cycle position, Hessenberg matrix, iteration count), so
// requests join and leave the batch between any two iterations.  One tick
// advances every running request by one FGMRES iteration; the residents'
// work goes to separate streams and overlaps on the device.
//
// Viscosity: a hierarchy is built for nu = 1.  With D_L = diag(nu I, I) and
// D_R = diag(I, I / nu) (velocity, pressure blocks), K_nu = D_L K_1 D_R
// exactly, and the V-cycle built on K_nu equals D_R^{-1} B_1 D_L^{-1} (the
// patch inverses, transfers and the bordered coarsest solve all commute
// with the block scalings).  FGMRES runs on K_nu itself (true residual of
// the request's own system); only the operator applications are scaled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <vector>

#include "hierarchy_internal.hpp"
#include "kernels.hpp"
#include "kernels_multi.hpp"

using namespace vk;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Slot {
  bool used = false;   // holds a request
  bool fresh = false;  // admitted this tick, state not initialised yet
  uint64_t ticket = 0;
  double nu = 1.0;
  int j = -1;          // position in the current restart cycle (-1: no Arnoldi step pending)
  int its = 0;
  double bnorm = 0.0, beta = 0.0;
  std::vector<double> H, g, cs, sn;
  std::vector<double> b;  // right-hand side until uploaded
  double* out = nullptr;  // caller's host buffer for the solution
};

struct Resident {
  int n = 0, k = 0;
  vk_hierarchy* h = nullptr;
  size_t off = 0, bytes = 0;      // hierarchy workspace in the pool
  size_t aux_off = 0, aux_bytes = 0;
  hipStream_t stream = nullptr;
  int N = 0, nvel = 0, S = 0;
  std::vector<Slot> slots;
  double last_used = 0.0;
  // auxiliary device arrays: solutions X [N][S], Arnoldi work vector W [N][S],
  // a one-column staging buffer, per-column parameters
  double *X = nullptr, *W = nullptr, *stage = nullptr, *colv = nullptr;  // colv: 8 arrays of 64
  int* coli = nullptr;                                                     // 4 arrays of 64
  // pinned host staging for the small per-tick uploads: one fixed region per
  // purpose, rewritten only in the next tick (every tick ends with the
  // resident's stream synchronised)
  double* hd = nullptr;  // 6 x 64 doubles + y
  int* hi = nullptr;     // 12 x 64 ints
  int busy() const {
    int c = 0;
    for (const Slot& s : slots) c += s.used;
    return c;
  }
};

struct Ticket {
  int state = 0;  // 0 queued, 1 running, 2 done
  vk_status status = VK_OK;
  int iterations = 0;
  double rel_residual = 0.0;
  double t_submit = 0.0, t_done = 0.0;
};

struct Pending {
  uint64_t ticket;
  int n, k;
  double nu;
  std::vector<double> b;
  double* out;
};

}  // namespace

struct vk_server {
  vk_server_opts opts{};
  char* pool = nullptr;
  size_t pool_bytes = 0;
  std::list<std::pair<size_t, size_t>> free_blocks;  // (offset, size), ascending offsets
  std::map<std::pair<int, int>, std::unique_ptr<Resident>> res;
  // host-assembled hierarchies waiting for pool space (kept so that a request
  // that has to wait does not trigger a new assembly every tick)
  std::map<std::pair<int, int>, vk_hierarchy*> parked;
  std::deque<Pending> queue;
  std::map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  int64_t completed = 0;
  std::vector<double> latencies;
  double t_first = -1.0, t_last = 0.0;
  int64_t evictions = 0;
  // caller-owned HIP streams; residents take them in turn (never created or destroyed here)
  std::vector<hipStream_t> streams;
  size_t next_stream = 0;
};

namespace {

thread_local std::string s_err;

template <typename F>
vk_status sguard(F&& f) {
  try {
    s_err.clear();
    return f();
  } catch (const Error& e) {
    s_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    s_err = "host allocation failed";
    return VK_ENOMEM;
  } catch (const std::exception& e) {
    s_err = e.what();
    return VK_EINVAL;
  }
}

bool pool_alloc(vk_server* s, size_t bytes, size_t* off) {
  bytes = (bytes + 255) / 256 * 256;
  for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      it->first += bytes;
      it->second -= bytes;
      if (it->second == 0) s->free_blocks.erase(it);
      return true;
    }
  }
  return false;
}

void pool_free(vk_server* s, size_t off, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  auto it = s->free_blocks.begin();
  while (it != s->free_blocks.end() && it->first < off) ++it;
  it = s->free_blocks.insert(it, {off, bytes});
  auto nx = std::next(it);
  if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_blocks.erase(nx);
  }
  if (it != s->free_blocks.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_blocks.erase(it);
    }
  }
}

size_t aux_bytes_for(int N, int S) {
  return ((size_t)2 * N * S + N + 8 * 64) * sizeof(double) + 4 * 64 * sizeof(int) + 1024;
}

void evict(vk_server* s, Resident* r) {
  if (r->stream) (void)hipStreamSynchronize(r->stream);
  if (r->hd) (void)hipHostFree(r->hd);
  if (r->hi) (void)hipHostFree(r->hi);
  vk_hierarchy_destroy(r->h);
  pool_free(s, r->off, r->bytes);
  s->evictions++;
  s->res.erase({r->n, r->k});
}

int levels_for(int n) {
  int L = 1;
  while ((4 << (L - 1)) < n) ++L;
  require((4 << (L - 1)) == n, VK_EINVAL, "mesh size must be 4 * 2^m (coarsest level 4 x 4)");
  require(L >= 2, VK_EINVAL, "mesh size must be at least 8");
  return L;
}

// Makes (n, k) resident, evicting idle hierarchies if the pool is full.
// Returns nullptr if it cannot fit even then.
Resident* make_resident(vk_server* s, int n, int k) {
  auto key = std::make_pair(n, k);
  auto it = s->res.find(key);
  if (it != s->res.end()) return it->second.get();
  vk_problem p{};
  p.dim = 2;
  p.family = VK_TH;
  p.k = k;
  p.n_coarse = 4;
  p.n_levels = levels_for(n);
  p.viscosity = 1.0;
  p.forcing = VK_F_BASELINE_MMS;
  vk_patch_opts po{VK_PATCH_COMPOSITE, s->opts.store, s->opts.omega};
  vk_hierarchy* h = nullptr;
  vk_status st = VK_OK;
  auto pk = s->parked.find(key);
  if (pk != s->parked.end()) {
    h = pk->second;
    s->parked.erase(pk);
  } else {
    st = vk_hierarchy_create(&p, &po, &h);
    if (st != VK_OK) throw Error(st, std::string("hierarchy: ") + vk_last_error());
  }
  std::unique_ptr<vk_hierarchy, vk_status (*)(vk_hierarchy*)> guard(h, vk_hierarchy_destroy);
  size_t bytes = 0;
  st = vk_hierarchy_workspace_bytes(h, s->opts.restart, s->opts.slots, &bytes);
  if (st != VK_OK) throw Error(st, vk_last_error());
  const int N = h->H.back().N;
  // workspace and auxiliary arrays form one block, so that admission and
  // eviction see the whole footprint
  const size_t ws = (bytes + 255) / 256 * 256;
  const size_t ab = aux_bytes_for(N, s->opts.slots);
  size_t off = 0;
  while (!pool_alloc(s, ws + ab, &off)) {
    // evict the least recently used idle resident
    Resident* victim = nullptr;
    for (auto& kv : s->res)
      if (kv.second->busy() == 0 && (!victim || kv.second->last_used < victim->last_used)) victim = kv.second.get();
    if (!victim) {
      s->parked[key] = guard.release();
      return nullptr;
    }
    evict(s, victim);
  }
  const size_t aoff = off + ws;
  auto r = std::make_unique<Resident>();
  r->n = n;
  r->k = k;
  r->off = off;
  r->bytes = ws + ab;  // the whole block
  r->aux_off = aoff;
  r->aux_bytes = ab;
  r->stream = s->streams[s->next_stream++ % s->streams.size()];
  st = vk_hierarchy_bind(h, s->pool + off, bytes, s->opts.restart, s->opts.slots, r->stream);
  if (st == VK_OK) st = vk_patches_setup(h);
  if (st != VK_OK) {
    const std::string msg = vk_last_error();
    pool_free(s, off, ws + ab);
    throw Error(st, "resident setup: " + msg);
  }
  r->h = guard.release();
  r->N = N;
  r->nvel = h->H.back().nvel;
  r->S = s->opts.slots;
  r->slots.resize(r->S);
  char* a = s->pool + aoff;
  r->X = (double*)a;
  r->W = r->X + (size_t)N * r->S;
  r->stage = r->W + (size_t)N * r->S;
  r->colv = r->stage + N;
  r->coli = (int*)(r->colv + 8 * 64);
  const int m = s->opts.restart;
  HIPCHECK(hipHostMalloc((void**)&r->hd, ((size_t)6 * 64 + (size_t)(m + 2) * 64) * sizeof(double)));
  HIPCHECK(hipHostMalloc((void**)&r->hi, (size_t)12 * 64 * sizeof(int)));
  for (int i = 0; i < 12 * 64; ++i) r->hi[i] = 0;  // region 0 stays the all-zero column array
  r->last_used = now_s();
  Resident* out = r.get();
  s->res[key] = std::move(r);
  return out;
}

// pinned host regions
enum { HD_NU = 0, HD_INV = 1, HD_ONE = 2, HD_SCALE_A = 3, HD_SCALE_C = 4, HD_Y = 6 };
enum { HI_ZERO = 0, HI_RST_A = 1, HI_RST_C = 2, HI_JC = 3, HI_JN = 4, HI_NVC_B = 5, HI_NVC_C = 6, HI_MASK_A = 7,
       HI_MASK_C = 8 };
inline double* hdp(Resident* r, int i) { return r->hd + 64 * i; }
inline int* hip_(Resident* r, int i) { return r->hi + 64 * i; }

// per-column arrays on the device (64 entries each)
enum { CV_NU = 0, CV_INVNU = 1, CV_ONE = 2, CV_SCALE = 3 };
enum { CI_JC = 0, CI_MASK = 1, CI_NVC = 2, CI_JNEXT = 3 };
inline double* cvp(Resident* r, int i) { return r->colv + 64 * i; }
inline int* cip(Resident* r, int i) { return r->coli + 64 * i; }

template <typename T>
void h2d(Resident* r, T* dst, const T* pinned_src, size_t count) {
  HIPCHECK(hipMemcpyAsync(dst, pinned_src, count * sizeof(T), hipMemcpyHostToDevice, r->stream));
}

void upload_nu(Resident* r) {
  double* nu = hdp(r, HD_NU);
  double* inv = hdp(r, HD_INV);
  double* one = hdp(r, HD_ONE);
  for (int c = 0; c < 64; ++c) {
    const bool u = c < r->S && r->slots[c].used;
    nu[c] = u ? r->slots[c].nu : 1.0;
    inv[c] = 1.0 / nu[c];
    one[c] = 1.0;
  }
  h2d(r, cvp(r, CV_NU), nu, 64);
  h2d(r, cvp(r, CV_INVNU), inv, 64);
  h2d(r, cvp(r, CV_ONE), one, 64);
}

// r = bb - K_nu X = bb - D_L K_1 D_R X for every column
void enqueue_residual(Resident* r) {
  vk_hierarchy* h = r->h;
  DevLevel& F = h->D[h->L() - 1];
  const hipStream_t st = r->stream;
  h2d(r, cip(r, CI_JNEXT), hip_(r, HI_ZERO), 64);
  launch_gather_slice(r->N, r->S, r->nvel, r->X, 0, cip(r, CI_JNEXT), cvp(r, CV_ONE), cvp(r, CV_INVNU), F.b, st);
  spmm_k(F, 0, r->S, F.b, nullptr, F.t, st);
  launch_residual_scaled(r->N, r->S, r->nvel, h->bb, F.t, cvp(r, CV_NU), h->r, st);
  check_launch();
}

// column norms of A (enqueued; read after the stream synchronises)
void enqueue_norms(Resident* r, const double* A, double* dst_small) {
  launch_dots_cols(r->N, r->S, 1, A, 0, A, r->h->partial, dst_small, r->stream);
  check_launch();
}

// V[0][:, c] = r[:, c] / beta_c for the columns in `cols` (phase 0: admission, 1: cycle end)
void enqueue_restart(Resident* r, const std::vector<int>& cols, int phase) {
  double* sc = hdp(r, phase ? HD_SCALE_C : HD_SCALE_A);
  int* jc = hip_(r, phase ? HI_RST_C : HI_RST_A);
  for (int c = 0; c < 64; ++c) {
    sc[c] = 0.0;
    jc[c] = -1;
  }
  for (int c : cols) {
    sc[c] = 1.0 / r->slots[c].beta;
    jc[c] = 0;
  }
  h2d(r, cvp(r, CV_SCALE), sc, 64);
  h2d(r, cip(r, CI_MASK), jc, 64);
  launch_scatter_slice(r->N, r->S, r->nvel, r->h->r, cvp(r, CV_SCALE), cvp(r, CV_SCALE), cip(r, CI_MASK), r->h->V,
                       (int64_t)r->N * r->S, r->stream);
  check_launch();
}

// One Arnoldi step for every column with j >= 0.
void enqueue_arnoldi(Resident* r, int m, int nu_pre, int nu_post) {
  vk_hierarchy* h = r->h;
  DevLevel& F = h->D[h->L() - 1];
  const hipStream_t st = r->stream;
  const int64_t slice = (int64_t)r->N * r->S;
  int* jc = hip_(r, HI_JC);
  int* jn = hip_(r, HI_JN);
  int* nvc = hip_(r, HI_NVC_B);
  for (int c = 0; c < 64; ++c) {
    jc[c] = -1;
    jn[c] = -1;
    nvc[c] = 0;
  }
  int jmax = 0;
  for (int c = 0; c < r->S; ++c) {
    const Slot& sl = r->slots[c];
    if (!sl.used || sl.j < 0) continue;
    jc[c] = sl.j;
    jn[c] = sl.j + 1;
    nvc[c] = sl.j + 1;
    jmax = std::max(jmax, sl.j);
  }
  h2d(r, cip(r, CI_JC), jc, 64);
  h2d(r, cip(r, CI_JNEXT), jn, 64);
  h2d(r, cip(r, CI_NVC), nvc, 64);
  // D_L^{-1} v_j -> V-cycle on K_1 -> z_j = D_R^{-1} (.)
  launch_gather_slice(r->N, r->S, r->nvel, h->V, slice, cip(r, CI_JC), cvp(r, CV_INVNU), cvp(r, CV_ONE), F.b, st);
  vcycle_multi(h, h->L() - 1, r->S, F.b, F.x, nu_pre, nu_post);
  launch_scatter_slice(r->N, r->S, r->nvel, F.x, cvp(r, CV_ONE), cvp(r, CV_NU), cip(r, CI_JC), h->Z, slice, st);
  // w = K_nu z_j = D_L K_1 (D_R z_j) and D_R z_j is the V-cycle output itself
  spmm_k(F, 0, r->S, F.x, nullptr, F.t, st);
  h2d(r, cip(r, CI_MASK), hip_(r, HI_ZERO), 64);
  launch_gather_slice(r->N, r->S, r->nvel, F.t, 0, cip(r, CI_MASK), cvp(r, CV_NU), cvp(r, CV_ONE), r->W, st);
  // CGS2 against v_0 .. v_j (per-column counts), norm, normalisation, store as v_{j+1}
  double* h1 = h->small;
  double* h2 = h->small + (size_t)(m + 2) * r->S;
  double* nn = h->small + (size_t)2 * (m + 2) * r->S;
  launch_dots_cols(r->N, r->S, jmax + 1, h->V, slice, r->W, h->partial, h1, st);
  if (jmax + 1 <= kFusedMaxNv) {
    // each update fused with the following reduction (one read of the basis fewer per pass)
    launch_axpy_dots_cols(false, r->N, r->S, jmax + 1, cip(r, CI_NVC), -1.0, h->V, slice, h1, r->W, h->partial, h2,
                          st);
    launch_axpy_dots_cols(true, r->N, r->S, jmax + 1, cip(r, CI_NVC), -1.0, h->V, slice, h2, r->W, h->partial, nn,
                          st);
  } else {
    launch_axpy_cols(r->N, r->S, jmax + 1, cip(r, CI_NVC), -1.0, h->V, slice, h1, r->W, st);
    launch_dots_cols(r->N, r->S, jmax + 1, h->V, slice, r->W, h->partial, h2, st);
    launch_axpy_cols(r->N, r->S, jmax + 1, cip(r, CI_NVC), -1.0, h->V, slice, h2, r->W, st);
    launch_dots_cols(r->N, r->S, 1, r->W, 0, r->W, h->partial, nn, st);
  }
  launch_div_sqrt_cols(r->N, r->S, r->W, nn, r->W, st);
  launch_scatter_slice(r->N, r->S, r->nvel, r->W, cvp(r, CV_ONE), cvp(r, CV_ONE), cip(r, CI_JNEXT), h->V, slice, st);
  check_launch();
}

void finish_ticket(vk_server* s, uint64_t t, vk_status st, int its, double rel) {
  Ticket& tk = s->tickets[t];
  tk.state = 2;
  tk.status = st;
  tk.iterations = its;
  tk.rel_residual = rel;
  tk.t_done = now_s();
  s->completed++;
  s->latencies.push_back(tk.t_done - tk.t_submit);
  s->t_last = tk.t_done;
}

}  // namespace

extern "C" {

const char* vk_server_last_error(void) { return s_err.c_str(); }

vk_status vk_server_create(const vk_server_opts* opts, void* d_pool, size_t pool_bytes, void* const* hip_streams,
                           int n_streams, vk_server** out) {
  return sguard([&]() -> vk_status {
    require(opts && d_pool && out && hip_streams, VK_EINVAL, "null argument");
    require(n_streams >= 1 && n_streams <= 64, VK_EINVAL, "n_streams must be in 1..64");
    for (int i = 0; i < n_streams; ++i)
      require(hip_streams[i] != nullptr, VK_EINVAL, "the null stream cannot serve a resident (use created streams)");
    require(((uintptr_t)d_pool & 255) == 0, VK_EINVAL, "pool must be 256-byte aligned");
    require(opts->slots >= 1 && opts->slots <= 64, VK_EINVAL, "slots must be in 1..64");
    require(opts->restart >= 1 && opts->restart <= 200 && opts->maxit >= 1, VK_EINVAL, "bad Krylov options");
    require(opts->store == VK_STORE_FP64 || opts->store == VK_STORE_FP32, VK_EINVAL, "bad store");
    require(opts->omega > 0 && opts->rtol > 0 && opts->nu_sweeps >= 0, VK_EINVAL, "bad smoother options");
    require(opts->max_queue >= 1, VK_EINVAL, "max_queue must be positive");
    auto s = std::make_unique<vk_server>();
    s->opts = *opts;
    s->pool = (char*)d_pool;
    s->pool_bytes = pool_bytes / 256 * 256;
    s->free_blocks.push_back({0, s->pool_bytes});
    for (int i = 0; i < n_streams; ++i) s->streams.push_back((hipStream_t)hip_streams[i]);
    *out = s.release();
    return VK_OK;
  });
}

vk_status vk_server_destroy(vk_server* s) {
  return sguard([&]() -> vk_status {
    if (!s) return VK_OK;
    while (!s->res.empty()) evict(s, s->res.begin()->second.get());
    for (auto& kv : s->parked) vk_hierarchy_destroy(kv.second);
    delete s;
    return VK_OK;
  });
}

vk_status vk_server_prepare(vk_server* s, int n, int k) {
  return sguard([&]() -> vk_status {
    require(s != nullptr, VK_EINVAL, "null server");
    Resident* r = make_resident(s, n, k);
    require(r != nullptr, VK_ENOMEM, "the hierarchy does not fit in the pool");
    return VK_OK;
  });
}

vk_status vk_server_problem_size(vk_server* s, int n, int k, int* n_free) {
  return sguard([&]() -> vk_status {
    require(s && n_free, VK_EINVAL, "null argument");
    require(k >= 2 && k <= 6, VK_EINVAL, "order out of range");
    (void)levels_for(n);
    *n_free = 2 * (k * n - 1) * (k * n - 1) + ((k - 1) * n + 1) * ((k - 1) * n + 1);
    return VK_OK;
  });
}

vk_status vk_server_submit(vk_server* s, const vk_request* req, double* h_x, uint64_t* ticket) {
  return sguard([&]() -> vk_status {
    require(s && req && req->h_b && h_x && ticket, VK_EINVAL, "null argument");
    require(req->viscosity > 0 && std::isfinite(req->viscosity), VK_EINVAL, "viscosity must be positive");
    require(req->k >= 2 && req->k <= 6, VK_EINVAL, "order out of range");
    (void)levels_for(req->n);
    if ((int)s->queue.size() >= s->opts.max_queue) return VK_EBUSY;
    const int k = req->k, n = req->n;
    const int N = 2 * (k * n - 1) * (k * n - 1) + ((k - 1) * n + 1) * ((k - 1) * n + 1);
    Pending p{s->next_ticket++, n, k, req->viscosity, std::vector<double>(req->h_b, req->h_b + N), h_x};
    for (double v : p.b) require(std::isfinite(v), VK_ENAN, "right-hand side is not finite");
    Ticket& tk = s->tickets[p.ticket];
    tk.t_submit = now_s();
    if (s->t_first < 0) s->t_first = tk.t_submit;
    *ticket = p.ticket;
    s->queue.push_back(std::move(p));
    return VK_OK;
  });
}

vk_status vk_server_tick(vk_server* s, int* active) {
  return sguard([&]() -> vk_status {
    require(s != nullptr, VK_EINVAL, "null server");
    const int m = s->opts.restart;
    // ---- admission: FIFO, no head-of-line blocking across problem types,
    // except that a request waiting for memory stops all later admissions
    for (auto it = s->queue.begin(); it != s->queue.end();) {
      Resident* r = nullptr;
      try {
        r = make_resident(s, it->n, it->k);
      } catch (const Error& e) {
        finish_ticket(s, it->ticket, e.code, 0, 0.0);
        it = s->queue.erase(it);
        continue;
      }
      if (!r) {
        bool any_busy = false;
        for (auto& kv : s->res) any_busy = any_busy || kv.second->busy() > 0;
        if (!any_busy) {  // can never fit
          finish_ticket(s, it->ticket, VK_ENOMEM, 0, 0.0);
          it = s->queue.erase(it);
          continue;
        }
        break;
      }
      int slot = -1;
      for (int c = 0; c < r->S; ++c)
        if (!r->slots[c].used) { slot = c; break; }
      if (slot < 0) { ++it; continue; }
      Slot& sl = r->slots[slot];
      sl = Slot();
      sl.used = true;
      sl.fresh = true;
      sl.ticket = it->ticket;
      sl.nu = it->nu;
      sl.b = std::move(it->b);
      sl.out = it->out;
      sl.H.assign((size_t)(m + 1) * m, 0.0);
      sl.g.assign(m + 1, 0.0);
      sl.cs.assign(m, 0.0);
      sl.sn.assign(m, 0.0);
      s->tickets[it->ticket].state = 1;
      r->last_used = now_s();
      it = s->queue.erase(it);
    }
    // ---- phase A: initialise fresh columns (upload b, project, residual, norms)
    std::vector<Resident*> act;
    for (auto& kv : s->res)
      if (kv.second->busy() > 0) act.push_back(kv.second.get());
    std::vector<std::vector<int>> fresh(act.size());
    for (size_t a = 0; a < act.size(); ++a) {
      Resident* r = act[a];
      vk_hierarchy* h = r->h;
      upload_nu(r);
      int* mask = hip_(r, HI_MASK_A);
      for (int c = 0; c < 64; ++c) mask[c] = 0;
      for (int c = 0; c < r->S; ++c) {
        Slot& sl = r->slots[c];
        if (!sl.fresh) continue;
        HIPCHECK(hipMemcpyAsync(r->stage, sl.b.data(), r->N * sizeof(double), hipMemcpyHostToDevice, r->stream));
        launch_column_put(r->N, r->S, c, r->stage, h->bb, r->stream);
        launch_column_put(r->N, r->S, c, nullptr, r->X, r->stream);
        HIPCHECK(hipStreamSynchronize(r->stream));  // the staging buffer is reused by the next column
        sl.b.clear();
        sl.b.shrink_to_fit();
        mask[c] = 1;
        fresh[a].push_back(c);
      }
      if (fresh[a].empty()) continue;
      h2d(r, h->mask, mask, (size_t)r->S);
      launch_project_cols(r->N, r->nvel, r->S, 1.0 / std::sqrt((double)h->H.back().npres), h->mask, h->bb,
                          h->partial, r->stream);
      enqueue_residual(r);
      enqueue_norms(r, h->r, h->small);
    }
    for (size_t a = 0; a < act.size(); ++a) {
      if (fresh[a].empty()) continue;
      Resident* r = act[a];
      std::vector<double> nrm(r->S);
      HIPCHECK(hipMemcpyAsync(nrm.data(), r->h->small, r->S * sizeof(double), hipMemcpyDeviceToHost, r->stream));
      HIPCHECK(hipStreamSynchronize(r->stream));
      std::vector<int> start;
      for (int c : fresh[a]) {
        Slot& sl = r->slots[c];
        sl.fresh = false;
        sl.bnorm = sl.beta = std::sqrt(nrm[c]);
        if (sl.bnorm == 0.0) {  // zero right-hand side: x = 0
          std::fill(sl.out, sl.out + r->N, 0.0);
          finish_ticket(s, sl.ticket, VK_OK, 0, 0.0);
          sl = Slot();
          continue;
        }
        sl.g.assign(m + 1, 0.0);
        sl.g[0] = sl.beta;
        sl.j = 0;
        start.push_back(c);
      }
      if (!start.empty()) enqueue_restart(r, start, 0);
    }
    // ---- phase B: one Arnoldi step for every running column
    const int pre = s->opts.nu_sweeps, post = s->opts.nu_sweeps;
    std::vector<Resident*> run;
    for (Resident* r : act) {
      bool any = false;
      for (const Slot& sl : r->slots) any = any || (sl.used && sl.j >= 0);
      if (!any) continue;
      enqueue_arnoldi(r, m, pre, post);
      run.push_back(r);
    }
    std::vector<std::vector<int>> ends(run.size());
    for (size_t a = 0; a < run.size(); ++a) {
      Resident* r = run[a];
      std::vector<double> hh((size_t)3 * (m + 2) * r->S);
      HIPCHECK(hipMemcpyAsync(hh.data(), r->h->small, hh.size() * sizeof(double), hipMemcpyDeviceToHost, r->stream));
      HIPCHECK(hipStreamSynchronize(r->stream));
      const int S = r->S;
      for (int c = 0; c < S; ++c) {
        Slot& sl = r->slots[c];
        if (!sl.used || sl.j < 0) continue;
        const int j = sl.j;
        double* H = sl.H.data();
        const double hn = std::sqrt(hh[(size_t)2 * (m + 2) * S + c]);
        require(std::isfinite(hn), VK_ENAN, "Arnoldi breakdown to a non-finite value");
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[(size_t)i * S + c] + hh[(size_t)(m + 2) * S + (size_t)i * S + c];
        H[(size_t)(j + 1) * m + j] = hn;
        for (int i = 0; i < j; ++i) {
          const double x0 = H[(size_t)i * m + j], x1 = H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = sl.cs[i] * x0 + sl.sn[i] * x1;
          H[(size_t)(i + 1) * m + j] = -sl.sn[i] * x0 + sl.cs[i] * x1;
        }
        const double x0 = H[(size_t)j * m + j], x1 = H[(size_t)(j + 1) * m + j];
        const double den = std::hypot(x0, x1);
        sl.cs[j] = x0 / den;
        sl.sn[j] = x1 / den;
        H[(size_t)j * m + j] = den;
        H[(size_t)(j + 1) * m + j] = 0.0;
        sl.g[j + 1] = -sl.sn[j] * sl.g[j];
        sl.g[j] = sl.cs[j] * sl.g[j];
        sl.its += 1;
        sl.j = j + 1;
        if (std::fabs(sl.g[j + 1]) <= s->opts.rtol * sl.bnorm || hn == 0.0 || sl.j == m || sl.its >= s->opts.maxit)
          ends[a].push_back(c);
      }
    }
    // ---- phase C: cycle ends: x += Z y, projection, true residual; retire or restart
    for (size_t a = 0; a < run.size(); ++a) {
      if (ends[a].empty()) continue;
      Resident* r = run[a];
      vk_hierarchy* h = r->h;
      const int S = r->S;
      double* y = hdp(r, HD_Y);
      int* nvc = hip_(r, HI_NVC_C);
      int* mask = hip_(r, HI_MASK_C);
      for (size_t i = 0; i < (size_t)(m + 2) * S; ++i) y[i] = 0.0;
      for (int c = 0; c < 64; ++c) {
        nvc[c] = 0;
        mask[c] = 0;
      }
      for (int c : ends[a]) {
        Slot& sl = r->slots[c];
        const int nk = sl.j;
        std::vector<double> yc(nk);
        for (int i = nk - 1; i >= 0; --i) {
          double acc = sl.g[i];
          for (int q = i + 1; q < nk; ++q) acc -= sl.H[(size_t)i * m + q] * yc[q];
          yc[i] = acc / sl.H[(size_t)i * m + i];
        }
        for (int i = 0; i < nk; ++i) y[(size_t)i * S + c] = yc[i];
        nvc[c] = nk;
        mask[c] = 1;
      }
      h2d(r, h->ydev, y, (size_t)(m + 2) * S);
      h2d(r, cip(r, CI_NVC), nvc, 64);
      h2d(r, h->mask, mask, (size_t)S);
      launch_axpy_cols(r->N, S, m, cip(r, CI_NVC), 1.0, h->Z, (int64_t)r->N * S, h->ydev, r->X, r->stream);
      launch_project_cols(r->N, r->nvel, S, 1.0 / std::sqrt((double)h->H.back().npres), h->mask, r->X, h->partial,
                          r->stream);
      enqueue_residual(r);
      enqueue_norms(r, h->r, h->small);
    }
    for (size_t a = 0; a < run.size(); ++a) {
      if (ends[a].empty()) continue;
      Resident* r = run[a];
      std::vector<double> nrm(r->S);
      HIPCHECK(hipMemcpyAsync(nrm.data(), r->h->small, r->S * sizeof(double), hipMemcpyDeviceToHost, r->stream));
      HIPCHECK(hipStreamSynchronize(r->stream));
      std::vector<int> restart;
      for (int c : ends[a]) {
        Slot& sl = r->slots[c];
        sl.beta = std::sqrt(nrm[c]);
        require(std::isfinite(sl.beta), VK_ENAN, "residual is not finite");
        const bool conv = sl.beta <= s->opts.rtol * sl.bnorm;
        if (conv || sl.its >= s->opts.maxit) {
          launch_column_get(r->N, r->S, c, r->X, r->stage, r->stream);
          HIPCHECK(hipMemcpyAsync(sl.out, r->stage, r->N * sizeof(double), hipMemcpyDeviceToHost, r->stream));
          HIPCHECK(hipStreamSynchronize(r->stream));
          finish_ticket(s, sl.ticket, conv ? VK_OK : VK_NOT_CONVERGED, sl.its, sl.beta / sl.bnorm);
          sl = Slot();
          continue;
        }
        std::fill(sl.H.begin(), sl.H.end(), 0.0);
        sl.g.assign(m + 1, 0.0);
        sl.g[0] = sl.beta;
        sl.j = 0;
        restart.push_back(c);
      }
      if (!restart.empty()) enqueue_restart(r, restart, 1);
      r->last_used = now_s();
    }
    for (Resident* r : act) HIPCHECK(hipStreamSynchronize(r->stream));
    int n_act = 0;
    for (auto& kv : s->res) n_act += kv.second->busy();
    if (active) *active = n_act + (int)s->queue.size();
    return VK_OK;
  });
}

vk_status vk_server_poll(vk_server* s, uint64_t ticket, vk_result* res) {
  return sguard([&]() -> vk_status {
    require(s && res, VK_EINVAL, "null argument");
    auto it = s->tickets.find(ticket);
    require(it != s->tickets.end(), VK_EINVAL, "unknown ticket");
    const Ticket& t = it->second;
    res->state = t.state;
    res->status = t.status;
    res->iterations = t.iterations;
    res->rel_residual = t.rel_residual;
    res->latency_s = t.state == 2 ? t.t_done - t.t_submit : 0.0;
    return VK_OK;
  });
}

vk_status vk_load_random(int k, int n, int n_modes, const double* coeffs, double* hb) {
  return sguard([&]() -> vk_status {
    require(coeffs && hb, VK_EINVAL, "null argument");
    require(k >= 2 && k <= 6 && n >= 1 && n <= 4096 / k, VK_EINVAL, "bad problem size");
    require(n_modes >= 1 && n_modes <= 64, VK_EINVAL, "n_modes out of range");
    assemble_random_load(VK_TH, k, n, n_modes, coeffs, hb);
    return VK_OK;
  });
}

vk_status vk_server_stats_get(vk_server* s, vk_server_stats* st) {
  return sguard([&]() -> vk_status {
    require(s && st, VK_EINVAL, "null argument");
    st->completed = s->completed;
    st->queued = (int)s->queue.size();
    int running = 0, resident = 0;
    size_t used = 0;
    for (auto& kv : s->res) {
      running += kv.second->busy();
      resident++;
      used += kv.second->bytes;
    }
    st->running = running;
    st->resident_hierarchies = resident;
    st->pool_bytes_used = used;
    st->evictions = s->evictions;
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      if (l.empty()) return 0.0;
      const double idx = p * (l.size() - 1);
      const size_t lo = (size_t)std::floor(idx), hi = (size_t)std::ceil(idx);
      return l[lo] + (l[hi] - l[lo]) * (idx - lo);
    };
    st->p50_latency_s = pct(0.50);
    st->p99_latency_s = pct(0.99);
    st->solves_per_s = (s->completed > 0 && s->t_last > s->t_first) ? s->completed / (s->t_last - s->t_first) : 0.0;
    return VK_OK;
  });
}

}  // extern "C"
