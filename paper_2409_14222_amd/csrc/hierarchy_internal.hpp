// Internal state of a bound hierarchy, shared by the solver (hierarchy.cpp)
// and the serving loop (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "vk_internal.hpp"

#define HIPCHECK(expr)                                                                                   \
  do {                                                                                                   \
    hipError_t _e = (expr);                                                                              \
    if (_e != hipSuccess) throw vk::Error(VK_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));       \
  } while (0)

namespace vk {

// patch size classes of the setup (one inversion kernel each): n <= 32, 64, 128, 224, 512, 768
constexpr int kClasses = 6;
constexpr int kClassLimit[kClasses] = {32, 64, 128, 224, 512, 768};
// patches above 224 DoFs: inverted in global scratch slots (at most this many at once), stored
// column-major (the symmetric tiled storage is limited to 224)
constexpr int kBigSlots = 256;
constexpr int kTiledMaxN = 224;
// the autotuner tries 8 and 16 waves per patch only on launches of at most this many patches
constexpr int kWideApplyMaxPatches = 4096;
// many-RHS K products run over union groups (FP64 matrix cores) above this many right-hand sides,
// and over runs of identical rows up to it (both give the same bits)
constexpr int kUnionMinRhs = 8;
// MI355X's last-level (Infinity) cache: many-RHS K products that move more bytes than this in
// one launch stream their single-use operands past the caches
constexpr double kLastLevelCacheBytes = 256.0 * (1 << 20);
// the fixed per-device scratch of the allocation-free smoothing call (vk_smooth_noalloc)
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
// its address on `device` (looked up once per device with that device current)
void* noalloc_scratch(int device);

struct DevLevel {
  int N = 0, nvel = 0, J = 0;
  double mean_row = 0, p_mean = 0, pt_mean = 0;
  int *rowptr = nullptr, *col = nullptr;
  double* val = nullptr;
  int *kgrp = nullptr, *pgrp = nullptr, *ptgrp = nullptr;  // row runs with identical patterns (K, P, P^T)
  int nkg = 0, npg = 0, nptg = 0;
  int kg_max = 8, pg_max = 8, ptg_max = 8;  // the longest run of each
  // K in union groups (bound for more than kUnionMinRhs right-hand sides, levels >= 1; nug = 0 otherwise)
  int nug = 0;
  int *ug_ptr = nullptr, *ug_row = nullptr, *ug_uptr = nullptr, *ug_col = nullptr;
  int64_t* ug_voff = nullptr;
  double* ug_val = nullptr;
  int64_t ug_nval = 0;
  int *prow = nullptr, *pcol = nullptr, *ptrow = nullptr, *ptcol = nullptr;
  double *pval = nullptr, *ptval = nullptr;
  int *pptr = nullptr, *pdofs = nullptr, *dptr = nullptr, *dslot = nullptr, *order = nullptr, *classes = nullptr;
  int64_t* inv_off = nullptr;
  double* scale = nullptr;
  void* inv = nullptr;
  void* delta = nullptr;
  double *b = nullptr, *x = nullptr, *t = nullptr;
  double* cd = nullptr;  // Chebyshev direction ([N][R], levels >= 1)
  double cheb_lambda = 0.0, cheb_theta = 0.0, cheb_delta = 0.0;  // estimate and interval centre / half-width
  int cheb_steps = 0;
  double* M = nullptr;  // coarsest level
  int class_count[kClasses] = {0, 0, 0, 0, 0, 0};  // patches per size class of kClassLimit (ids in `classes`)
  // launch shapes (never change results): lanes per CSR row of K, P, P^T;
  // waves per patch for the large (n > 64, first in `order`) and small patches
  int k_lanes = 32, p_lanes = 8, pt_lanes = 8, waves_large = 1, waves_small = 1, n_large = 0;
  int nt_large = 1, nt_small = 1;  // non-temporal (streaming) loads of the inverses
  int depth_large = 2, depth_small = 2;  // tile steps in flight (symmetric tiled storage)
  int merged = 0;  // one apply launch over all patches with the large patches' shape
  int max_n = 0;
  int4* meta = nullptr;            // per patch in processing order: {first slot, n, inverse offset}
  bool tri = false;                // inverses in symmetric tiled storage (bound for one right-hand side)
};

// Sequential carving of one caller buffer into 256-byte aligned pieces.  Run
// once with base == nullptr to size the workspace.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) / 256 * 256;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace vk

struct vk_hierarchy {
  using DevLevel = vk::DevLevel;
  using Problem = vk::Problem;
  using LevelHost = vk::LevelHost;
  Problem pr;
  vk_patch_opts opts{};
  std::vector<LevelHost> H;
  std::vector<double> coarse_M;
  std::vector<std::vector<int>> class_lists;  // per level: ids of class 0, then 1, then 2
  bool bound = false, ready = false;
  hipStream_t stream = nullptr;
  int device = -1;  // current device at bind (where the workspace lives)
  int max_restart = 0;
  int max_rhs = 1;
  int *nvc = nullptr, *mask = nullptr;  // per-column iteration counts / active flags (multi-RHS)
  std::vector<DevLevel> D;
  double *V = nullptr, *Z = nullptr, *bb = nullptr, *r = nullptr, *partial = nullptr, *small = nullptr, *ydev = nullptr;
  double* big_scratch = nullptr;  // kBigSlots-limited slots for the inversion of patches above 224 DoFs
  int big_slots = 0;
  int64_t big_slot_elems = 0;
  int* singular = nullptr;
  std::vector<double> ybuf;
  std::vector<std::vector<int4>> meta_host;  // staging of the per-patch metadata uploads
  // captured FGMRES iterations, keyed by (j, restart, nu_pre, nu_post, right-hand sides; 0 for the
  // single-vector step)
  std::map<std::tuple<int, int, int, int, int>, hipGraphExec_t> graphs;
  bool capturing = false;
  // kernel timing of the finest-level patch apply
  bool timing = false;
  int64_t t_launches = 0;
  double t_ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free, ev_pending;
  // timing of whole finest-level smoothing sweeps (residual, patch apply, scatter)
  bool sweep_timing = false;
  int64_t s_sweeps = 0;
  double s_ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> sw_pending;
  // pinned read-back of the Hessenberg columns (two slots) and their copy-done events, so that
  // the next Arnoldi step can be enqueued before the host has read the current one
  double* hh_pin = nullptr;
  size_t hh_pin_elems = 0;
  hipEvent_t ev_copy[2] = {nullptr, nullptr};

  bool fp32() const { return opts.store == VK_STORE_FP32; }
  bool cheb() const { return opts.smoother == VK_SMOOTH_CHEBYSHEV; }
  int L() const { return (int)H.size(); }
};


namespace vk {
void check_launch();
// Y = K X (mode 0), B - K X (1), Y += K X (2) on level d, [N][R] multivectors: over the union
// groups for more than kUnionMinRhs right-hand sides, else over the runs of identical rows
void spmm_k(const DevLevel& d, int mode, int R, const double* X, const double* B, double* Y, hipStream_t s);
void vcycle_multi(vk_hierarchy* h, int l, int R, const double* Rv, double* E, int nu_pre, int nu_post);
}  // namespace vk
