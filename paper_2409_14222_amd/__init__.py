"""Python binding of libvk.so: the MI355X matrix-full additive Vanka multigrid
Stokes solver (monolithic h-multigrid preconditioned FGMRES for Taylor-Hood).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch is used for device memory (one workspace tensor per hierarchy, plus the
caller's vectors) and for the HIP stream.  Importing fails loudly if the
library has not been built (python paper_2409_14222_amd/build.py).
"""
import ctypes
import os

import numpy as np

# torch first: it brings the HIP runtime that owns the device memory and the
# streams; libvk then binds to that same runtime (one runtime per process).
import torch  # noqa: F401  (import order matters)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libvk.so")
if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build it with `python {_HERE}/build.py`")
lib = ctypes.CDLL(LIBPATH)

# ---------------------------------------------------------------- constants (include/vk.h)
VK_OK, VK_NOT_CONVERGED = 0, 1
VK_EINVAL, VK_ENOMEM, VK_EHIP, VK_ESINGULAR, VK_ENAN, VK_EBUSY, VK_ESTATE = -1, -2, -3, -4, -5, -6, -7
VK_TH, VK_SV, VK_TH_QUAD, VK_BDM = 0, 1, 2, 3
VK_F_BASELINE_MMS, VK_F_PAPER_MMS, VK_F_RANDOM, VK_F_CUBE_MMS = 0, 1, 2, 3
VK_PATCH_COMPOSITE, VK_PATCH_STAR, VK_PATCH_MACRO, VK_PATCH_EXTENDED = 0, 1, 2, 3
VK_STORE_FP64, VK_STORE_FP32 = 0, 1
VK_SMOOTH_DAMPED, VK_SMOOTH_CHEBYSHEV = 0, 1
VK_WEIGHT_MULTIPLICITY, VK_WEIGHT_NONE = 0, 1

_c_int, _c_dbl, _p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p


class vk_problem(ctypes.Structure):
    _fields_ = [("dim", _c_int), ("family", _c_int), ("k", _c_int), ("n_coarse", _c_int), ("n_levels", _c_int),
                ("viscosity", _c_dbl), ("forcing", _c_int), ("n_modes", _c_int),
                ("h_forcing_coeffs", ctypes.POINTER(_c_dbl)), ("penalty", _c_dbl)]


class vk_patch_opts(ctypes.Structure):
    _fields_ = [("construct", _c_int), ("store", _c_int), ("omega", _c_dbl), ("smoother", _c_int),
                ("weighting", _c_int), ("est_steps", _c_int), ("est_seed", ctypes.c_uint64)]


class vk_level_info(ctypes.Structure):
    _fields_ = [("n", _c_int), ("n_free", _c_int), ("n_velocity", _c_int), ("nnz", ctypes.c_int64),
                ("n_patches", _c_int), ("sum_n", ctypes.c_int64), ("sum_n2", ctypes.c_int64), ("max_n", _c_int),
                ("p_nnz", ctypes.c_int64), ("inv_elems_full", ctypes.c_int64), ("inv_elems_tri", ctypes.c_int64),
                ("cheb_lambda", _c_dbl), ("cheb_steps", _c_int)]


class vk_tuning(ctypes.Structure):
    _fields_ = [("k_lanes", _c_int), ("p_lanes", _c_int), ("pt_lanes", _c_int), ("apply_waves_large", _c_int),
                ("apply_waves_small", _c_int), ("apply_nontemporal_large", _c_int),
                ("apply_nontemporal_small", _c_int), ("apply_depth_large", _c_int), ("apply_depth_small", _c_int),
                ("apply_merged", _c_int)]


class vk_solve_opts(ctypes.Structure):
    _fields_ = [("restart", _c_int), ("maxit", _c_int), ("rtol", _c_dbl), ("nu_pre", _c_int), ("nu_post", _c_int),
                ("use_graphs", _c_int)]


class vk_solve_info(ctypes.Structure):
    _fields_ = [("iterations", _c_int), ("converged", _c_int), ("rel_residual", _c_dbl),
                ("h_history", ctypes.POINTER(_c_dbl))]


class vk_server_opts(ctypes.Structure):
    _fields_ = [("slots", _c_int), ("store", _c_int), ("omega", _c_dbl), ("nu_sweeps", _c_int), ("restart", _c_int),
                ("maxit", _c_int), ("rtol", _c_dbl), ("max_queue", _c_int)]


class vk_request(ctypes.Structure):
    _fields_ = [("n", _c_int), ("k", _c_int), ("viscosity", _c_dbl), ("h_b", _p)]


class vk_result(ctypes.Structure):
    _fields_ = [("state", _c_int), ("status", _c_int), ("iterations", _c_int), ("rel_residual", _c_dbl),
                ("latency_s", _c_dbl)]


class vk_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("queued", _c_int), ("running", _c_int),
                ("resident_hierarchies", _c_int), ("pool_bytes_used", ctypes.c_size_t), ("evictions", ctypes.c_int64),
                ("p50_latency_s", _c_dbl), ("p99_latency_s", _c_dbl), ("solves_per_s", _c_dbl)]


_P = ctypes.POINTER
_SIGS = {
    "vk_last_error": ([], ctypes.c_char_p),
    "vk_hierarchy_create": ([_P(vk_problem), _P(vk_patch_opts), _P(_p)], _c_int),
    "vk_hierarchy_destroy": ([_p], _c_int),
    "vk_hierarchy_workspace_bytes": ([_p, _c_int, _c_int, _P(ctypes.c_size_t)], _c_int),
    "vk_hierarchy_bind": ([_p, _p, ctypes.c_size_t, _c_int, _c_int, _p], _c_int),
    "vk_patches_setup": ([_p], _c_int),
    "vk_level_info_get": ([_p, _c_int, _P(vk_level_info)], _c_int),
    "vk_level_csr": ([_p, _c_int, _p, _p, _p], _c_int),
    "vk_level_prolongation": ([_p, _c_int, _p, _p, _p], _c_int),
    "vk_level_patches": ([_p, _c_int, _p, _p], _c_int),
    "vk_level_union_groups": ([_p, _c_int, _p, _p, _p, _p, _p, _p, _p], _c_int),
    "vk_dof_coords": ([_p, _c_int, _p, _p], _c_int),
    "vk_rhs": ([_p, _p], _c_int),
    "vk_patch_gather": ([_p, _c_int, _c_int, _c_int, _p], _c_int),
    "vk_patch_inverse": ([_p, _c_int, _c_int, _p], _c_int),
    "vk_spmv": ([_p, _c_int, _p, _p], _c_int),
    "vk_spmv_multi": ([_p, _c_int, _p, _p, _c_int], _c_int),
    "vk_restrict": ([_p, _c_int, _p, _p], _c_int),
    "vk_prolong_add": ([_p, _c_int, _p, _p], _c_int),
    "vk_smooth": ([_p, _c_int, _p, _p, _c_int], _c_int),
    "vk_smooth_noalloc": ([_p, _c_int, _p, _p, _c_int], _c_int),
    "vk_coarse_solve": ([_p, _p, _p], _c_int),
    "vk_vcycle": ([_p, _p, _p, _c_int, _c_int], _c_int),
    "vk_solve": ([_p, _p, _p, _P(vk_solve_opts), _P(vk_solve_info)], _c_int),
    "vk_smooth_multi": ([_p, _c_int, _p, _p, _c_int, _c_int], _c_int),
    "vk_vcycle_multi": ([_p, _p, _p, _c_int, _c_int, _c_int], _c_int),
    "vk_solve_multi": ([_p, _p, _p, _c_int, _P(vk_solve_opts), _p], _c_int),
    "vk_rhs_random": ([_p, _c_int, _p, _p], _c_int),
    "vk_autotune": ([_p, _c_int], _c_int),
    "vk_autotune_cached": ([_p, _c_int, ctypes.c_char_p, _P(_c_int)], _c_int),
    "vk_tuning_get": ([_p, _c_int, _P(vk_tuning)], _c_int),
    "vk_tuning_set": ([_p, _c_int, _P(vk_tuning)], _c_int),
    "vk_kernel_timing": ([_p, _c_int, _c_int, _P(ctypes.c_int64), _P(_c_dbl)], _c_int),
    "vk_sweep_timing": ([_p, _c_int, _c_int, _P(ctypes.c_int64), _P(_c_dbl)], _c_int),
    "vk_server_last_error": ([], ctypes.c_char_p),
    "vk_server_create": ([_P(vk_server_opts), _p, ctypes.c_size_t, _P(_p), ctypes.c_int, _P(_p)], _c_int),
    "vk_server_destroy": ([_p], _c_int),
    "vk_server_prepare": ([_p, _c_int, _c_int], _c_int),
    "vk_server_problem_size": ([_p, _c_int, _c_int, _P(_c_int)], _c_int),
    "vk_server_submit": ([_p, _P(vk_request), _p, _P(ctypes.c_uint64)], _c_int),
    "vk_server_tick": ([_p, _P(_c_int)], _c_int),
    "vk_server_poll": ([_p, ctypes.c_uint64, _P(vk_result)], _c_int),
    "vk_server_stats_get": ([_p, _P(vk_server_stats)], _c_int),
    "vk_load_random": ([_c_int, _c_int, _c_int, _p, _p], _c_int),
    "vk_hessenberg_eigenvalues": ([_c_int, _p, _p, _p], _c_int),
    "vk_coarse_inverse": ([_p, _p], _c_int),
    "vk_solution_errors": ([_p, _p, _p], _c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res
EXPORTS = tuple(_SIGS)


class VkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vk status {code}: {msg}")
        self.code = code


def check(status):
    if status < 0:
        raise VkError(status, lib.vk_last_error().decode())
    return status


def _ptr(a):
    """Address of a numpy array or a torch tensor (device pointer for CUDA tensors)."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def hessenberg_eigenvalues(H):
    """Eigenvalues of an upper Hessenberg matrix by the library's QR iteration (host)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    n = H.shape[0]
    re = np.empty(n); im = np.empty(n)
    check(lib.vk_hessenberg_eigenvalues(n, _ptr(H), _ptr(re), _ptr(im)))
    return re + 1j * im


class Hierarchy:
    """One Stokes problem hierarchy.  Host-side data is available right after
    construction; device work needs bind() (allocates the workspace with torch
    on the current device and binds the current stream) and setup()."""

    def __init__(self, k, n_coarse, n_levels, dim=2, viscosity=1.0, forcing=VK_F_BASELINE_MMS, coeffs=None,
                 construct=None, store=VK_STORE_FP64, omega=0.5, family=VK_TH, smoother=VK_SMOOTH_DAMPED,
                 weighting=VK_WEIGHT_MULTIPLICITY, est_steps=10, est_seed=0, penalty=0.0):
        if construct is None:
            construct = {VK_SV: VK_PATCH_MACRO, VK_BDM: VK_PATCH_EXTENDED}.get(family, VK_PATCH_COMPOSITE)
        self._coeffs = None
        n_modes = 0
        cptr = None
        if coeffs is not None:
            self._coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
            n_modes = self._coeffs.shape[-1]
            cptr = self._coeffs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.prob = vk_problem(dim, family, k, n_coarse, n_levels, viscosity, forcing, n_modes, cptr, penalty)
        self.opts = vk_patch_opts(construct, store, omega, smoother, weighting, est_steps, est_seed)
        h = ctypes.c_void_p()
        check(lib.vk_hierarchy_create(ctypes.byref(self.prob), ctypes.byref(self.opts), ctypes.byref(h)))
        self.h = h
        self.n_levels = n_levels
        self.dim = dim
        self.ws = None
        self.stream = None

    def __del__(self, _destroy=lib.vk_hierarchy_destroy):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _destroy(h)
            self.h = None

    # ------------------------------------------------------------ host data
    def level_info(self, level):
        info = vk_level_info()
        check(lib.vk_level_info_get(self.h, level, ctypes.byref(info)))
        return info

    def csr(self, level):
        inf = self.level_info(level)
        rp = np.empty(inf.n_free + 1, np.int32); col = np.empty(inf.nnz, np.int32); val = np.empty(inf.nnz)
        check(lib.vk_level_csr(self.h, level, _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col, val

    def union_groups(self, level):
        """K's union groups on `level` (host copies): gptr, grow, uptr, ucol, voff, val."""
        sizes = np.zeros(4, np.int64)
        check(lib.vk_level_union_groups(self.h, level, _ptr(sizes), None, None, None, None, None, None))
        ng, nr, nc, nv = (int(x) for x in sizes)
        gptr = np.empty(ng + 1, np.int32); grow = np.empty(nr, np.int32); uptr = np.empty(ng + 1, np.int32)
        ucol = np.empty(nc, np.int32); voff = np.empty(ng, np.int64); val = np.empty(nv)
        check(lib.vk_level_union_groups(self.h, level, _ptr(sizes), _ptr(gptr), _ptr(grow), _ptr(uptr), _ptr(ucol),
                                        _ptr(voff), _ptr(val)))
        return gptr, grow, uptr, ucol, voff, val

    def prolongation(self, level):
        inf = self.level_info(level)
        rp = np.empty(inf.n_free + 1, np.int32); col = np.empty(inf.p_nnz, np.int32); val = np.empty(inf.p_nnz)
        check(lib.vk_level_prolongation(self.h, level, _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col, val

    def patches(self, level):
        inf = self.level_info(level)
        ptr = np.empty(inf.n_patches + 1, np.int32); dofs = np.empty(inf.sum_n, np.int32)
        check(lib.vk_level_patches(self.h, level, _ptr(ptr), _ptr(dofs)))
        return ptr, dofs

    def solution_errors(self, x):
        """(relative H^1 velocity error, mean-free L^2 pressure error) of a finest-level solution (host array)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        err = np.empty(2)
        check(lib.vk_solution_errors(self.h, _ptr(x), _ptr(err)))
        return float(err[0]), float(err[1])

    def coarse_inverse(self):
        n = self.level_info(0).n_free
        out = np.empty((n, n))
        check(lib.vk_coarse_inverse(self.h, _ptr(out)))
        return out

    def dof_coords(self, level):
        inf = self.level_info(level)
        X = np.empty((inf.n_free, self.dim)); kind = np.empty(inf.n_free, np.int32)
        check(lib.vk_dof_coords(self.h, level, _ptr(X), _ptr(kind)))
        return X, kind

    def rhs(self):
        b = np.empty(self.level_info(self.n_levels - 1).n_free)
        check(lib.vk_rhs(self.h, _ptr(b)))
        return b

    # ------------------------------------------------------------ device
    def workspace_bytes(self, max_restart=30, max_rhs=1):
        nb = ctypes.c_size_t()
        check(lib.vk_hierarchy_workspace_bytes(self.h, max_restart, max_rhs, ctypes.byref(nb)))
        return nb.value

    def bind(self, max_restart=30, device="cuda", max_rhs=1):
        import torch
        nbytes = self.workspace_bytes(max_restart, max_rhs)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.ws.device)
        check(lib.vk_hierarchy_bind(self.h, aligned, nbytes + 256 - (aligned - base), max_restart, max_rhs,
                                    self.stream.cuda_stream))
        self.max_restart = max_restart
        self.max_rhs = max_rhs
        return self

    def setup(self):
        check(lib.vk_patches_setup(self.h))
        return self

    def patch_gather(self, level, first, count, out):
        check(lib.vk_patch_gather(self.h, level, first, count, _ptr(out)))

    def patch_inverse(self, level, patch, out):
        check(lib.vk_patch_inverse(self.h, level, patch, _ptr(out)))

    def spmv(self, level, x, y):
        check(lib.vk_spmv(self.h, level, _ptr(x), _ptr(y)))

    def spmv_multi(self, level, X, Y, nrhs):
        check(lib.vk_spmv_multi(self.h, level, _ptr(X), _ptr(Y), nrhs))

    def restrict(self, level, rf, rc):
        check(lib.vk_restrict(self.h, level, _ptr(rf), _ptr(rc)))

    def prolong_add(self, level, ec, ef):
        check(lib.vk_prolong_add(self.h, level, _ptr(ec), _ptr(ef)))

    def smooth(self, level, b, x, nsweeps):
        check(lib.vk_smooth(self.h, level, _ptr(b), _ptr(x), nsweeps))

    def smooth_noalloc(self, level, b, x, nsweeps):
        """vk_smooth with the sweep scratch in the library's fixed per-device array (allocates nothing)."""
        check(lib.vk_smooth_noalloc(self.h, level, _ptr(b), _ptr(x), nsweeps))

    def coarse_solve(self, r, e):
        check(lib.vk_coarse_solve(self.h, _ptr(r), _ptr(e)))

    def vcycle(self, r, e, nu_pre=2, nu_post=2):
        check(lib.vk_vcycle(self.h, _ptr(r), _ptr(e), nu_pre, nu_post))

    def solve(self, b, x, restart=30, maxit=100, rtol=1e-10, nu_pre=2, nu_post=2, history=False, graphs=False):
        opts = vk_solve_opts(restart, maxit, rtol, nu_pre, nu_post, int(graphs))
        hist = np.zeros(maxit + 1) if history else None
        info = vk_solve_info(0, 0, 0.0, hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if history else None)
        status = check(lib.vk_solve(self.h, _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(info)))
        out = {"status": status, "iterations": info.iterations, "converged": bool(info.converged),
               "rel_residual": info.rel_residual}
        if history:
            out["history"] = hist[: info.iterations + 1].copy()
        return out

    def rhs_random(self, coeffs):
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        b = np.empty(self.level_info(self.n_levels - 1).n_free)
        check(lib.vk_rhs_random(self.h, coeffs.shape[-1], _ptr(coeffs), _ptr(b)))
        return b

    def smooth_multi(self, level, B, X, nrhs, nsweeps):
        check(lib.vk_smooth_multi(self.h, level, _ptr(B), _ptr(X), nrhs, nsweeps))

    def vcycle_multi(self, R, E, nrhs, nu_pre=2, nu_post=2):
        check(lib.vk_vcycle_multi(self.h, _ptr(R), _ptr(E), nrhs, nu_pre, nu_post))

    def solve_multi(self, B, X, nrhs, restart=30, maxit=100, rtol=1e-10, nu_pre=2, nu_post=2, graphs=False):
        """B, X: row-major [N][nrhs] device tensors.  Returns one result dict per column."""
        opts = vk_solve_opts(restart, maxit, rtol, nu_pre, nu_post, int(graphs))
        infos = (vk_solve_info * nrhs)()
        status = check(lib.vk_solve_multi(self.h, _ptr(B), _ptr(X), nrhs, ctypes.byref(opts), infos))
        return status, [{"iterations": i.iterations, "converged": bool(i.converged), "rel_residual": i.rel_residual}
                        for i in infos]

    def autotune(self, reps=5, cache=None):
        """Autotune the launch shapes; with `cache` (a file path) reuse the shapes stored there for
        this hierarchy and device, or store the new ones.  Returns the per-level shapes."""
        if cache is None:
            check(lib.vk_autotune(self.h, reps))
        else:
            hit = ctypes.c_int()
            check(lib.vk_autotune_cached(self.h, reps, os.fsencode(cache), ctypes.byref(hit)))
            self.tuning_cache_hit = bool(hit.value)
        return [self.tuning(l) for l in range(self.n_levels)]

    def tuning(self, level):
        t = vk_tuning()
        check(lib.vk_tuning_get(self.h, level, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in vk_tuning._fields_}

    def set_tuning(self, level, **kw):
        cur = self.tuning(level)
        cur.update(kw)
        t = vk_tuning(**cur)
        check(lib.vk_tuning_set(self.h, level, ctypes.byref(t)))

    def kernel_timing(self, enable=True, reset=False):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        check(lib.vk_kernel_timing(self.h, int(enable), int(reset), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def sweep_timing(self, enable=True, reset=False):
        """(finest-level sweeps, their total milliseconds) since the last reset."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        check(lib.vk_sweep_timing(self.h, int(enable), int(reset), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


def scheck(status):
    if status < 0:
        raise VkError(status, lib.vk_server_last_error().decode())
    return status


def load_random(k, n, coeffs):
    """Load vector of the smooth random forcing for the 2D (n, k) problem (host)."""
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    N = 2 * (k * n - 1) ** 2 + ((k - 1) * n + 1) ** 2
    b = np.empty(N)
    scheck(lib.vk_load_random(k, n, coeffs.shape[-1], _ptr(coeffs), _ptr(b)))
    return b


class Server:
    """Continuous-batching Stokes server on one GPU (see vk.h).  The device
    pool is one torch tensor; results land in host numpy arrays."""

    def __init__(self, pool_bytes, slots=16, store=VK_STORE_FP32, omega=0.5, nu_sweeps=2, restart=30, maxit=100,
                 rtol=1e-10, max_queue=100000, device="cuda", streams=4):
        import torch
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=device)
        base = self.pool.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.opts = vk_server_opts(slots, store, omega, nu_sweeps, restart, maxit, rtol, max_queue)
        # torch owns the streams the resident hierarchies run on (default priority)
        self.streams = [torch.cuda.Stream(device=self.pool.device) for _ in range(int(streams))]
        handles = (ctypes.c_void_p * len(self.streams))(*[st.cuda_stream for st in self.streams])
        s = ctypes.c_void_p()
        scheck(lib.vk_server_create(ctypes.byref(self.opts), aligned, int(pool_bytes), handles, len(self.streams),
                                    ctypes.byref(s)))
        self.s = s
        self._keep = {}

    def close(self):
        if getattr(self, "s", None) is not None and self.s.value:
            lib.vk_server_destroy(self.s)
            self.s = None

    def __del__(self, _destroy=lib.vk_server_destroy):
        s = getattr(self, "s", None)
        if s is not None and s.value:
            _destroy(s)
            self.s = None

    def prepare(self, n, k):
        scheck(lib.vk_server_prepare(self.s, n, k))

    def size(self, n, k):
        v = ctypes.c_int()
        scheck(lib.vk_server_problem_size(self.s, n, k, ctypes.byref(v)))
        return v.value

    def submit(self, n, k, viscosity, b):
        """Returns (status, ticket, x): x is filled when the request completes."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        N = self.size(n, k)
        if b.shape != (N,):
            raise ValueError(f"right-hand side of the ({n}, {k}) problem must have {N} entries, got {b.shape}")
        x = np.zeros(N)
        req = vk_request(n, k, viscosity, b.ctypes.data)
        t = ctypes.c_uint64()
        st = lib.vk_server_submit(self.s, ctypes.byref(req), _ptr(x), ctypes.byref(t))
        if st == VK_EBUSY:  # queue full: the caller retries later
            return st, 0, None
        scheck(st)
        if st == VK_OK:
            self._keep[t.value] = x
        return st, t.value, x

    def tick(self):
        a = ctypes.c_int()
        scheck(lib.vk_server_tick(self.s, ctypes.byref(a)))
        return a.value

    def poll(self, ticket):
        r = vk_result()
        scheck(lib.vk_server_poll(self.s, ticket, ctypes.byref(r)))
        return {"state": r.state, "status": r.status, "iterations": r.iterations, "rel_residual": r.rel_residual,
                "latency_s": r.latency_s}

    def stats(self):
        st = vk_server_stats()
        scheck(lib.vk_server_stats_get(self.s, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in vk_server_stats._fields_}
