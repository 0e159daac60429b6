"""Benchmark: Stokes solves per second to 1e-10 relative residual.

Workload (default): P4-P3 Taylor-Hood on the unit square, 64x64 squares each
cut into two triangles, 5-level hierarchy (4x4 .. 64x64), composite Vanka
patches, V(2,2) cycles with damping 0.5, FGMRES(30) to 1e-10, plain FP64.
One step = one full solve (hierarchy resident, patches factored); the
right-hand side is resident in HBM before the timed region.

Prints one JSON line with the throughput, per-solve latency percentiles, the
roofline of the dominant kernel (finest-level patch apply, timed with HIP
events around every launch inside the timed region), the Vanka DoF-sweep rate
(finest-level sweeps timed with events in three further solves) and a CPU
baseline: one full oracle solve of the same workload after its setup, at one
thread and at the host's thread count.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "p4p3-64": dict(k=4, n0=4, levels=5, desc="P4-P3 Taylor-Hood, 64x64 two-triangle mesh of the unit square, "
                                           "5-level hierarchy, composite Vanka, V(2,2), omega 0.5, FGMRES(30) to 1e-10"),
    "p2p1-16": dict(k=2, n0=4, levels=3, desc="P2-P1 Taylor-Hood, 16x16 two-triangle mesh of the unit square, "
                                           "3-level hierarchy, vertex Vanka, V(2,2), omega 0.5, FGMRES(30) to 1e-10"),
    "p2p1-3d-16": dict(k=2, n0=4, levels=3, dim=3,
                       desc="3D P2-P1 Taylor-Hood, 16^3 cubes each split into 6 Kuhn tetrahedra, 3-level hierarchy "
                            "(4^3, 8^3, 16^3), vertex Vanka (up to 196 DoFs), V(2,2), omega 0.5, FGMRES(30) to 1e-10"),
    "sv-p3dp2-64": dict(k=3, n0=4, levels=5, family="sv", nrhs=64, store="fp32",
                        desc="Scott-Vogelius P3-dP2 on the barycentric refinement of the 64x64 two-triangle mesh, "
                             "5 non-nested levels (4..64), macro-element Vanka (56 DoFs), 64 random smooth forcings "
                             "solved in lockstep, FP32 matrix-core patch GEMMs, V(2,2), omega 0.5, FGMRES(30) to 1e-10"),
    "bdm4-80": dict(k=4, n0=5, levels=5, family="bdm",
                    desc="BDM4-dP3 with symmetric interior penalty (alpha 2 (k+1)^2), 80x80 two-triangle mesh, "
                         "5x5 coarsest mesh and 4 refinements (the paper's l = 4), extended cell Vanka (up to 115 "
                         "DoFs), the paper's manufactured solution, V(2,2), omega 0.5, FGMRES(30) to 1e-10"),
}
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel measured with rocprofv3
# FETCH_SIZE/WRITE_SIZE (scaled by a plain-copy calibration), keyed by the
# source file of that kernel (its hash) and the workload; any change to that
# file invalidates them (reported as null).
# Sources: profiles/patch_apply_p4p3_64_fp64.md, profiles/many_rhs_sv_p3dp2_64.md,
# profiles/patch_apply_bdm4_80_fp64.md, profiles/patch_apply_p2p1_3d_16_fp64.md
MEASURED_TRAFFIC = {
    ("patch_apply.hip", "5deac05388636b60", "p4p3-64", "fp64", 1): 487.8e6,
    ("patch_apply.hip", "5deac05388636b60", "bdm4-80", "fp64", 1): 764.8e6,
    ("patch_apply.hip", "5deac05388636b60", "p2p1-3d-16", "fp64", 1): 533.5e6,
    ("patch_gemm.hip", "010fc9744420da47", "sv-p3dp2-64", "fp32", 64): 456.6e6,
}


def kernel_source_hash(name):
    import hashlib
    path = os.path.join(ROOT, "paper_2409_14222_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sample(spec):
    """The oracle, as it stands, on the benchmarked workload (run in a child process): setup (assembly,
    patch extraction and LU factorisation) timed on one thread, then one full FGMRES solve of the same
    right-hand side at one thread and at the host's thread count (BLAS/OpenMP pools limited with
    threadpoolctl).  No extrapolation: each figure is one measured solve."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import fields, solve
    workload, smoother, weighting = spec.split(":")
    w = WORKLOADS[workload]
    dim = w.get("dim", 2)
    kw = dict(smoother=smoother, weighting=weighting)
    nproc = len(os.sched_getaffinity(0))
    threads = min(nproc, int(os.environ.get("OMP_NUM_THREADS", nproc)))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        if w.get("family") == "sv":
            g = synth.forcing_coeffs(synth.SEED)
            H, V = solve.setup(2, w["k"], w["n0"], w["levels"], 1.0, lambda nu: fields.random_sine_field(g, nu),
                               family="sv", **kw)
        elif w.get("family") == "bdm":
            H, V = solve.setup(2, w["k"], w["n0"], w["levels"], 1.0, fields.paper_mms, family="bdm", **kw)
        else:
            H, V = solve.setup(dim, w["k"], w["n0"], w["levels"], 1.0,
                               fields.cube_mms if dim == 3 else fields.baseline_mms, **kw)
        t_setup = time.perf_counter() - t0
    runs = []
    for nt in sorted({1, threads}):
        with threadpool_limits(nt):
            times = []
            while True:  # one solve of a large workload; short ones repeat (up to 50 or ~5 s), median
                t0 = time.perf_counter()
                x, its, _, conv = solve.solve(H, V)
                times.append(time.perf_counter() - t0)
                if len(times) >= 50 or sum(times) > 5.0 or times[0] > 2.0:
                    break
            dt = float(np.median(times))
        runs.append({"threads": nt, "solve_s": dt, "repeats": len(times), "iterations": its,
                     "converged": bool(conv), "solves_per_s": 1.0 / dt, "setup_plus_solve_per_s": 1.0 / (t_setup + dt)})
    best = max(runs, key=lambda r: r["solves_per_s"])
    return {"value": best["solves_per_s"], "unit": "solves/s", "cores": best["threads"], "kind": "oracle",
            "sample": f"full oracle FGMRES solves of the workload ({best['iterations']} iterations, "
                      f"{best['solve_s']:.2f} s, median of {best['repeats']}) after its setup ({t_setup:.1f} s on "
                      f"one thread); solves at 1 and {threads} threads",
            "setup_s": t_setup, "runs": runs, "nproc": nproc, "cpu_model": cpu_model()}


def serve_bench(args):
    """Serving workload: 512 requests, mesh n in {16, 32, 64, 128}, order k in {2, 3, 4} (uniform),
    log10(viscosity) ~ U[-2, 2], smooth random forcing (seed 20240922 + 1000 + id).  Run (i): all
    requests at t = 0 (throughput); run (ii): Poisson arrivals at 0.8 x the measured capacity
    (latency).  Hierarchies are prepared and right-hand sides assembled before the clock starts."""
    import numpy as np
    import torch

    import paper_2409_14222_amd as vk
    import synth
    rng = np.random.default_rng(synth.SEED)
    nreq = args.serve_requests
    ns = rng.choice([16, 32, 64, 128], nreq)
    ks = rng.choice([2, 3, 4], nreq)
    nus = 10.0 ** rng.uniform(-2.0, 2.0, nreq)
    gaps = rng.exponential(1.0, nreq)  # unit-rate inter-arrival times, scaled below
    store = vk.VK_STORE_FP32 if args.store == "fp32" else vk.VK_STORE_FP64
    t0 = time.perf_counter()
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=16) as ex:  # the library call releases the GIL
        rhs = list(ex.map(lambda a: vk.load_random(int(a[1]), int(a[0]), synth.forcing_coeffs(synth.SEED + 1000 + a[2])),
                          zip(ns, ks, range(nreq))))
    t_rhs = time.perf_counter() - t0

    def make_server():
        srv = vk.Server(args.serve_pool_gb * (1 << 30), slots=args.serve_slots, store=store)
        for n in (16, 32, 64, 128):
            for k in (2, 3, 4):
                srv.prepare(n, k)
        return srv

    def run(srv, arrival):
        torch.cuda.synchronize()
        start = time.perf_counter()
        handles = [None] * nreq
        nxt = 0
        while True:
            now = time.perf_counter() - start
            while nxt < nreq and arrival[nxt] <= now:
                handles[nxt] = srv.submit(int(ns[nxt]), int(ks[nxt]), float(nus[nxt]), rhs[nxt])
                nxt += 1
            active = srv.tick()
            if nxt == nreq and active == 0:
                break
            if active == 0 and nxt < nreq:
                time.sleep(max(0.0, min(arrival[nxt] - (time.perf_counter() - start), 0.01)))
        elapsed = time.perf_counter() - start
        res = [srv.poll(h[1]) for h in handles]
        lat = np.array([r["latency_s"] for r in res])
        ok = all(r["status"] == 0 and r["rel_residual"] <= 1e-10 for r in res)
        return elapsed, lat, ok, res

    t0 = time.perf_counter()
    srv = make_server()
    t_prep = time.perf_counter() - t0
    el, lat, ok, res = run(srv, np.zeros(nreq))
    cap = nreq / el
    arrival = np.cumsum(gaps) / (0.8 * cap)
    el2, lat2, ok2, _ = run(srv, arrival)
    st = srv.stats()
    out = {
        "metric": "Stokes solves/s to 1e-10 rel. residual (served, continuous batching)",
        "value": cap, "unit": "solves/s", "n_gpus": 1, "steps": nreq, "warmup": 0,
        "ms_per_step": 1e3 * el / nreq, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if store == vk.VK_STORE_FP64 else "f64 (patch inverses stored/applied in f32)",
        "data": "synthetic (seeded random smooth forcings, seeded Poisson arrivals)",
        "config": {"workload": f"{nreq} requests, n in {{16,32,64,128}}, k in {{2,3,4}}, nu log-uniform in "
                               f"[1e-2, 1e2], V(2,2), omega 0.5, FGMRES(30) to 1e-10",
                   "slots_per_hierarchy": args.serve_slots, "pool_gb": args.serve_pool_gb, "store": args.store},
        "all_at_once": {"solves_per_s": cap, "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)),
                        "p99_latency_ms": 1e3 * float(np.percentile(lat, 99)), "all_converged": ok,
                        "mean_iterations": float(np.mean([r["iterations"] for r in res]))},
        "poisson_0p8_capacity": {"rate_per_s": 0.8 * cap, "solves_per_s": nreq / el2,
                                 "p50_latency_ms": 1e3 * float(np.percentile(lat2, 50)),
                                 "p99_latency_ms": 1e3 * float(np.percentile(lat2, 99)), "all_converged": ok2},
        "resident_hierarchies": st["resident_hierarchies"], "pool_bytes_used": st["pool_bytes_used"],
        "setup_s": {"prepare_12_hierarchies": t_prep, "assemble_rhs": t_rhs},
    }
    print(json.dumps(out))


def paper_grid(args):
    """Iteration counts at the paper's experiment settings (Sec. 4): 5x5 coarsest mesh (cut from top
    left to bottom right; squares with --grid-family quad; BDM_k-dP_{k-1} with --grid-family bdm), the
    paper's manufactured solution, zero
    initial guess, unrestarted FGMRES (at most 100 iterations) to a 1e-10 relative residual, V(nu, nu) with nu = 1..4, l = 1..4 refinements; for
    each order k and smoother (damped additive Vanka, omega 0.5, 1/multiplicity weights; Chebyshev on
    [lambda / 4, 1.1 lambda] with unweighted or 1/multiplicity-weighted patch sums).  One JSON line per
    (k, l, smoother) with the iteration counts, the solve times and the per-level estimates."""
    import numpy as np
    import torch

    import paper_2409_14222_amd as vk
    torch.cuda.init()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    smoothers = [("damped", vk.VK_SMOOTH_DAMPED, vk.VK_WEIGHT_MULTIPLICITY),
                 ("chebyshev", vk.VK_SMOOTH_CHEBYSHEV, vk.VK_WEIGHT_NONE),
                 ("chebyshev-weighted", vk.VK_SMOOTH_CHEBYSHEV, vk.VK_WEIGHT_MULTIPLICITY)]
    keep = args.grid_smoothers.split(",")
    smoothers = [s for s in smoothers if s[0] in keep]
    fam = {"quad": vk.VK_TH_QUAD, "bdm": vk.VK_BDM}.get(args.grid_family, vk.VK_TH)
    for k in [int(v) for v in args.grid_k.split(",")]:
        for ell in [int(v) for v in args.grid_levels.split(",")]:
            for name, sm, wt in smoothers:
                t0 = time.perf_counter()
                H = vk.Hierarchy(k, 5, ell + 1, forcing=vk.VK_F_PAPER_MMS, smoother=sm, weighting=wt, family=fam)
                H.bind(max_restart=100).setup()
                t_setup = time.perf_counter() - t0
                b = torch.tensor(H.rhs(), device="cuda")
                x = torch.empty_like(b)
                its, ms, est = {}, {}, {}
                for nu in (1, 2, 3, 4):
                    H.solve(b, x, restart=100, maxit=100, nu_pre=nu, nu_post=nu)  # warm-up
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    r = H.solve(b, x, restart=100, maxit=100, nu_pre=nu, nu_post=nu, history=True)
                    torch.cuda.synchronize()
                    ms[nu] = 1e3 * (time.perf_counter() - t1)
                    its[nu] = r["iterations"] if r["converged"] else None
                    # the first iteration whose FGMRES residual estimate reaches 1e-10 (the quantity a
                    # solver that stops on the estimate counts; the library also checks the true residual)
                    h = r["history"]
                    hit = [j for j in range(len(h)) if h[j] <= 1e-10 * h[0]]
                    est[nu] = hit[0] if hit else None
                lam = [H.level_info(l).cheb_lambda for l in range(1, ell + 1)] if sm else []
                print(json.dumps({"family": args.grid_family, "k": k, "l": ell, "n": 5 << ell,
                                  "dofs": H.level_info(ell).n_free,
                                  "smoother": name, "iterations": its, "iterations_estimate": est,
                                  "solve_ms": ms,
                                  "lambda": lam, "setup_s": t_setup}), flush=True)
                del H


def stopping_study(args):
    """Stopping-criteria study at the paper's settings (Sec. 4, stopping criteria): 5x5 coarsest mesh,
    the paper's manufactured solution (zero pressure), unrestarted FGMRES from a zero guess, V(nu, nu).
    The same system is solved with relative tolerances 1e-2 * 2^-i, i = 0, 1, ..., down to 1e-15 or
    until a solve no longer converges within 100 iterations; after every solve the library measures the
    relative H^1 velocity error and the mean-free L^2 pressure error.  The tolerance needed for a
    quantity is the largest one from which on every stricter solve stays within 1 % of the error of
    the strictest solve.  One JSON line per (k, l, smoother)."""
    import numpy as np
    import torch

    import paper_2409_14222_amd as vk
    torch.cuda.init()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    nu = args.study_nu
    smoothers = {"damped": (vk.VK_SMOOTH_DAMPED, vk.VK_WEIGHT_MULTIPLICITY),
                 "chebyshev": (vk.VK_SMOOTH_CHEBYSHEV, vk.VK_WEIGHT_NONE)}
    for k in [int(v) for v in args.grid_k.split(",")]:
        for ell in [int(v) for v in args.grid_levels.split(",")]:
            for name in args.study_smoothers.split(","):
                sm, wt = smoothers[name]
                H = vk.Hierarchy(k, 5, ell + 1, forcing=vk.VK_F_PAPER_MMS, smoother=sm, weighting=wt,
                                 family={"quad": vk.VK_TH_QUAD, "bdm": vk.VK_BDM}.get(args.grid_family, vk.VK_TH))
                H.bind(max_restart=100).setup()
                b = torch.tensor(H.rhs(), device="cuda")
                x = torch.empty_like(b)
                rows = []
                i = 0
                while True:
                    rtol = 1e-2 * 2.0 ** -i
                    if rtol < 1e-15:
                        break
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r = H.solve(b, x, restart=100, maxit=100, rtol=rtol, nu_pre=nu, nu_post=nu)
                    torch.cuda.synchronize()
                    ms = 1e3 * (time.perf_counter() - t0)
                    if not r["converged"]:
                        break
                    eu, ep = H.solution_errors(x.cpu().numpy())
                    rows.append({"rtol": rtol, "its": r["iterations"], "e_u": eu, "e_p": ep, "ms": ms})
                    i += 1
                out = {"family": args.grid_family, "k": k, "l": ell, "n": 5 << ell,
                       "dofs": H.level_info(ell).n_free, "smoother": name, "nu": nu, "rows": rows}
                if rows:
                    for key, tag in (("e_u", "velocity"), ("e_p", "pressure")):
                        ref = rows[-1][key]
                        need = rows[-1]
                        for row in reversed(rows):
                            if row[key] <= 1.01 * ref:
                                need = row
                            else:
                                break
                        out[tag] = {"rtol": need["rtol"], "its": need["its"], "error": need[key],
                                    "ms": need["ms"], "strictest_error": ref}
                print(json.dumps(out), flush=True)
                del H


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="p4p3-64", choices=sorted(WORKLOADS))
    ap.add_argument("--store", default=None, choices=["fp64", "fp32"], help="default: the workload's (else fp64)")
    ap.add_argument("--nrhs", type=int, default=None,
                    help="right-hand sides solved together (random smooth forcings, seeds 20240922 + j); "
                         "with --store fp32 the patch applies are FP32 matrix-core GEMMs; default: the "
                         "workload's (else 1)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay every Arnoldi step from a captured HIP graph (the apply kernel is then not "
                         "event-timed; the roofline entry is omitted)")
    ap.add_argument("--serve", action="store_true", help="serving workload (continuous batching) instead of one solve")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-pool-gb", type=int, default=96)
    ap.add_argument("--smoother", default="damped", choices=["damped", "chebyshev"],
                    help="chebyshev: Chebyshev-accelerated additive Vanka on [lambda/4, 1.1 lambda] (Sec. 3)")
    ap.add_argument("--weighting", default=None, choices=["multiplicity", "none"],
                    help="patch-sum weights; default: multiplicity for damped, none for chebyshev")
    ap.add_argument("--paper-grid", action="store_true",
                    help="iteration counts at the paper's settings (5x5 coarsest mesh, unrestarted FGMRES)")
    ap.add_argument("--stopping-study", action="store_true",
                    help="tolerance needed for discretisation-level errors (paper settings, --grid-k/--grid-levels)")
    ap.add_argument("--grid-smoothers", default="damped,chebyshev,chebyshev-weighted",
                    help="smoothers of --paper-grid")
    ap.add_argument("--study-nu", type=int, default=1)
    ap.add_argument("--study-smoothers", default="damped,chebyshev")
    ap.add_argument("--grid-family", default="tri", choices=["tri", "quad", "bdm"],
                    help="Taylor-Hood on the two-triangle mesh (P_k) or on squares (Q_k), or BDM_k-dP_{k-1} "
                         "with interior penalty on the two-triangle mesh")
    ap.add_argument("--grid-k", default="2,3,4,5,6")
    ap.add_argument("--grid-levels", default="1,2,3,4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 256 MiB device copy (y = x), the reference for HBM counter scaling")
    ap.add_argument("--stream-bandwidth", action="store_true",
                    help="run only plain streaming kernels over 2 GiB (a read-only reduction and a copy) and "
                         "print their HBM rates: the attainable bandwidth next to the 8 TB/s peak")
    ap.add_argument("--cpu-sample", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_sample:
        print(json.dumps(cpu_sample(args.cpu_sample)))
        return
    if args.stream_bandwidth:
        import torch
        n = 256 * 1024 * 1024  # 2 GiB of float64
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        out = {}
        for name, fn, nbytes in (("read (sum)", lambda: x.sum(), 8 * n), ("copy (y = x)", lambda: y.copy_(x), 16 * n)):
            for _ in range(3):
                fn()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(20):
                fn()
            b.record()
            b.synchronize()
            s_per = a.elapsed_time(b) / 20 / 1e3
            out[name] = {"GB/s": nbytes / s_per / 1e9, "frac_of_8TBs": nbytes / s_per / 8e12}
        print(json.dumps(out))
        return
    if args.copy_calibration:
        import torch
        n = 32 * 1024 * 1024  # 256 MiB of float64 read, 256 MiB written per launch
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 8 * n, "copy_calibration_bytes_written": 8 * n}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver path here is single-GPU (multi-GPU sharding is a design "
              "note, not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.paper_grid:
        paper_grid(args)
        return
    if args.stopping_study:
        stopping_study(args)
        return

    import numpy as np
    import torch

    import paper_2409_14222_amd as vk
    w = WORKLOADS[args.workload]
    if args.store is None:
        args.store = w.get("store", "fp64")
    if args.nrhs is None:
        args.nrhs = w.get("nrhs", 1)
    store = vk.VK_STORE_FP32 if args.store == "fp32" else vk.VK_STORE_FP64
    torch.cuda.init()
    stream = torch.cuda.Stream()  # a non-default stream (needed for graph capture)
    torch.cuda.set_stream(stream)
    t0 = time.perf_counter()
    dim = w.get("dim", 2)
    cheb = args.smoother == "chebyshev"
    if args.weighting is None:
        args.weighting = "none" if cheb else "multiplicity"
    fam = {"sv": vk.VK_SV, "bdm": vk.VK_BDM}.get(w.get("family"), vk.VK_TH)
    if fam == vk.VK_BDM and args.nrhs != 1:
        raise SystemExit("the BDM workload solves the paper's manufactured solution (--nrhs 1)")
    H = vk.Hierarchy(w["k"], w["n0"], w["levels"], dim=dim, store=store,
                     forcing=vk.VK_F_CUBE_MMS if dim == 3 else (vk.VK_F_PAPER_MMS if fam == vk.VK_BDM
                                                                else vk.VK_F_BASELINE_MMS),
                     family=fam,
                     smoother=vk.VK_SMOOTH_CHEBYSHEV if cheb else vk.VK_SMOOTH_DAMPED,
                     weighting=vk.VK_WEIGHT_NONE if args.weighting == "none" else vk.VK_WEIGHT_MULTIPLICITY)
    t_host = time.perf_counter() - t0
    t0 = time.perf_counter()
    R = args.nrhs
    if R < 1 or R > 64:
        raise SystemExit("--nrhs must be in 1..64")
    H.bind(max_rhs=R)
    H.setup()
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    t0 = time.perf_counter()
    tuning = H.autotune(reps=20)
    t_tune = time.perf_counter() - t0
    Lf = w["levels"] - 1
    info = H.level_info(Lf)
    import synth
    if R == 1 and w.get("family") != "sv":
        b = torch.tensor(H.rhs(), device="cuda")
    else:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=16) as ex:  # the library call releases the GIL
            cols = list(ex.map(lambda j: H.rhs_random(synth.forcing_coeffs(synth.SEED + j)), range(R)))
        b = torch.tensor(np.stack(cols, axis=1), device="cuda").contiguous()
        if R == 1:
            b = b[:, 0].contiguous()
    x = torch.empty_like(b)

    def one_solve():
        if R == 1:
            return [H.solve(b, x, graphs=args.graphs)]
        return H.solve_multi(b, x, R, graphs=args.graphs)[1]

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    H.kernel_timing(enable=not args.graphs, reset=True)
    lat = []
    its = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        res = one_solve()
        lat.append(time.perf_counter() - s0)
        its.extend(r["iterations"] for r in res)
        if not all(r["converged"] for r in res):
            raise SystemExit(f"solve did not converge: {res}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    launches, kms = H.kernel_timing(enable=False, reset=True)
    solves_per_s = args.steps * R / elapsed
    its_mean = float(np.mean(its))
    # Vanka DoF-sweep rate: finest-level sweeps (residual, patch apply, scatter) timed with events in
    # three further eager solves, outside the timed region
    H.sweep_timing(enable=True, reset=True)
    for _ in range(3):
        if R == 1:
            H.solve(b, x)
        else:
            H.solve_multi(b, x, R)
    n_sweeps, sweep_ms = H.sweep_timing(enable=False, reset=True)
    sweep_s = sweep_ms / 1e3

    # dominant kernel: finest-level additive patch apply (a GEMM over R columns when R > 1).  With
    # one right-hand side the method needs each symmetric inverse's triangle, sum n (n + 1) / 2
    # entries (the algorithmic bytes); the tiled storage the kernel reads holds more (whole 8 x 8
    # diagonal tiles, zero rows below n: inv_elems_tri, reported beside it).  With several
    # right-hand sides the full column-major inverses are read (sum n^2)
    s = 4 if store == vk.VK_STORE_FP32 else 8
    tri_entries = (info.sum_n2 + info.sum_n) // 2
    inv_bytes = (tri_entries if R == 1 else info.sum_n2) * s
    vec_bytes = info.sum_n * 4 + info.sum_n * R * (8 + s)
    apply_bytes = inv_bytes + vec_bytes
    stored_bytes = (info.inv_elems_tri if R == 1 else info.sum_n2) * s + vec_bytes
    apply_flops = 2.0 * info.sum_n2 * R
    avg_s = kms / 1e3 / max(launches, 1)
    src = "patch_apply.hip" if R == 1 else "patch_gemm.hip"
    traffic = MEASURED_TRAFFIC.get((src, kernel_source_hash(src), args.workload, args.store, R))
    achieved = apply_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    out = {
        "metric": "Stokes solves/s to 1e-10 rel. residual",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if store == vk.VK_STORE_FP64 else "f64 (patch inverses stored/applied in f32)",
        "data": "synthetic (manufactured solution)",
        "config": {"workload": w["desc"], "dofs_free": info.n_free, "nnz": info.nnz, "patches": info.n_patches,
                   "patch_dofs_sum": info.sum_n, "max_patch": info.max_n, "store": args.store,
                   "graphs": args.graphs, "smoother": args.smoother, "weighting": args.weighting},
        "iterations": its_mean,
        "nrhs": R,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99))},
        "vanka_dof_sweeps_per_s_finest": info.n_free * R * n_sweeps / sweep_s if sweep_s > 0 else None,
        "patch_dofs_per_s_finest": info.sum_n * R * n_sweeps / sweep_s if sweep_s > 0 else None,
        "finest_sweep_us": 1e6 * sweep_s / max(n_sweeps, 1),
        "setup_s": {"host_assembly": t_host, "device_upload_gather_invert": t_dev, "autotune": t_tune},
        "tuning": tuning,
        "roofline": {"kernel": "patch_apply_tri_kernel (finest level)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": apply_bytes, "stored_bytes_per_launch": stored_bytes,
                     "stored_over_algorithmic": stored_bytes / apply_bytes,
                     "traffic_over_algorithmic": traffic / apply_bytes if traffic else None,
                     "avg_launch_us": avg_s * 1e6, "launches": launches},
    }
    if R > 1:
        peak_tf = 157.3  # FP32 dense matrix-core (and vector) peak of MI355X
        tf = apply_flops / avg_s / 1e12 if avg_s > 0 else 0.0
        out["roofline"]["flops_per_launch"] = apply_flops
        out["roofline"]["compute"] = {"achieved": tf, "peak": peak_tf if store == vk.VK_STORE_FP32 else 78.6,
                                      "unit": "TFLOP/s",
                                      "frac": tf / (peak_tf if store == vk.VK_STORE_FP32 else 78.6)}
        out["roofline"]["kernel"] = ("patch_gemm_mfma_kernel (finest level, FP32 matrix cores)"
                                     if store == vk.VK_STORE_FP32 else "patch_gemm_f64_kernel (finest level)")
        out["data"] = "synthetic (seeded random smooth forcings)"
        out["metric"] = "Stokes solves/s to 1e-10 rel. residual (each of the nrhs right-hand sides counts)"
    if args.graphs:
        out.pop("roofline")
    if not args.no_cpu_baseline:
        env = dict(os.environ, HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample",
                            f"{args.workload}:{args.smoother}:{args.weighting}"], capture_output=True, text=True,
                           env=env, timeout=900)
        if r.returncode == 0:
            out["cpu_baseline"] = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            out["cpu_baseline"] = {"error": r.stderr[-500:]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
