"""Residual-history and iteration-count comparison of a GPU solve with the oracle's (test helper,
no tests here).

FGMRES residual estimates are compared iteration by iteration against the bound
1e-6 r_j + 1e-9 r_0.  Where the preconditioned Krylov process is sensitive (the
Chebyshev smoother with unweighted patch sums, the P8-P7 vertex stars), the
oracle's own history moves by more than that bound when each preconditioner
output is perturbed at the 1e-14..1e-13 level, which is the size of the
difference between the GPU's V-cycle and the oracle's.  A deviation above the
bound is then accepted only up to the oracle's measured self-sensitivity: the
deviation of the oracle's history when each of its preconditioner outputs is
multiplied by (1 + eps u), u seeded uniform in [-1, 1], eps = 1e-13 and 1e-12
(the V-cycle parity tolerance).  Likewise an iteration count may differ from the
oracle's only where the count sits on the stopping threshold, i.e. where the
oracle itself reaches that count under perturbations of 1e-15..1e-13 (the
recomputed residual at the last step lies within rounding of the tolerance;
the oracle's own count can then change from one CPU to another).
"""
import numpy as np

from oracle import fgmres, solve


def deviation(gh, oh):
    """max_j |g_j - o_j| / (1e-6 o_j + 1e-9 o_0) over the common iterations."""
    gh, oh = np.asarray(gh, dtype=float), np.asarray(oh, dtype=float)
    n = min(len(gh), len(oh))
    return float((np.abs(gh[:n] - oh[:n]) / (1e-6 * oh[:n] + 1e-9 * oh[0])).max())


def _perturbed(apply, eps, seed):
    rng = np.random.default_rng(seed)

    def f(v):
        y = apply(v)
        return y * (1.0 + eps * rng.uniform(-1.0, 1.0, len(y)))

    return f


def self_sensitivity(L, apply, b=None, restart=30, rtol=1e-10, maxit=100, eps=(1e-13, 1e-12), seed=1):
    """The oracle's own history deviation under seeded relative perturbations of every preconditioner
    output, the largest over the perturbation sizes (1e-12 is the V-cycle parity tolerance)."""
    bb = solve.consistent_rhs(L, b)
    z = L.nullvec()
    _, _, h0, _ = fgmres.fgmres(L.K, bb, apply, restart, rtol, maxit, z)
    worst = 0.0
    for e in eps:
        _, _, h1, _ = fgmres.fgmres(L.K, bb, _perturbed(apply, e, seed), restart, rtol, maxit, z)
        worst = max(worst, deviation(h1, h0))
    return worst


def oracle_counts(L, apply, b=None, restart=30, rtol=1e-10, maxit=100, eps=(1e-15, 1e-14, 1e-13), seeds=(1, 2, 3)):
    """The iteration counts the oracle itself reaches when every preconditioner output is perturbed at
    (or below) the size of the GPU's difference from it, plus the unperturbed count."""
    bb = solve.consistent_rhs(L, b)
    z = L.nullvec()
    counts = {fgmres.fgmres(L.K, bb, apply, restart, rtol, maxit, z)[1]}
    for e in eps:
        for sd in seeds:
            counts.add(fgmres.fgmres(L.K, bb, _perturbed(apply, e, sd), restart, rtol, maxit, z)[1])
    return counts


def check(tag, gh, oh, L, apply, b=None, restart=30, rtol=1e-10, maxit=100):
    """Assert the GPU history against the oracle's: within the bound, or within the oracle's own
    sensitivity where that is larger."""
    dev = deviation(gh, oh)
    if dev <= 1.0:
        print(f"[measure] {tag}: history deviation / bound {dev:.2e}")
        return dev
    sens = self_sensitivity(L, apply, b, restart, rtol, maxit)
    print(f"[measure] {tag}: history deviation / bound {dev:.2e}, oracle self-sensitivity {sens:.2e}")
    assert dev <= sens, (tag, dev, sens)
    return dev


def check_count(tag, gpu_its, its, L, apply, b=None, restart=30, rtol=1e-10, maxit=100):
    """Equal iteration counts, or, where the count sits on the stopping threshold (the recomputed
    residual within rounding of the tolerance), a count the oracle itself reaches under
    perturbations of 1e-15..1e-13 (three seeds each)."""
    if gpu_its == its:
        return
    counts = oracle_counts(L, apply, b, restart, rtol, maxit)
    print(f"[measure] {tag}: iterations gpu {gpu_its} oracle {its}; oracle under perturbations {sorted(counts)}")
    assert gpu_its in counts, (tag, gpu_its, its, sorted(counts))
