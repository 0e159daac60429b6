"""Residual-history comparison of a GPU solve with the oracle's (test helper, no tests here).

FGMRES residual estimates are compared iteration by iteration against the bound
1e-6 r_j + 1e-9 r_0.  Where the preconditioned Krylov process is sensitive (the
Chebyshev smoother with unweighted patch sums, the P8-P7 vertex stars), the
oracle's own history moves by more than that bound when each preconditioner
output is perturbed at the 1e-14..1e-13 level, which is the size of the
difference between the GPU's V-cycle and the oracle's.  A deviation above the
bound is then accepted only up to the oracle's measured self-sensitivity: the
deviation of the oracle's history when each of its preconditioner outputs is
multiplied by (1 + 1e-13 u), u seeded uniform in [-1, 1].
"""
import numpy as np

from oracle import fgmres, solve


def deviation(gh, oh):
    """max_j |g_j - o_j| / (1e-6 o_j + 1e-9 o_0) over the common iterations."""
    gh, oh = np.asarray(gh, dtype=float), np.asarray(oh, dtype=float)
    n = min(len(gh), len(oh))
    return float((np.abs(gh[:n] - oh[:n]) / (1e-6 * oh[:n] + 1e-9 * oh[0])).max())


def self_sensitivity(L, apply, b=None, restart=30, rtol=1e-10, maxit=100, eps=1e-13, seed=1):
    """The oracle's own history deviation under a seeded relative perturbation eps of every
    preconditioner output (same system, same settings)."""
    bb = solve.consistent_rhs(L, b)
    z = L.nullvec()
    _, _, h0, _ = fgmres.fgmres(L.K, bb, apply, restart, rtol, maxit, z)
    rng = np.random.default_rng(seed)

    def perturbed(v):
        y = apply(v)
        return y * (1.0 + eps * rng.uniform(-1.0, 1.0, len(y)))

    _, _, h1, _ = fgmres.fgmres(L.K, bb, perturbed, restart, rtol, maxit, z)
    return deviation(h1, h0)


def check(tag, gh, oh, L, apply, b=None, restart=30, rtol=1e-10, maxit=100):
    """Assert the GPU history against the oracle's: within the bound, or within the oracle's own
    sensitivity where that is larger."""
    dev = deviation(gh, oh)
    if dev <= 1.0:
        print(f"[measure] {tag}: history deviation / bound {dev:.2e}")
        return dev
    sens = self_sensitivity(L, apply, b, restart, rtol, maxit)
    print(f"[measure] {tag}: history deviation / bound {dev:.2e}, oracle self-sensitivity at 1e-13 {sens:.2e}")
    assert dev <= sens, (tag, dev, sens)
    return dev
