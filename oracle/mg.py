"""Monolithic multigrid V-cycle (oracle), Sec. 3.

One V(nu_pre, nu_post) cycle approximates K_L^{-1} r on the finest level:

  level l > 0 :  e = 0
                 nu_pre smoothing sweeps on K_l e = r (damped additive Vanka, or nu_pre
                 Chebyshev-accelerated steps of it: oracle.chebyshev)
                 r_c = P_l^T (r - K_l e)          (restriction R = P^T)
                 e_c = V(l - 1, r_c)
                 e  += P_l e_c                     (canonical prolongation)
                 nu_post smoothing sweeps on K_l e = r
  level 0     :  coarsest solve

Coarse operators are rediscretised on every level (for Taylor-Hood this is
the Galerkin product P^T K P, Sec. 3).  The paper does not say how the
coarsest problem is solved, and K_0 is singular (constant pressure); the
oracle solves the bordered system [[K_0, z], [z^T, 0]] [e; mu] = [r; 0]
with z the normalised constant pressure, by a dense LU.
"""
import numpy as np
import scipy.linalg as sla

from .vanka import AdditiveVanka


class VCycle:
    def __init__(self, hier, omega=0.5, nu_pre=2, nu_post=2, construct="composite",
                 weighting="multiplicity", smoother="damped", est_steps=10, est_seed=0):
        from .patches import build_patches
        self.hier = hier
        self.levels = hier.levels
        self.P = hier.P
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.smoothers = [None] + [
            AdditiveVanka(L.K, build_patches(L, construct), omega, weighting)
            for L in self.levels[1:]]
        # Chebyshev acceleration (Sec. 3): per-level largest-eigenvalue estimate of B K
        self.cheb = None
        if smoother == "chebyshev":
            from . import chebyshev as ch
            self.cheb = [None]
            for l in range(1, len(self.levels)):
                S = self.smoothers[l]
                B = lambda r, S=S: S.weight * S.correction(r)
                v0 = ch.start_vector(self.levels[l].N, est_seed, l)
                lam = ch.arnoldi_lambda(self.levels[l].K, B, v0, est_steps)
                self.cheb.append(ch.ChebyshevVanka(S, lam))
        elif smoother != "damped":
            raise ValueError(smoother)
        L0 = self.levels[0]
        z = L0.nullvec()
        N0 = L0.N
        Kb = np.zeros((N0 + 1, N0 + 1))
        Kb[:N0, :N0] = L0.K.toarray()
        Kb[:N0, N0] = z
        Kb[N0, :N0] = z
        self.coarse_lu = sla.lu_factor(Kb)
        self.N0 = N0

    def coarse_solve(self, r):
        rhs = np.concatenate([r, [0.0]])
        return sla.lu_solve(self.coarse_lu, rhs)[: self.N0]

    def smooth(self, l, b, x, nsweeps):
        if self.cheb is not None:
            return self.cheb[l].sweeps(b, x, nsweeps)
        for _ in range(nsweeps):
            x = self.smoothers[l].sweep(b, x)
        return x

    def cycle(self, l, r):
        if l == 0:
            return self.coarse_solve(r)
        K = self.levels[l].K
        e = np.zeros_like(r)
        e = self.smooth(l, r, e, self.nu_pre)
        rc = self.P[l].T @ (r - K @ e)
        ec = self.cycle(l - 1, rc)
        e = e + self.P[l] @ ec
        e = self.smooth(l, r, e, self.nu_post)
        return e

    def apply(self, r):
        return self.cycle(len(self.levels) - 1, r)
