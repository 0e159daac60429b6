"""End-to-end oracle solve: hierarchy, V-cycle preconditioner, FGMRES (Sec. 3, Sec. 4).

The pressure-singular system is made consistent by removing the constant
pressure component from the right-hand side (b <- b - (z.b) z), and the
returned pressure is normalised by the same projection.
"""
import numpy as np

from . import fgmres as _fg
from . import mg, th


def setup(dim, k, n0, nlevels, nu, field_factory, omega=0.5, nu_sweeps=2, construct="composite",
          weighting="multiplicity", family="th", smoother="damped", est_steps=10, est_seed=0):
    if family == "sv":
        from . import sv
        H = sv.SVHierarchy(k, n0, nlevels, nu, field_factory)
        construct = "macro"
    elif family == "bdm":
        from . import bdm
        H = bdm.BDMHierarchy(k, n0, nlevels, nu, field_factory)
    elif family == "qk":
        from . import qk
        H = qk.QKHierarchy(k, n0, nlevels, nu, field_factory)
    else:
        H = th.THHierarchy(dim, k, n0, nlevels, nu, field_factory)
    V = mg.VCycle(H, omega=omega, nu_pre=nu_sweeps, nu_post=nu_sweeps, construct=construct,
                  weighting=weighting, smoother=smoother, est_steps=est_steps, est_seed=est_seed)
    return H, V


def consistent_rhs(level, b=None):
    z = level.nullvec()
    b = level.b if b is None else b
    return b - (z @ b) * z


def solve(H, V, b=None, restart=30, rtol=1e-10, maxit=100):
    L = H.finest
    z = L.nullvec()
    b = consistent_rhs(L, b)
    return _fg.fgmres(L.K, b, V.apply, restart, rtol, maxit, z)
