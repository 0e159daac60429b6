"""Discretisation-error norms (oracle), Sec. 4.4.

The velocity error is the relative H^1 norm ||u - u_h||_1 / ||u||_1; the
pressure error is the L^2 norm of (p - p_h) after removing the L^2 mean of
the difference (the pressure is only determined up to a constant).  The
paper integrates with adaptive quadrature; the oracle uses the fixed
collapsed Gauss rule with k + 6 points per direction.
"""
import numpy as np

from . import quad


def errors(level, x):
    dim, k = level.dim, level.k
    qp, qw = level.quad_rule(k + 6)
    Pv, Gv, Pp = level.vb.eval(qp), level.vb.grad(qp), level.pb.eval(qp)
    F = level.field
    e1 = n1 = 0.0
    ep_int = ep2 = area = 0.0
    for cell in level.cells:
        v0, J = level.cell_geometry(cell)
        detJ = abs(np.linalg.det(J))
        g = Gv @ np.linalg.inv(J)
        w = qw * detJ
        xq = v0[None, :] + qp @ J.T
        U = np.zeros((len(Pv[0]), dim))
        for i, G in enumerate(level.cell_nodes(cell, k)):
            idx = level.vel_index(G)
            if idx >= 0:
                U[i] = x[dim * idx: dim * idx + dim]
            else:
                U[i] = F.u(np.array(G, dtype=float)[None, :] / level.Mv)[0]
        Pl = np.array([x[level.p_dof(G)] for G in level.cell_nodes(cell, k - 1)])
        uh = Pv @ U
        guh = np.einsum("qid,ic->qcd", g, U)
        ue, gue = F.u(xq), F.grad_u(xq)
        e1 += w @ (np.sum((ue - uh) ** 2, 1) + np.sum((gue - guh) ** 2, (1, 2)))
        n1 += w @ (np.sum(ue ** 2, 1) + np.sum(gue ** 2, (1, 2)))
        dp = F.p(xq) - Pp @ Pl
        ep_int += w @ dp
        ep2 += w @ dp ** 2
        area += w.sum()
    mean = ep_int / area
    return np.sqrt(e1 / n1), np.sqrt(max(ep2 - 2 * mean * ep_int + mean * mean * area, 0.0))
