"""Quadrature rules for the oracle.

The bilinear forms a(.,.) and b(.,.) of the weak Stokes problem (Sec. 2,
the variational formulation) have polynomial integrands on affine cells and
the load <f, v> does not; both are integrated with one fixed rule: the
collapsed ("conical", Duffy) product of Gauss-Legendre rules on the
reference simplex.

With q Gauss-Legendre points per direction the collapsed triangle rule is
exact for total degree <= 2q - 2 and the collapsed tetrahedron rule for
total degree <= 2q - 3 (the Jacobian adds one, resp. two, powers of the
collapsed coordinate).
"""
import numpy as np


def gauss_legendre01(q):
    """q-point Gauss-Legendre rule on [0, 1] (nodes ascending, weights sum 1)."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(q):
    """Collapsed rule on the reference triangle {(0,0),(1,0),(0,1)}.

    Maps (s, t) in [0,1]^2 to (x, y) = (s, t (1 - s)) with Jacobian (1 - s).
    Returns points (q*q, 2) and weights (q*q,) summing to 1/2.
    """
    g, w = gauss_legendre01(q)
    pts, wts = [], []
    for i in range(q):
        for j in range(q):
            s, t = g[i], g[j]
            pts.append((s, t * (1.0 - s)))
            wts.append(w[i] * w[j] * (1.0 - s))
    return np.array(pts), np.array(wts)


def tetrahedron_rule(q):
    """Collapsed rule on the reference tetrahedron with vertices 0, e1, e2, e3.

    (s, t, r) in [0,1]^3 -> (s, t (1-s), r (1-s)(1-t)), Jacobian (1-s)^2 (1-t).
    Weights sum to 1/6.
    """
    g, w = gauss_legendre01(q)
    pts, wts = [], []
    for i in range(q):
        for j in range(q):
            for l in range(q):
                s, t, r = g[i], g[j], g[l]
                pts.append((s, t * (1.0 - s), r * (1.0 - s) * (1.0 - t)))
                wts.append(w[i] * w[j] * w[l] * (1.0 - s) ** 2 * (1.0 - t))
    return np.array(pts), np.array(wts)


def simplex_rule(dim, q):
    return triangle_rule(q) if dim == 2 else tetrahedron_rule(q)
