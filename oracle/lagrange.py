"""Equispaced Lagrange P_k bases on the reference simplex (oracle).

The Taylor-Hood velocity space is continuous vector P_k and the pressure
space continuous P_{k-1} (Sec. 2, the Taylor-Hood pairs; Case 1 of Sec. 3).
The paper does not name a nodal basis; the oracle uses equispaced nodes.

Construction: the nodal basis is the monomial basis multiplied by the
inverse of the Vandermonde matrix V[i, m] = mono_m(node_i), so that
phi_j(node_i) = delta_ij.  This is deliberately the textbook route.
"""
import itertools

import numpy as np


def monomial_exponents(dim, k):
    """All exponent tuples of total degree <= k (fixed order)."""
    out = []
    for deg in range(k + 1):
        for e in itertools.product(range(deg + 1), repeat=dim):
            if sum(e) == deg:
                out.append(e)
    return out


def lattice_nodes(dim, k):
    """Integer lattice coordinates of the P_k nodes: tuples a with sum(a) <= k.

    The node position on the reference simplex is a / k.  For k = 0 the only
    node is the origin (not used: Taylor-Hood pressures have k - 1 >= 1).
    """
    out = []
    for a in itertools.product(range(k + 1), repeat=dim):
        if sum(a) <= k:
            out.append(a)
    return out


class LagrangeBasis:
    """P_k nodal basis on the reference simplex with vertices 0, e_1..e_dim."""

    def __init__(self, dim, k):
        self.dim, self.k = dim, k
        self.lattice = lattice_nodes(dim, k)
        self.nodes = np.array(self.lattice, dtype=float) / k
        self.exps = monomial_exponents(dim, k)
        V = self._mono(self.nodes)
        # coefficients C[m, j]: phi_j = sum_m C[m, j] mono_m
        self.C = np.linalg.inv(V)

    def _mono(self, x):
        x = np.atleast_2d(x)
        return np.stack([np.prod(x ** np.array(e), axis=1) for e in self.exps], axis=1)

    def _mono_grad(self, x):
        x = np.atleast_2d(x)
        g = np.zeros((x.shape[0], len(self.exps), self.dim))
        for m, e in enumerate(self.exps):
            for d in range(self.dim):
                if e[d] == 0:
                    continue
                e2 = list(e)
                e2[d] -= 1
                g[:, m, d] = e[d] * np.prod(x ** np.array(e2), axis=1)
        return g

    def eval(self, x):
        """phi_j(x_p): array (npts, nbasis)."""
        return self._mono(x) @ self.C

    def grad(self, x):
        """d phi_j / d xi_d at x_p: array (npts, nbasis, dim)."""
        return np.einsum("pmd,mj->pjd", self._mono_grad(x), self.C)
