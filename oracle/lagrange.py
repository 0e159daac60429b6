"""Equispaced Lagrange P_k bases on the reference simplex (oracle).

The Taylor-Hood velocity space is continuous vector P_k and the pressure
space continuous P_{k-1} (Sec. 2, the Taylor-Hood pairs; Case 1 of Sec. 3).
The paper does not name a nodal basis; the oracle uses equispaced nodes.

Definition: the node with lattice index a (sum a <= k, position a / k) has the
barycentric multi-index alpha = (k - sum a, a_1, .., a_dim), and its basis
function is the product over the barycentric coordinates lambda_i of
  P_{alpha_i}(lambda_i),  P_m(t) = prod_{j < m} (k t - j) / (j + 1),
which is 1 at the node and vanishes at every other node of the lattice (the
closed form of the equispaced simplex basis).  It is evaluated as written, so
its values carry a few roundings at any k.

The monomial route (the nodal basis as the monomials times the inverse of the
Vandermonde matrix on the nodes) gives the same polynomials in exact
arithmetic; it stays here as `VandermondeBasis`, a check of the product form
at low orders: its Vandermonde matrix has condition 3e3 at k = 4 but 7e7 at
k = 8, where the coefficients lose about eight digits.
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


def _factor(k, m, t):
    """P_m(t) = prod_{j < m} (k t - j) / (j + 1) and its derivative, for an array t."""
    val = np.ones_like(t)
    der = np.zeros_like(t)
    for j in range(m):
        f = (k * t - j) / (j + 1)
        der = der * f + val * (k / (j + 1))
        val = val * f
    return val, der


class LagrangeBasis:
    """P_k nodal basis on the reference simplex with vertices 0, e_1..e_dim (product form)."""

    def __init__(self, dim, k):
        self.dim, self.k = dim, k
        self.lattice = lattice_nodes(dim, k)
        self.nodes = np.array(self.lattice, dtype=float) / k
        self.alpha = np.array([(k - sum(a),) + tuple(a) for a in self.lattice], dtype=int)

    def _bary(self, x):
        x = np.atleast_2d(np.asarray(x, dtype=float))
        return np.concatenate([1.0 - x.sum(1, keepdims=True), x], axis=1)

    def _factors(self, x):
        lam = self._bary(x)
        npts, nb = lam.shape[0], len(self.lattice)
        F = np.empty((npts, nb, self.dim + 1))
        D = np.empty((npts, nb, self.dim + 1))
        for j, al in enumerate(self.alpha):
            for i in range(self.dim + 1):
                F[:, j, i], D[:, j, i] = _factor(self.k, al[i], lam[:, i])
        return F, D

    def eval(self, x):
        """phi_j(x_p): array (npts, nbasis)."""
        F, _ = self._factors(x)
        return np.prod(F, axis=2)

    def grad(self, x):
        """d phi_j / d xi_d at x_p: array (npts, nbasis, dim).  lambda_0 = 1 - sum xi, lambda_{d+1} = xi_d."""
        F, D = self._factors(x)
        npts, nb, nl = F.shape
        # derivative of the product with respect to lambda_i (the other factors kept)
        dl = np.empty_like(F)
        for i in range(nl):
            others = np.prod(np.delete(F, i, axis=2), axis=2)
            dl[:, :, i] = D[:, :, i] * others
        return dl[:, :, 1:] - dl[:, :, :1]


class VandermondeBasis:
    """The same space through the monomial Vandermonde inverse (a check of LagrangeBasis)."""

    def __init__(self, dim, k):
        self.dim, self.k = dim, k
        self.lattice = lattice_nodes(dim, k)
        self.nodes = np.array(self.lattice, dtype=float) / k
        self.exps = monomial_exponents(dim, k)
        self.V = self._mono(self.nodes)
        self.C = np.linalg.inv(self.V)  # phi_j = sum_m C[m, j] mono_m

    def _mono(self, x):
        x = np.atleast_2d(x)
        return np.stack([np.prod(x ** np.array(e), axis=1) for e in self.exps], axis=1)

    def eval(self, x):
        return self._mono(x) @ self.C
