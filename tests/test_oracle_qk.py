"""Pins for the quadrilateral Taylor-Hood (Q_k, Q_{k-1}) oracle (CPU only).

Checked against what the mathematics fixes: the nodal and reproduction properties of
the tensor basis, exactness of the tensor Gauss rule, rigid motions in the kernel of
the strain form, the constant pressure in the kernel of K, exact transfer of coarse
polynomials (nested spaces), the velocity convergence rate O(h^k) of the manufactured
solution, patch bookkeeping, and the multigrid solve against a direct solve.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fields, norms, patches, qk, solve


@pytest.mark.parametrize("kk", [1, 2, 3, 5, 7])
def test_tensor_basis_nodal_and_reproducing(kk):
    B = qk.TensorBasis(kk)
    assert len(B.nodes) == (kk + 1) ** 2
    assert np.abs(B.eval(B.nodes) - np.eye(len(B.nodes))).max() <= 1e-13
    rng = np.random.default_rng(0)
    x = rng.random((25, 2))
    assert np.abs(B.eval(x).sum(1) - 1.0).max() <= 1e-12
    # a polynomial of degree kk in each variable is reproduced exactly
    f = lambda p: (p[:, 0] - 0.3) ** kk * (p[:, 1] + 0.1) ** kk - 2.0 * p[:, 0] * p[:, 1] ** max(kk - 1, 0)
    assert np.abs(B.eval(x) @ f(B.nodes) - f(x)).max() <= 1e-12
    h = 1e-6
    for d in range(2):
        e = np.zeros(2); e[d] = h
        fd = (B.eval(x + e) - B.eval(x - e)) / (2 * h)
        assert np.abs(B.grad(x)[:, :, d] - fd).max() <= 1e-5


@pytest.mark.parametrize("q", [1, 3, 6])
def test_square_rule_exact(q):
    pts, w = qk.square_rule(q)
    for a in range(2 * q):
        for b in range(2 * q):
            exact = 1.0 / ((a + 1) * (b + 1))
            assert abs(w @ (pts[:, 0] ** a * pts[:, 1] ** b) - exact) <= 1e-14
    a = 2 * q
    assert abs(w @ pts[:, 0] ** a - 1.0 / (a + 1)) > 1e-10


@pytest.mark.parametrize("k", [2, 3, 4])
def test_element_kernels(k):
    L = qk.QKLevel(k, 2, 1.3, fields.baseline_mms(1.3))
    cell = L.cells[3]
    A, B, _ = L.element_matrices(cell)
    X = np.array([np.array(G, dtype=float) / L.Mv for G in L.cell_nodes(cell, k)])
    nb = len(X)
    rigid = [np.tile([1.0, 0.0], nb), np.tile([0.0, 1.0], nb), np.ravel(np.stack([-X[:, 1], X[:, 0]], 1))]
    for r in rigid:
        assert np.abs(A @ r).max() <= 1e-11 * np.abs(A).max()
    # div of a constant field is zero
    for r in rigid[:2]:
        assert np.abs(B @ r).max() <= 1e-12 * np.abs(B).max()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("k,n", [(2, 4), (3, 3)])
def test_assembled_system(k, n):
    L = qk.QKLevel(k, n, 1.0, fields.baseline_mms(1.0))
    assert L.N == 2 * (k * n - 1) ** 2 + ((k - 1) * n + 1) ** 2
    K = L.K
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    assert np.abs(K @ L.nullvec()).max() <= 1e-12 * abs(K).max()
    # the bordered system is nonsingular (the pair is inf-sup stable on squares)
    z = L.nullvec()
    Kb = np.block([[K.toarray(), z[:, None]], [z[None, :], np.zeros((1, 1))]])
    assert np.linalg.cond(Kb) < 1e12


@pytest.mark.parametrize("k", [2, 3])
def test_prolongation_is_exact_on_coarse_polynomials(k):
    H = qk.QKHierarchy(k, 2, 2, 1.0, fields.baseline_mms)
    C, F = H.levels
    P = H.P[1]
    # velocity: x(1-x)y(1-y) is in Q_k (k >= 2) and vanishes on the boundary; pressure: any Q_{k-1}
    g = lambda X: X[:, 0] * (1 - X[:, 0]) * X[:, 1] * (1 - X[:, 1]) * (1.0 + 0.5 * X[:, 0] ** (k - 2))
    q = lambda X: (X[:, 0] + 0.3) ** (k - 1) * (0.7 - X[:, 1]) ** (k - 1)
    for Lv in (C, F):
        X, kind = Lv.dof_coords()
        Lv._vec = np.where(kind == 0, g(X), np.where(kind == 1, -g(X), q(X)))
    assert np.abs(P @ C._vec - F._vec).max() <= 1e-13


def test_velocity_converges_at_order_k():
    for k in (2, 3):
        errs = []
        for n in (2, 4, 8):
            L = qk.QKLevel(k, n, 1.0, fields.paper_mms(1.0))
            z = L.nullvec()
            b = solve.consistent_rhs(L)
            Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
            x = spla.spsolve(Kb, np.concatenate([b, [0.0]]))[: L.N]
            errs.append(norms.errors(L, x)[0])
        rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert abs(rates[-1] - k) <= 0.25, (k, errs, rates)


@pytest.mark.parametrize("k,n", [(2, 4), (3, 4), (4, 4)])
def test_patches_cover_pressure_once_and_have_star_sizes(k, n):
    L = qk.QKLevel(k, n, 1.0, fields.baseline_mms(1.0))
    P = patches.build_patches(L)
    expected = (n + 1) ** 2 + (0 if k == 2 else 2 * n * (n + 1) + n * n)
    assert len(P) == expected
    pres = np.concatenate([[d for d in I if d >= L.nu_free] for I in P])
    assert np.array_equal(np.sort(pres), np.arange(L.nu_free, L.N))
    assert max(len(I) for I in P) == 2 * (2 * k + 1) ** 2 + 1  # an interior vertex star
    for I in P:
        assert list(I) == sorted(I)
    firsts = [min(d for d in I if d >= L.nu_free) for I in P]
    assert firsts == sorted(firsts)


def test_multigrid_solve_matches_direct_and_is_h_robust():
    counts = []
    for nl in (2, 3):
        H, V = solve.setup(2, 2, 4, nl, 1.0, fields.baseline_mms, family="qk")
        x, its, hist, conv = solve.solve(H, V)
        assert conv
        counts.append(its)
    L = H.finest
    z = L.nullvec()
    b = solve.consistent_rhs(L)
    Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    xd = spla.spsolve(Kb, np.concatenate([b, [0.0]]))[: L.N]
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert abs(counts[1] - counts[0]) <= 2, counts
