"""Pins for the oracle's discretisation (CPU only).

Each test checks the oracle against something other than itself: closed-form
integrals, the Kronecker property, the kernel of the strain-rate form,
exact reproduction of polynomial solutions, convergence rates, the Galerkin
identity of nested conforming spaces, and brute-force counts.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fields, lagrange, norms, quad, th


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("q", [2, 4, 7])
def test_triangle_rule_exact_on_monomials(q):
    # int_T x^a y^b = a! b! / (a + b + 2)!  on the reference triangle
    pts, w = quad.triangle_rule(q)
    for a in range(2 * q - 1):
        for b in range(2 * q - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = w @ (pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(got - exact) <= 1e-14 * max(1.0, exact) + 1e-16, (a, b)


@pytest.mark.parametrize("q", [2, 5])
def test_tet_rule_exact_on_monomials(q):
    pts, w = quad.tetrahedron_rule(q)
    for a, b, c in itertools.product(range(2 * q - 2), repeat=3):
        if a + b + c > 2 * q - 3:
            continue
        exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
        got = w @ (pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
        assert abs(got - exact) <= 1e-14 * max(1.0, exact) + 1e-17


def test_triangle_rule_not_exact_beyond_degree():
    # a plausible off-by-one in the collapsed map would make this exact too
    q = 3
    pts, w = quad.triangle_rule(q)
    a = 2 * q
    exact = math.factorial(a) / math.factorial(a + 2)
    assert abs(w @ pts[:, 0] ** a - exact) > 1e-8


# ---------------------------------------------------------------- Lagrange basis
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 4), (3, 1), (3, 2)])
def test_lagrange_kronecker_and_partition_of_unity(dim, k):
    B = lagrange.LagrangeBasis(dim, k)
    assert len(B.nodes) == math.comb(k + dim, dim)
    assert np.allclose(B.eval(B.nodes), np.eye(len(B.nodes)), atol=1e-12)
    rng = np.random.default_rng(0)
    x = rng.random((20, dim)) / dim
    assert np.allclose(B.eval(x).sum(1), 1.0, atol=1e-12)
    assert np.allclose(B.grad(x).sum(1), 0.0, atol=1e-10)
    # gradient against a central difference
    h = 1e-6
    for d in range(dim):
        e = np.zeros(dim); e[d] = h
        fd = (B.eval(x + e) - B.eval(x - e)) / (2 * h)
        assert np.allclose(B.grad(x)[:, :, d], fd, atol=1e-6)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_product_form_equals_vandermonde_basis(dim, k):
    """The closed product form and the monomial Vandermonde route define the same polynomials;
    at these orders the Vandermonde route is accurate (condition below 1e4)."""
    B, V = lagrange.LagrangeBasis(dim, k), lagrange.VandermondeBasis(dim, k)
    rng = np.random.default_rng(3)
    x = rng.random((40, dim)) / dim
    assert np.abs(B.eval(x) - V.eval(x)).max() <= 1e-12


@pytest.mark.parametrize("k", [6, 7, 8])
def test_high_order_basis_is_nodal_and_exact(k):
    """k = 6..8 (the Vandermonde route loses up to 8 digits here): Kronecker property to a few
    roundings, partition of unity, and exact reproduction of a degree-k polynomial."""
    B = lagrange.LagrangeBasis(2, k)
    assert np.abs(B.eval(B.nodes) - np.eye(len(B.nodes))).max() <= 1e-13
    rng = np.random.default_rng(1)
    x = rng.random((30, 2)) / 2
    assert np.abs(B.eval(x).sum(1) - 1.0).max() <= 1e-12
    f = lambda p: (p[:, 0] - 0.3) ** (k - 2) * (p[:, 1] + 0.2) ** 2 - p[:, 0] * p[:, 1] ** (k - 1)
    assert np.abs(B.eval(x) @ f(B.nodes) - f(x)).max() <= 1e-12
    h = 1e-6
    for d in range(2):
        e = np.zeros(2); e[d] = h
        fd = (B.eval(x + e) - B.eval(x - e)) / (2 * h)
        assert np.abs(B.grad(x)[:, :, d] - fd).max() <= 1e-4


# ---------------------------------------------------------------- element matrices
@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2)])
def test_strain_form_kernel_is_rigid_motions(dim, k):
    """a(u, v) = 2 nu int eps(u):eps(v) vanishes exactly on rigid motions (ker eps)."""
    L = th.THLevel(dim, k, 1, 1.7, (fields.poly_k2 if dim == 2 else fields.poly_3d_k2)(1.7))
    for cell in L.cells[:3]:
        A, Bl, _ = L.element_matrices(cell)
        X = np.array(L.cell_nodes(cell, k), dtype=float) / L.Mv
        modes = []
        for c in range(dim):             # translations
            m = np.zeros((len(X), dim)); m[:, c] = 1.0; modes.append(m.ravel())
        for c, d in itertools.combinations(range(dim), 2):   # rotations
            m = np.zeros((len(X), dim)); m[:, c] = -X[:, d]; m[:, d] = X[:, c]; modes.append(m.ravel())
        for m in modes:
            assert np.abs(A @ m).max() <= 1e-12 * np.abs(A).max()
        # a stretching mode is not in the kernel (catches a dropped symmetric term)
        m = np.zeros((len(X), dim)); m[:, 0] = X[:, 0]
        assert np.abs(A @ m.ravel()).max() > 1e-3 * np.abs(A).max()
        # B applied to a translation is zero; B^T applied to a constant pressure is -int div v
        for m in modes[:dim]:
            assert np.abs(Bl @ m).max() < 1e-13


def test_element_a_matches_closed_form_on_reference_triangle():
    """P1-sized check by hand: for k=2 on the reference right triangle (scaled by 1/n with n=1),
    the x-x block of a for phi = linear vertex function lambda_1 = x, tested with itself:
    nu * int (|grad x|^2 + (d_x x)^2) = nu * 2 * |T| = nu."""
    L = th.THLevel(2, 2, 1, 1.0, fields.poly_k2(1.0))
    cell = L.cells[0]     # (0,0), (1,0), (0,1)
    nodes = L.cell_nodes(cell, 2)
    Xn = np.array(nodes, dtype=float) / 2
    A, _, _ = L.element_matrices(cell)
    u = np.zeros((len(Xn), 2)); u[:, 0] = Xn[:, 0]      # u = (x, 0)
    val = u.ravel() @ A @ u.ravel()
    assert abs(val - 1.0) < 1e-13
    u2 = np.zeros((len(Xn), 2)); u2[:, 0] = Xn[:, 1]    # u = (y, 0): eps has only 1/2 off-diagonal
    assert abs(u2.ravel() @ A @ u2.ravel() - 0.5) < 1e-13


# ---------------------------------------------------------------- counts
def _count_closure_pattern(k, n):
    """Brute force: DoF pairs that share a cell (no pressure-pressure), free DoFs only."""
    Mv, Mp = k * n, (k - 1) * n
    pairs = set()
    for j in range(n):
        for i in range(n):
            for tri in (((i, j), (i + 1, j), (i, j + 1)), ((i + 1, j + 1), (i, j + 1), (i + 1, j))):
                v0 = np.array(tri[0]); e1 = np.array(tri[1]) - v0; e2 = np.array(tri[2]) - v0
                vel, pre = [], []
                for a in range(k + 1):
                    for b in range(k + 1 - a):
                        G = k * v0 + a * e1 + b * e2
                        if 0 < G[0] < Mv and 0 < G[1] < Mv:
                            vel += [("u", G[0], G[1], 0), ("u", G[0], G[1], 1)]
                for a in range(k):
                    for b in range(k - a):
                        G = (k - 1) * v0 + a * e1 + b * e2
                        pre.append(("p", G[0], G[1]))
                for s in vel:
                    for t in vel + pre:
                        pairs.add((s, t)); pairs.add((t, s))
    return len(pairs)


@pytest.mark.parametrize("k,n", [(2, 4), (2, 8), (3, 4), (4, 4)])
def test_dof_and_nnz_counts(k, n):
    L = th.THLevel(2, k, n, 1.0, fields.baseline_mms(1.0))
    assert L.N == 2 * (k * n - 1) ** 2 + ((k - 1) * n + 1) ** 2
    assert L.K.nnz == _count_closure_pattern(k, n)


def test_counts_of_the_workloads():
    # P2-P1 on 16x16 and P4-P3 on 4x4 (coarsest level of the 64x64 hierarchy)
    L = th.THLevel(2, 2, 16, 1.0, fields.baseline_mms(1.0))
    assert (L.N, L.K.nnz) == (2211, 59248)
    L = th.THLevel(2, 4, 4, 1.0, fields.baseline_mms(1.0))
    assert (L.N, L.K.nnz) == (619, 29720)


def test_matrix_symmetric_and_constant_pressure_in_kernel():
    for k, n in ((2, 4), (4, 2)):
        L = th.THLevel(2, k, n, 1.3, fields.baseline_mms(1.3))
        K = L.K
        assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
        z = L.nullvec()
        assert np.abs(K @ z).max() <= 1e-13
        # the zero pressure-pressure block is structurally absent
        assert abs(K[L.nu_free:, L.nu_free:]).max() == 0.0


# ---------------------------------------------------------------- exactness and rates
def _direct(L, b=None):
    z = L.nullvec()
    b = L.b if b is None else b
    b = b - (z @ b) * z
    Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[: L.N]


def _nodal_exact(L, F):
    X, kind = L.dof_coords()
    ex = np.zeros(L.N)
    for c in range(L.dim):
        m = kind == c
        ex[m] = F.u(X[m])[:, c]
    m = kind == L.dim
    ex[m] = F.p(X[m])
    return ex, m


@pytest.mark.parametrize("dim,k,n,fac", [(2, 2, 3, fields.poly_k2), (2, 4, 2, fields.poly_k4),
                                         (3, 2, 2, fields.poly_3d_k2)])
def test_polynomial_solution_reproduced_exactly(dim, k, n, fac):
    nu = 0.7
    L = th.THLevel(dim, k, n, nu, fac(nu))
    x = _direct(L)
    ex, pm = _nodal_exact(L, fac(nu))
    d = x - ex
    d[pm] -= d[pm].mean()
    assert np.abs(d).max() <= 1e-10


def test_polynomial_with_wrong_forcing_is_not_reproduced():
    # same velocity/pressure, forcing with the pressure gradient dropped: must fail to reproduce
    nu = 0.7
    F = fields.poly_k2(nu)
    bad = fields.Field(2, F.u, F.p, lambda x: F.f(x) - np.array([1.0, 1.0]), F.grad_u)
    L = th.THLevel(2, 2, 3, nu, bad)
    x = _direct(L)
    ex, pm = _nodal_exact(L, F)
    d = x - ex
    d[pm] -= d[pm].mean()
    assert np.abs(d[pm]).max() > 1e-3


@pytest.mark.parametrize("k", [2, 3])
def test_convergence_rates(k):
    """Taylor-Hood gives O(h^k) in the velocity H^1 norm and the pressure L^2 norm (Sec. 2)."""
    errs = []
    for n in (4, 8, 16):
        L = th.THLevel(2, k, n, 1.0, fields.baseline_mms(1.0))
        errs.append(norms.errors(L, _direct(L)))
    eu = np.array([e[0] for e in errs]); ep = np.array([e[1] for e in errs])
    ru = np.log2(eu[1] / eu[2]); rp = np.log2(ep[1] / ep[2])
    assert abs(ru - k) <= 0.25
    assert rp >= k - 0.25


# ---------------------------------------------------------------- transfers
@pytest.mark.parametrize("k", [2, 3, 4])
def test_prolongation_reproduces_coarse_fields_and_galerkin(k):
    F = fields.baseline_mms
    Lc = th.THLevel(2, k, 2, 1.0, F(1.0))
    Lf = th.THLevel(2, k, 4, 1.0, F(1.0))
    P = th.prolongation(Lc, Lf)
    # fields of the coarse spaces, interpolated on both levels: prolongation must map one onto
    # the other exactly.  Velocity: the degree-4 bubble (the only polynomial of degree <= k that
    # vanishes on the whole boundary needs k >= 4), else zero.  Pressure: any P_{k-1}.
    bub = lambda X: X[:, 0] * (1 - X[:, 0]) * X[:, 1] * (1 - X[:, 1])
    u = (lambda X: np.stack([bub(X), -2.0 * bub(X)], 1)) if k >= 4 else (lambda X: np.zeros((len(X), 2)))
    p = lambda X: (X[:, 0] - 0.3) ** (k - 1) + X[:, 1] - 0.5 * X[:, 0] * X[:, 1] ** (k - 2)

    def interp(L):
        X, kind = L.dof_coords()
        v = np.zeros(L.N)
        for c in range(2):
            m = kind == c
            v[m] = u(X[m])[:, c]
        m = kind == 2
        v[m] = p(X[m])
        return v

    assert np.abs(P @ interp(Lc) - interp(Lf)).max() <= 1e-12
    # a pressure of one degree too many is not reproduced (catches a wrong pressure degree)
    q = lambda X: X[:, 0] ** k
    Xc, kc = Lc.dof_coords(); Xf, kf = Lf.dof_coords()
    vc = np.where(kc == 2, q(Xc), 0.0); vf = np.where(kf == 2, q(Xf), 0.0)
    assert np.abs(P @ vc - vf).max() > 1e-4
    # constant pressure maps to constant pressure
    zc, zf = Lc.nullvec(), Lf.nullvec()
    ratio = (P @ zc)[Lf.nu_free:] / zf[Lf.nu_free:]
    assert np.allclose(ratio, ratio[0], rtol=1e-13)
    # conforming nested spaces: rediscretisation equals the Galerkin product (Sec. 3)
    G = P.T @ Lf.K @ P - Lc.K
    assert abs(G).max() <= 1e-12 * abs(Lc.K).max()


def test_kuhn_hierarchy_is_nested():
    """Every fine Kuhn tetrahedron lies inside one coarse tetrahedron (P2 nodes included)."""
    Lc = th.THLevel(3, 2, 1, 1.0, fields.poly_3d_k2(1.0))
    Lf = th.THLevel(3, 2, 2, 1.0, fields.poly_3d_k2(1.0))
    P = th.prolongation(Lc, Lf)
    G = P.T @ Lf.K @ P - Lc.K
    assert abs(G).max() <= 1e-12 * abs(Lc.K).max()
