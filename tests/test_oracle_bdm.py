"""Pins for the (BDM_k, dP_{k-1}) interior-penalty oracle (CPU only).

Checked against what the mathematics fixes rather than against the oracle's own
formulas: the normal continuity of the glued dual basis, exact reproduction of vector
polynomials of degree k by the DoF functionals, the strain identity of the
interior-penalty form for a continuous polynomial field (volume and consistency
terms), symmetry and coercivity, an exactly divergence-free discrete velocity,
exact transfer of coarse polynomials (nested spaces), the O(h^k) convergence of the
manufactured solution, patch bookkeeping and the multigrid solve against a direct solve.
The penalty threshold test pins the default alpha against the coercivity limit.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as leg

from oracle import bdm, fields, lagrange, quad, solve


def interpolant(L, w, q=None):
    """Free-DoF vector of the BDM interpolant of the field w (the DoF functionals written out)."""
    k = L.k
    x = np.zeros(L.N)
    g, gw = np.polynomial.legendre.leggauss(k + 3)
    g, gw = 0.5 * (g + 1), 0.5 * gw
    for e, r in L.edge_rank.items():
        a, b = (np.array(v, dtype=float) / L.n for v in e)
        t = (b - a) / np.linalg.norm(b - a)
        nrm = np.array([t[1], -t[0]])
        pts = a + g[:, None] * (b - a)
        for j in range(k + 1):
            c = np.zeros(j + 1); c[j] = 1.0
            x[r * (k + 1) + j] = gw @ ((w(pts) @ nrm) * leg.legval(2 * g - 1, c))
    qp, qw = quad.simplex_rule(2, k + 3)
    for ci, cell in enumerate(L.cells):
        v0, J = L.cell_geometry(cell)
        pts = v0 + qp @ J.T
        xc = v0 + J @ np.array([1.0, 1.0]) / 3
        xi = (pts - xc) * L.n
        qs = []
        if k >= 2:
            # nodal P_{k-2} basis in reference coordinates (brute-force Vandermonde solve)
            lat = lagrange.lattice_nodes(2, k - 2) if k > 2 else [(0, 0)]
            nodes = np.array(lat, float) / max(k - 2, 1)
            ex = lagrange.monomial_exponents(2, k - 2)
            V = np.array([[X ** a * Y ** b for a, b in ex] for X, Y in nodes])
            Vq = np.array([[X ** a * Y ** b for a, b in ex] for X, Y in qp])
            La = Vq @ np.linalg.inv(V)                          # (np, nnodes)
            for c in range(2):
                for m in range(len(lat)):
                    v = np.zeros_like(xi); v[:, c] = La[:, m]
                    qs.append(v)
            for m, a in enumerate(lat):
                if sum(a) == k - 2:
                    qs.append(np.stack([-xi[:, 1] * La[:, m], xi[:, 0] * La[:, m]], 1))
        if not qs:
            continue
        # orthonormalise in order (Gram-Schmidt = QR with a positive diagonal), inner product |T|^-1 int_T
        Qr = np.stack(qs, 1)                                   # (np, ni, 2)
        sw = np.sqrt(2 * qw)
        M = (sw[:, None, None] * Qr).transpose(0, 2, 1).reshape(-1, len(qs))
        _, R = np.linalg.qr(M)
        R = R * np.sign(np.diag(R))[:, None]
        Qo = np.einsum("pmc,mi->pic", Qr, np.linalg.inv(R))
        vals = np.array([2 * qw @ np.sum(w(pts) * Qo[:, i, :], 1) for i in range(len(qs))])
        base = L.nu_edges + ci * L.ni_loc
        x[base:base + L.ni_loc] = vals
    if q is not None:
        for ci, cell in enumerate(L.cells):
            v0, J = L.cell_geometry(cell)
            kk = k - 1
            nodes = L.pb.lattice()
            pts = np.array([v0 + J @ np.array(a, float) / kk for a in nodes]) if kk >= 1 else \
                (v0 + J @ np.array([1.0, 1.0]) / 3)[None, :]
            x[L.cell_pdofs(ci)] = q(pts)
    return x


def poly_field(k):
    """A vector field of degree k with w.n = 0 on the boundary and eps_xy = 0 everywhere."""
    def w(X):
        x, y = X[:, 0], X[:, 1]
        return np.stack([x * (1 - x) * (1 + 0.5 * x ** (k - 2)), y * (1 - y) * (2 - y ** (k - 2))], 1)
    return w


def hw(L, w, q=None):
    return interpolant(L, w, q)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_basis_is_normal_continuous_and_reproduces_polynomials(k):
    L = bdm.BDMLevel(k, 3, 1.0, fields.paper_mms(1.0))
    rng = np.random.default_rng(k)
    # normal component of each edge basis function agrees from both sides of its edge
    g = np.linspace(0.05, 0.95, 7)
    for e in L.interior_edges[::3]:
        a, b, Le, t, ne = L.edge_frame(e)
        pts = a + g[:, None] * (b - a)
        T1, T2 = L.edge_cells[e]
        P1, _ = L.phi(T1, pts)
        P2, _ = L.phi(T2, pts)
        d1, d2 = L.cell_vel_dofs(T1), L.cell_vel_dofs(T2)
        for i, d in enumerate(d1):
            if d < 0:
                continue
            j = np.flatnonzero(d2 == d)
            other = P2[:, j[0], :] @ ne if len(j) else np.zeros(len(g))
            assert np.abs(P1[:, i, :] @ ne - other).max() <= 1e-10
    # a random vector polynomial of degree k is reproduced on every cell by its interpolant
    C = rng.standard_normal((2, k + 1, k + 1))
    def w(X):
        out = np.zeros((len(X), 2))
        for c in range(2):
            for a in range(k + 1):
                for bb in range(k + 1 - a):
                    out[:, c] += C[c, a, bb] * X[:, 0] ** a * X[:, 1] ** bb
        return out
    # the boundary normal trace is not zero here, so compare on cells whose edges are all interior
    xv = hw(L, w)
    qp, _ = quad.simplex_rule(2, 4)
    for ci, cell in enumerate(L.cells):
        if np.any(L.cell_vel_dofs(ci) < 0):
            continue
        v0, J = L.cell_geometry(cell)
        pts = v0 + qp @ J.T
        uh, _ = L.velocity(ci, xv, pts)
        assert np.abs(uh - w(pts)).max() <= 1e-9 * max(1.0, np.abs(w(pts)).max())


@pytest.mark.parametrize("k", [2, 3, 4])
def test_strain_identity_for_a_continuous_polynomial(k):
    nu = 0.7
    w = poly_field(k)
    # w = (f1(x), f2(y)): eps = diag(f1', f2'), so -div(2 nu eps(w)) = -2 nu (f1'', f2'')
    def f(X):
        x, y = X[:, 0], X[:, 1]
        # f1 = x (1 - x)(1 + x^(k-2)/2) = x - x^2 + (x^(k-1) - x^k)/2
        d2f1 = -2.0 + 0.5 * ((k - 1) * (k - 2) * x ** max(k - 3, 0) - k * (k - 1) * x ** (k - 2))
        # f2 = y (1 - y)(2 - y^(k-2)) = 2 y - 2 y^2 - y^(k-1) + y^k
        d2f2 = -4.0 - (k - 1) * (k - 2) * y ** max(k - 3, 0) + k * (k - 1) * y ** (k - 2)
        return -2.0 * nu * np.stack([d2f1, d2f2], 1)
    F = fields.Field(2, w, lambda X: np.zeros(len(X)), f, None)
    L = bdm.BDMLevel(k, 4, nu, F)
    x = hw(L, w)
    A = L.K[:L.nu_free, :L.nu_free]
    r = A @ x[:L.nu_free] - L.b[:L.nu_free]
    assert np.abs(r).max() <= 1e-12 * (abs(A) @ np.abs(x[:L.nu_free])).max()
    # the edge consistency term is what makes it hold: the volume part alone does not
    rows, cols, vals = [], [], []
    for ci in range(len(L.cells)):
        Ae = L.element_matrices(ci)[0]
        vd = L.cell_vel_dofs(ci)
        f = vd >= 0
        rr, cc = np.meshgrid(vd[f], vd[f], indexing="ij")
        rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(Ae[np.ix_(f, f)].ravel())
    Avol = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(L.nu_free, L.nu_free)).tocsr()
    assert np.abs(Avol @ x[:L.nu_free] - L.b[:L.nu_free]).max() > 1e-3 * np.abs(L.b[:L.nu_free]).max()


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_symmetric_coercive_and_pressure_kernel(k):
    L = bdm.BDMLevel(k, 2, 1.3, fields.paper_mms(1.3))
    K = L.K
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    A = K[:L.nu_free, :L.nu_free].toarray()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > 1e-6 * ev.max()
    assert np.abs(K @ L.nullvec()).max() <= 1e-11 * abs(K).max()
    z = L.nullvec()
    Kb = np.block([[K.toarray(), z[:, None]], [z[None, :], np.zeros((1, 1))]])
    assert np.linalg.cond(Kb) < 1e13


def direct(L, b=None):
    z = L.nullvec()
    b = solve.consistent_rhs(L, b)
    Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:L.N]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_discrete_velocity_is_divergence_free(k):
    L = bdm.BDMLevel(k, 4, 1.0, fields.paper_mms(1.0))
    x = direct(L)
    qp, _ = quad.simplex_rule(2, 3)
    worst = 0.0
    for ci, cell in enumerate(L.cells):
        v0, J = L.cell_geometry(cell)
        _, G = L.velocity(ci, x, v0 + qp @ J.T)
        worst = max(worst, np.abs(G[:, 0, 0] + G[:, 1, 1]).max())
    assert worst <= 1e-9


@pytest.mark.parametrize("k", [1, 2, 3])
def test_prolongation_is_exact_on_coarse_polynomials(k):
    H = bdm.BDMHierarchy(k, 2, 2, 1.0, fields.paper_mms)
    C, Fi = H.levels
    w = poly_field(max(k, 2)) if k >= 2 else (lambda X: np.stack([X[:, 0] * 0 + 0.0, X[:, 1] * 0.0], 1))
    q = lambda X: (X[:, 0] + 0.3) ** (k - 1) - 0.2 * X[:, 1] ** (k - 1) + (0.1 * X[:, 0] * X[:, 1] ** (k - 2) if k >= 2 else 0.0)
    if k == 1:
        # BDM_1: the field must be in P_1 with w.n = 0 on the boundary: only zero; use the pressure part
        w = lambda X: np.zeros((len(X), 2))
    xc, xf = hw(C, w, q), hw(Fi, w, q)
    assert np.abs(H.P[1] @ xc - xf).max() <= 1e-11
    # the restriction of a fine random vector is the transpose action
    rng = np.random.default_rng(1)
    r = rng.standard_normal(Fi.N)
    assert np.allclose(H.P[1].T @ r, (r @ H.P[1]))


def test_converges_at_order_k():
    for k in (2, 3):
        errs = []
        for n in (2, 4, 8):
            L = bdm.BDMLevel(k, n, 1.0, fields.paper_mms(1.0))
            errs.append(bdm.errors(L, direct(L)))
        ru = math.log2(errs[1][0] / errs[2][0])
        rp = math.log2(errs[1][1] / errs[2][1])
        assert abs(ru - k) <= 0.25, (k, errs)
        assert rp >= k - 0.5, (k, errs)


@pytest.mark.parametrize("k,n", [(1, 3), (2, 4), (3, 3)])
def test_extended_patches(k, n):
    L = bdm.BDMLevel(k, n, 1.0, fields.paper_mms(1.0))
    P = bdm.build_patches(L)
    assert len(P) == len(L.cells)
    pres = np.concatenate([[d for d in I if d >= L.nu_free] for I in P])
    assert np.array_equal(np.sort(pres), np.arange(L.nu_free, L.N))
    full = 4 * (k * k - 1) + 9 * (k + 1) + k * (k + 1) // 2
    assert max(len(I) for I in P) == full
    # every free velocity DoF is in some patch
    vel = set()
    for I in P:
        vel.update(d for d in I if d < L.nu_free)
        assert list(I) == sorted(I)
    assert vel == set(range(L.nu_free))


def test_multigrid_solve_matches_direct_and_is_h_robust():
    counts = []
    for nl in (2, 3):
        H, V = solve.setup(2, 2, 2, nl, 1.0, fields.paper_mms, family="bdm")
        x, its, hist, conv = solve.solve(H, V)
        assert conv
        counts.append(its)
    L = H.finest
    xd = direct(L)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    # extended patches keep the counts low and slowly varying in h (Sec. 4.3)
    assert max(counts) <= 30 and counts[1] - counts[0] <= 5, counts


def test_default_penalty_is_coercive_with_margin():
    # the smallest coercive alpha, found by bisection on the smallest eigenvalue of the velocity block,
    # stays below half the default at every order
    for k in (1, 2, 4):
        L0 = bdm.BDMLevel(k, 3, 1.0, fields.paper_mms(1.0), alpha=0.0)
        L1 = bdm.BDMLevel(k, 3, 1.0, fields.paper_mms(1.0), alpha=1.0)
        A0 = L0.K[:L0.nu_free, :L0.nu_free].toarray()
        Pen = L1.K[:L1.nu_free, :L1.nu_free].toarray() - A0
        half = 0.5 * bdm.default_alpha(k)
        assert np.linalg.eigvalsh(A0 + half * Pen).min() > 0
        # and with no penalty the form is indefinite (the consistency terms alone are not coercive)
        assert np.linalg.eigvalsh(A0).min() < 0
