"""Pins for the oracle's Scott-Vogelius (P3, dP2) discretisation on barycentric meshes (CPU only).

Checked against closed-form counts, exact reproduction of a polynomial
solution, third-order convergence, the pointwise divergence-free velocity
and the invariance of the velocity under gradient forcing that the
pressure-robust pair must show (Sec. 2), a one-dimensional kernel by dense
SVD, the transfers on fields they must reproduce, brute-force integration of
the L^2 pressure projection, and the solver against a direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import fields, mg, patches, quad, solve, sv
from oracle.vanka import AdditiveVanka


def _direct(L):
    z = L.nullvec()
    b = solve.consistent_rhs(L)
    Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[: L.N]


# ---------------------------------------------------------------- counts
@pytest.mark.parametrize("n", [2, 4, 8])
def test_counts_closed_form(n):
    # P3 nodes of the barycentric refinement: (n+1)^2 + 2n^2 vertices, 9n^2 + 2n edges (2 nodes
    # each), 6n^2 sub-cells (1 node each) -> 27n^2 + 6n + 1; 12n of them on the boundary.
    # dP2 pressure: 6 per sub-cell -> 36 n^2.
    L = sv.SVLevel(3, n, 1.0, fields.baseline_mms(1.0))
    assert L.n_vel_nodes_all == 27 * n * n + 6 * n + 1
    assert L.nu_free == 2 * (27 * n * n - 6 * n + 1)
    assert L.np_ == 36 * n * n
    assert L.N == 90 * n * n - 12 * n + 2
    P = patches.build_patches(L, "macro")
    assert len(P) == 2 * n * n
    sizes = np.array([len(I) for I in P])
    # a macro triangle with no vertex on the boundary (2 (n-2)^2 of them): 18 pressure + 2 x 19
    # velocity; every other patch loses boundary velocity nodes
    assert np.sum(sizes == 56) == 2 * (n - 2) ** 2
    assert np.all(sizes <= 56) and np.all(sizes >= 18)


def test_counts_of_the_finest_levels():
    # the hierarchy of the 64 x 64 workload, levels 4 .. 16 (larger ones follow the closed form)
    want = {4: (1394, 43988, 32, 1644, 85000), 8: (5666, 191924, 128, 6860, 369224),
            16: (22850, 802292, 512, 28044, 1539784)}
    for n, (N, nnz, J, sn, sn2) in want.items():
        L = sv.SVLevel(3, n, 1.0, fields.baseline_mms(1.0))
        P = patches.build_patches(L, "macro")
        assert (L.N, L.K.nnz, len(P), sum(map(len, P)), sum(len(I) ** 2 for I in P)) == (N, nnz, J, sn, sn2)


def test_macro_patch_contents():
    L = sv.SVLevel(3, 3, 1.0, fields.baseline_mms(1.0))
    P = patches.build_patches(L, "macro")
    owner = np.full(L.N, -1)
    for i, I in enumerate(P):
        assert list(I) == sorted(set(I))
        pres = [d for d in I if d >= L.nu_free]
        # the 18 pressure DoFs of macro triangle i, each in exactly one patch
        assert pres == list(range(L.nu_free + 18 * i, L.nu_free + 18 * i + 18))
        assert np.all(owner[pres] == -1)
        owner[pres] = i
    assert np.all(owner[L.nu_free:] >= 0)


# ---------------------------------------------------------------- discretisation
@pytest.mark.parametrize("nu", [1.0, 0.37])
def test_polynomial_solution_reproduced_exactly(nu):
    L = sv.SVLevel(3, 3, nu, fields.poly_k3(nu))
    x = _direct(L)
    ev, ep, div = sv.errors(L, x)
    assert ev <= 1e-10 and ep <= 1e-10 and div <= 1e-10
    X, kind = L.dof_coords()
    vel = kind < 2
    assert np.abs(x[vel] - fields.poly_k3(nu).u(X[vel])[np.arange(vel.sum()), kind[vel]]).max() <= 1e-11


def test_wrong_forcing_is_not_reproduced():
    nu = 1.0
    good = fields.poly_k3(nu)
    bad = fields.Field(2, good.u, good.p, lambda x: good.f(x) * 1.01, good.grad_u)
    L = sv.SVLevel(3, 3, nu, bad)
    assert sv.errors(L, _direct(L))[0] > 1e-6


def test_third_order_convergence_and_divergence_free_velocity():
    errs = []
    for n in (2, 4, 8):
        L = sv.SVLevel(3, n, 1.0, fields.baseline_mms(1.0))
        ev, ep, div = sv.errors(L, _direct(L))
        errs.append((ev, ep))
        assert div <= 1e-9          # div V_h lies in Q_h, so the discrete velocity is pointwise div-free
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(np.abs(rates - 3.0) <= 0.25), rates


def test_velocity_invariant_under_gradient_forcing():
    """Pressure robustness: f -> f + grad psi changes only the pressure (psi of degree 5, not in dP2;
    the load integrands stay within the rule's exact degree)."""
    base = fields.baseline_mms(1.0)
    psi = lambda x: 5 * x[:, 0] ** 4 * x[:, 1] - 2 * x[:, 0] * x[:, 1] ** 3
    gpsi = lambda x: np.stack([20 * x[:, 0] ** 3 * x[:, 1] - 2 * x[:, 1] ** 3,
                               5 * x[:, 0] ** 4 - 6 * x[:, 0] * x[:, 1] ** 2], 1)
    L0 = sv.SVLevel(3, 4, 1.0, base)
    L1 = sv.SVLevel(3, 4, 1.0, fields.with_gradient(base, psi, gpsi))
    x0, x1 = _direct(L0), _direct(L1)
    nv = L0.nu_free
    assert np.abs(x0[:nv] - x1[:nv]).max() <= 1e-10 * np.abs(x0[:nv]).max()
    assert np.abs(x0[nv:] - x1[nv:]).max() > 1e-3        # the pressure does move
    # Taylor-Hood on the same macro mesh is not pressure-robust: its velocity moves
    from oracle import th
    T0 = th.THLevel(2, 3, 4, 1.0, base)
    T1 = th.THLevel(2, 3, 4, 1.0, fields.with_gradient(base, psi, gpsi))
    t0, t1 = _direct(T0), _direct(T1)
    assert np.abs(t0[:T0.nu_free] - t1[:T0.nu_free]).max() > 1e-8


def test_kernel_is_the_constant_pressure():
    L = sv.SVLevel(3, 2, 1.0, fields.baseline_mms(1.0))
    K = L.K.toarray()
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    s = np.linalg.svd(K, compute_uv=False)
    assert np.sum(s < 1e-10 * s[0]) == 1
    assert np.abs(K @ L.nullvec()).max() <= 1e-13 * np.abs(K).max()


# ---------------------------------------------------------------- transfers
@pytest.fixture(scope="module")
def pair():
    return sv.SVLevel(3, 2, 1.0, fields.baseline_mms(1.0)), sv.SVLevel(3, 4, 1.0, fields.baseline_mms(1.0))


def test_velocity_transfer_reproduces_cubics_away_from_the_boundary():
    C, F = sv.SVLevel(3, 4, 1.0, fields.baseline_mms(1.0)), sv.SVLevel(3, 8, 1.0, fields.baseline_mms(1.0))
    P = sv.prolongation(C, F)
    q = lambda x: np.stack([x[:, 0] ** 3 - 2 * x[:, 0] * x[:, 1] ** 2 + 0.5, x[:, 1] ** 3 + x[:, 0] * x[:, 1]], 1)
    XC, kc = C.dof_coords()
    XF, kf = F.dof_coords()
    ec = np.zeros(C.N)
    vc = kc < 2
    ec[vc] = q(XC[vc])[np.arange(vc.sum()), kc[vc]]
    ef = P @ ec
    vf = kf < 2
    away = vf & np.all((XF > 1.0 / C.n + 1e-12) & (XF < 1.0 - 1.0 / C.n - 1e-12), axis=1)
    assert away.sum() > 0
    want = q(XF[away])[np.arange(away.sum()), kf[away]]
    assert np.abs(ef[away] - want).max() <= 1e-12


def test_pressure_transfer_reproduces_global_quadratics(pair):
    C, F = pair
    P = sv.prolongation(C, F)
    q = lambda x: 1.0 + 2 * x[:, 0] - x[:, 1] + 3 * x[:, 0] * x[:, 1] - x[:, 1] ** 2
    XC, kc = C.dof_coords()
    XF, kf = F.dof_coords()
    ec = np.where(kc == 2, q(XC), 0.0)
    ef = P @ ec
    assert np.abs(ef[kf == 2] - q(XF[kf == 2])).max() <= 1e-12
    one = np.where(kc == 2, 1.0, 0.0)
    assert np.abs((P @ one)[kf == 2] - 1.0).max() <= 1e-13


def test_clipping_against_grid_counting():
    rng = np.random.default_rng(3)
    for _ in range(20):
        A = rng.random((3, 2))
        B = rng.random((3, 2))
        poly = sv._clip([a for a in A], [b for b in B])
        got = sv._area(poly) if len(poly) >= 3 else 0.0
        m = 600
        g = (np.arange(m) + 0.5) / m
        X, Y = np.meshgrid(g, g)
        pts = np.stack([X.ravel(), Y.ravel()], 1)

        def inside(T, p):
            s = []
            for e in range(3):
                a, b = T[e], T[(e + 1) % 3]
                s.append((b[0] - a[0]) * (p[:, 1] - a[1]) - (b[1] - a[1]) * (p[:, 0] - a[0]))
            s = np.stack(s, 1)
            return np.all(s >= 0, 1) | np.all(s <= 0, 1)
        est = np.mean(inside(A, pts) & inside(B, pts))
        assert abs(got - est) <= 6.0 / m, (got, est)


def test_pressure_projection_against_brute_force_subdivision(pair):
    """Fine sub-cells that straddle coarse sub-cells: integrate coarse x fine basis over a uniform
    m x m subdivision of the fine sub-cell, each small triangle given to the coarse sub-cell of its
    centroid.  Small triangles whose vertices lie in different coarse sub-cells bound the error."""
    C, F = pair
    P = sv.prolongation(C, F).tocsr()
    qp, qw = quad.simplex_rule(2, 4)
    rng = np.random.default_rng(5)
    pc = rng.standard_normal(C.N)
    pc[: C.nu_free] = 0.0
    m = 24
    checked = straddling = 0
    for fc in range(len(F.cells)):
        cell = F.cells[fc]
        V = np.array(cell, dtype=float) / F.n3
        cand = sv._coarse_candidates(C, V.mean(0)[None, :])[0]

        def coarse_val(p):
            for cc in cand:
                lam, xi = sv._bary(C.cells[cc], p[None, :], C.n3)
                if lam.min() >= -1e-12:
                    return cc, C.pb.eval(xi)[0] @ pc[C.cell_pdofs(cc)]
            raise AssertionError

        G = np.zeros(F.nbp)
        cut = 0.0
        owners = set()
        E1, E2 = V[1] - V[0], V[2] - V[0]
        for i in range(m):
            for j in range(m - i):
                tris = [((i, j), (i + 1, j), (i, j + 1))]
                if i + j < m - 1:
                    tris.append(((i + 1, j + 1), (i, j + 1), (i + 1, j)))
                for t in tris:
                    P3 = np.array([V[0] + (a * E1 + b * E2) / m for a, b in t])
                    cc = coarse_val(P3.mean(0))[0]
                    owners.add(cc)
                    Jt = np.stack([P3[1] - P3[0], P3[2] - P3[0]], 1)
                    w = qw * abs(np.linalg.det(Jt))
                    x = P3[0][None, :] + qp @ Jt.T
                    _, xic = sv._bary(C.cells[cc], x, C.n3)
                    vals = C.pb.eval(xic) @ pc[C.cell_pdofs(cc)]
                    _, xif = sv._bary(cell, x, F.n3)
                    G += np.einsum("q,qa,q->a", w, F.pb.eval(xif), vals)
                    if len({coarse_val(v)[0] for v in P3}) > 1 or cc != coarse_val(P3[0])[0]:
                        cut += w.sum()
        _, Jf = F.cell_geometry(cell)
        Mf = np.einsum("q,qa,qb->ab", qw * abs(np.linalg.det(Jf)), F.pb.eval(qp), F.pb.eval(qp))
        exact_G = Mf @ (P[F.cell_pdofs(fc)] @ pc)
        # on a small triangle given to the wrong coarse sub-cell the integrand errs by at most
        # max|psi_a| (<= 1.5 for the P2 basis on the triangle, attained bound checked below) times
        # the sum of the two coarse polynomials' magnitudes there
        vmax = 2 * max(abs(C.pb.eval(sv._bary(C.cells[c], V, C.n3)[1]) @ pc[C.cell_pdofs(c)]).max()
                       for c in cand) + 1.0
        assert np.abs(F.pb.eval(qp)).max() <= 1.5
        if cut == 0.0:
            assert np.abs(G - exact_G).max() <= 1e-12 * np.abs(exact_G).max()
        else:
            assert np.abs(G - exact_G).max() <= 1.5 * cut * vmax * 10, (fc, G, exact_G, cut)
            assert np.abs(G - exact_G).max() <= 0.05 * np.abs(exact_G).max()
        checked += 1
        straddling += len(owners) > 1
        if straddling >= 3:
            break
    assert straddling >= 3


# ---------------------------------------------------------------- smoother and solver
def test_macro_sweep_equals_dense_operator():
    L = sv.SVLevel(3, 2, 1.0, fields.baseline_mms(1.0))
    S = AdditiveVanka(L.K, patches.build_patches(L, "macro"), 0.5)
    M = S.dense_operator()
    b = synth.vector(L.N, 11)
    x = synth.vector(L.N, 12)
    want = x + 0.5 * S.weight * (M @ (b - L.K @ x))
    assert np.abs(S.sweep(b, x) - want).max() <= 1e-12 * np.abs(want).max()


def test_vcycle_linear_and_solver_matches_direct():
    H, V = solve.setup(2, 3, 2, 2, 1.0, fields.baseline_mms, family="sv")
    L = H.finest
    u, v = synth.vector(L.N, 21), synth.vector(L.N, 22)
    # linear (the multiplicity weights act from the left, so B is not symmetric)
    Bu, Bv, Bw = V.apply(u), V.apply(v), V.apply(2.5 * u - v)
    assert np.abs(Bw - (2.5 * Bu - Bv)).max() <= 1e-11 * np.abs(Bw).max()
    x, its, hist, conv = solve.solve(H, V)
    xd = _direct(L)
    b = solve.consistent_rhs(L)
    assert conv and np.linalg.norm(b - L.K @ x) <= 1.05e-10 * np.linalg.norm(b)
    # forward error within the condition number on the range of K (kernel: the constant pressure)
    s = np.linalg.svd(L.K.toarray(), compute_uv=False)
    kappa = s[0] / s[-2]
    assert np.linalg.norm(x - xd) <= kappa * 1.05e-10 * np.linalg.norm(xd)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)


def test_iterations_are_h_robust():
    counts = []
    for nl in (2, 3):
        H, V = solve.setup(2, 3, 4, nl, 1.0, fields.baseline_mms, family="sv")
        x, its, hist, conv = solve.solve(H, V)
        assert conv
        counts.append(its)
    assert counts[1] - counts[0] <= 2 and counts[1] <= 30, counts
