"""Pins for the oracle's patches, smoother, V-cycle and FGMRES (CPU only).

Checked against closed-form patch sizes, brute-force dense operators,
special cases that reduce to textbook methods (block Jacobi, an exact solve),
sparse direct solves, and the paper's h-robustness behaviour.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fgmres, fields, mg, patches, solve, th, vanka


def _level(k, n, nu=1.0):
    return th.THLevel(2, k, n, nu, fields.baseline_mms(nu))


# ---------------------------------------------------------------- patches
@pytest.mark.parametrize("k", [2, 3, 4])
def test_patch_sizes_closed_form(k):
    """Interior vertex patch: hexagon of P_k nodes, 1 + 3k(k+1), times 2, plus one pressure;
    interior edge patch: (k+1)^2 nodes of the two cells, times 2, plus k-2 pressures;
    interior cell patch: (k+1)(k+2)/2 nodes, times 2, plus (k-2)(k-3)/2 pressures."""
    n = 6
    L = _level(k, n)
    P = patches.build_patches(L)
    J = (n + 1) ** 2 + (3 * n * n + 2 * n if k >= 3 else 0) + (2 * n * n if k >= 4 else 0)
    assert len(P) == J
    sizes = [len(I) for I in P]
    vert = 2 * (1 + 3 * k * (k + 1)) + 1
    assert max(sizes) == vert
    # full-size patches: entities whose star closure has no boundary node; for vertices
    # 2 <= i, j <= n-2; for edges and cells, the edges/cells of the inner (n-2)^2 squares
    assert sizes.count(vert) == (n - 3) ** 2
    m = n - 2
    if k >= 3:
        edge = 2 * (k + 1) ** 2 + (k - 2)
        assert sizes.count(edge) == 3 * m * m - 2 * m
    if k >= 4:
        cell = (k + 1) * (k + 2) + (k - 2) * (k - 3) // 2
        assert sizes.count(cell) == 2 * (n - 2) ** 2     # cells with no vertex on the boundary
    # every DoF is covered; pressure DoFs lie in exactly one patch (disjoint pressure partition)
    mult = np.zeros(L.N, dtype=int)
    for I in P:
        assert list(I) == sorted(set(I))
        mult[I] += 1
    assert mult.min() >= 1
    assert np.all(mult[L.nu_free:] == 1)
    # ordering: ascending smallest pressure DoF
    keys = [min(d for d in I if d >= L.nu_free) for I in P]
    assert keys == sorted(keys)


def test_patch_counts_of_p2p1_16():
    L = _level(2, 16)
    P = patches.build_patches(L)
    sizes = [len(I) for I in P]
    assert (len(P), sum(sizes), sum(s * s for s in sizes), max(sizes)) == (289, 9327, 330081, 39)
    hist = {s: sizes.count(s) for s in set(sizes)}
    assert hist == {3: 2, 9: 2, 11: 4, 15: 56, 27: 2, 29: 2, 33: 52, 39: 169}


def test_star_option_vertex_only():
    L = _level(4, 4)
    P = patches.build_patches(L, "star")
    assert len(P) == 25
    # the open star of an interior vertex holds 1 + 6*2 + 6*1 pressure DoFs for P3
    assert max(len(I) for I in P) == 2 * 61 + 1 + 12 + 6


# ---------------------------------------------------------------- patch matrices
def test_patch_matrix_is_brute_force_submatrix_and_translation_invariant():
    L = _level(2, 4)
    S = vanka.AdditiveVanka(L.K, patches.build_patches(L))
    Kd = L.K.toarray()
    X, kind = L.dof_coords()
    interior = []
    for i, I in enumerate(S.patches):
        Ki = S.patch_matrix(i)
        assert np.array_equal(Ki, Kd[np.ix_(I, I)])
        assert np.array_equal(Ki, Ki.T) or np.abs(Ki - Ki.T).max() < 1e-14
        if len(I) == 39:
            interior.append(i)
    # every interior vertex patch of the uniform mesh sees the same matrix (same local geometry)
    ref = S.patch_matrix(interior[0])
    for i in interior[1:]:
        assert np.abs(S.patch_matrix(i) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_patch_inverses():
    L = _level(4, 2)
    S = vanka.AdditiveVanka(L.K, patches.build_patches(L))
    for i, I in enumerate(S.patches):
        Ki = S.patch_matrix(i)
        Kinv = sla.lu_solve(S.lu[i], np.eye(len(I)))
        c = np.linalg.cond(Ki)
        assert np.abs(Ki @ Kinv - np.eye(len(I))).max() <= 50 * len(I) * np.finfo(float).eps * c
        assert np.abs(Kinv - Kinv.T).max() <= 50 * len(I) * np.finfo(float).eps * c * np.abs(Kinv).max()


# ---------------------------------------------------------------- smoother
def test_sweep_equals_dense_operator():
    L = _level(2, 4)
    S = vanka.AdditiveVanka(L.K, patches.build_patches(L), omega=0.5)
    M = S.dense_operator()
    rng = np.random.default_rng(1)
    b, x = rng.standard_normal(L.N), rng.standard_normal(L.N)
    ref = x + 0.5 * (M @ (b - L.K.toarray() @ x)) / S.mult
    assert np.abs(S.sweep(b, x) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_disjoint_patches_reduce_to_block_jacobi():
    rng = np.random.default_rng(2)
    N = 40
    A = rng.standard_normal((N, N)); A = A + A.T + 2 * N * np.eye(N)
    K = sp.csr_matrix(A)
    blocks = [list(range(0, 7)), list(range(7, 20)), list(range(20, 40))]
    S = vanka.AdditiveVanka(K, blocks, omega=1.0)
    b, x = rng.standard_normal(N), rng.standard_normal(N)
    D = np.zeros_like(A)
    for I in blocks:
        D[np.ix_(I, I)] = A[np.ix_(I, I)]
    ref = x + np.linalg.solve(D, b - A @ x)
    assert np.abs(S.sweep(b, x) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_single_patch_without_one_pressure_solves_exactly():
    """One patch with every DoF except the last pressure, omega = 1, no weights: the sweep from
    x = 0 is an exact solve, up to the constant pressure (the dropped DoF pins it to zero)."""
    L = _level(2, 3)
    N = L.N
    rng = np.random.default_rng(3)
    xs = rng.standard_normal(N)
    b = L.K @ xs
    S = vanka.AdditiveVanka(L.K, [list(range(N - 1))], omega=1.0, weighting="none")
    x = S.sweep(b, np.zeros(N))
    d = x - xs
    assert np.abs(d[: L.nu_free]).max() <= 1e-9
    assert np.abs(d[L.nu_free:] + xs[N - 1]).max() <= 1e-9


def test_unweighted_sum_is_not_a_contraction_but_weighted_is():
    """Records the reading of Algorithm 1's weights: with w_i = identity and omega = 0.5 the
    P2-P1 vertex-patch sweep has spectral radius > 1; with multiplicity weights it is < 1 on
    the complement of the constant-pressure kernel."""
    L = _level(2, 4)
    P = patches.build_patches(L)
    K = L.K.toarray()
    for weighting, expect_bad in (("none", True), ("multiplicity", False)):
        S = vanka.AdditiveVanka(L.K, P, omega=0.5, weighting=weighting)
        E = np.eye(L.N) - 0.5 * (S.weight[:, None] * S.dense_operator()) @ K
        ev = np.abs(np.linalg.eigvals(E))
        ev = np.sort(ev)[:-1]      # the kernel mode (eigenvalue exactly 1) is excluded
        assert (ev.max() > 1.5) == expect_bad


# ---------------------------------------------------------------- V-cycle
def test_vcycle_is_linear_and_two_level_without_smoothing_is_coarse_correction():
    H = th.THHierarchy(2, 2, 2, 2, 1.0, fields.baseline_mms)
    V = mg.VCycle(H, nu_pre=2, nu_post=2)
    rng = np.random.default_rng(4)
    N = H.finest.N
    r1, r2 = rng.standard_normal(N), rng.standard_normal(N)
    lhs = V.apply(2.0 * r1 - 3.0 * r2)
    rhs = 2.0 * V.apply(r1) - 3.0 * V.apply(r2)
    assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(lhs).max()
    V0 = mg.VCycle(H, nu_pre=0, nu_post=0)
    Lc = H.levels[0]
    z = Lc.nullvec()
    Kb = np.block([[Lc.K.toarray(), z[:, None]], [z[None, :], np.zeros((1, 1))]])
    P = H.P[1].toarray()
    ec = np.linalg.solve(Kb, np.concatenate([P.T @ r1, [0.0]]))[:-1]
    assert np.abs(V0.apply(r1) - P @ ec).max() <= 1e-11 * np.abs(P @ ec).max()


# ---------------------------------------------------------------- FGMRES
def test_fgmres_textbook_properties():
    """Identity preconditioner: full GMRES on an n x n system converges in <= n steps, and the
    Givens estimate equals the true residual of each iterate (monotone)."""
    rng = np.random.default_rng(5)
    n = 25
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    b = rng.standard_normal(n)
    x, its, hist, conv = fgmres.fgmres(sp.csr_matrix(A), b, lambda v: v, restart=n, rtol=1e-12, maxit=n)
    assert conv and its <= n
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.01
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))
    # restarted variant reaches the same solution
    x2, its2, _, conv2 = fgmres.fgmres(sp.csr_matrix(A), b, lambda v: v, restart=5, rtol=1e-12, maxit=500)
    assert conv2 and np.abs(x2 - np.linalg.solve(A, b)).max() <= 1e-10


def test_fgmres_multigrid_matches_direct_solve():
    H, V = solve.setup(2, 2, 4, 2, 1.0, fields.baseline_mms)
    L = H.finest
    x, its, hist, conv = solve.solve(H, V)
    assert conv and its <= 30
    z = L.nullvec()
    b = solve.consistent_rhs(L)
    Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    xd = spla.spsolve(Kb, np.concatenate([b, [0.0]]))[: L.N]
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert abs(z @ x) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.slow
def test_iterations_are_h_robust():
    """Iteration counts barely change under refinement (Sec. 4.1, nu > 1)."""
    its = []
    for nl in (3, 4):
        H, V = solve.setup(2, 2, 4, nl, 1.0, fields.baseline_mms)
        its.append(solve.solve(H, V)[1])
    assert abs(its[1] - its[0]) <= 2
    assert max(its) <= 20
