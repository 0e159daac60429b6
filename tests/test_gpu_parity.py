"""GPU parity: the HIP path (through the C ABI) against the oracle.

Every stage is compared element by element on the same seeded inputs:
SpMV, transfers, patch gather, patch inverses, one smoothing sweep, the
coarsest solve, one V-cycle and the full FGMRES solve.  Tolerances follow
from the arithmetic: the GPU applies explicit patch inverses (Gauss-Jordan)
where the oracle uses LU solves, so patch-level differences scale with
n * eps * cond(K_i); everything else is a handful of roundings.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle_history
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def p2p1():
    """P2-P1 on 16x16, levels 4/8/16 (the small workload)."""
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print("[gpu] building P2-P1 16x16 hierarchy", flush=True)
    H = vk.Hierarchy(2, 4, 3).bind().setup()
    OH, OV = solve.setup(2, 2, 4, 3, 1.0, fields.baseline_mms)
    return H, OH, OV


@pytest.fixture(scope="module")
def p4p3():
    """P4-P3 on 16x16, levels 4/8/16: several patch size classes up to 123."""
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print("[gpu] building P4-P3 16x16 hierarchy", flush=True)
    H = vk.Hierarchy(4, 4, 3).bind().setup()
    OH, OV = solve.setup(2, 4, 4, 3, 1.0, fields.baseline_mms)
    return H, OH, OV


@pytest.fixture(scope="module")
def p2p1_3d():
    """3D P2-P1 on Kuhn tetrahedra, levels 2/4/8 cubes per direction (vertex patches up to 196)."""
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print("[gpu] building 3D P2-P1 8^3 hierarchy", flush=True)
    H = vk.Hierarchy(2, 2, 3, dim=3, forcing=vk.VK_F_CUBE_MMS).bind().setup()
    OH, OV = solve.setup(3, 2, 2, 3, 1.0, fields.cube_mms)
    return H, OH, OV


@pytest.fixture(scope="module")
def p3dp2_sv():
    """Scott-Vogelius P3-dP2 on barycentric refinements of 4x4/8x8/16x16: non-nested transfers,
    56-DoF macro patches."""
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print("[gpu] building SV P3-dP2 16x16 hierarchy", flush=True)
    H = vk.Hierarchy(3, 4, 3, family=vk.VK_SV).bind().setup()
    OH, OV = solve.setup(2, 3, 4, 3, 1.0, fields.baseline_mms, family="sv")
    return H, OH, OV


@pytest.fixture(scope="module")
def p8p7():
    """P8-P7 on 4x4, levels 2/4: interior vertex patches of 435 DoFs (inverted blocked in global
    memory, stored column-major)."""
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print("[gpu] building P8-P7 4x4 hierarchy", flush=True)
    H = vk.Hierarchy(8, 2, 2, forcing=vk.VK_F_PAPER_MMS).bind().setup()
    OH, OV = solve.setup(2, 8, 2, 2, 1.0, fields.paper_mms)
    return H, OH, OV


@pytest.fixture(scope="module")
def p6p5():
    """P6-P5 on 8x8, levels 2/4/8: vertex patches of 255 DoFs on two levels."""
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print("[gpu] building P6-P5 8x8 hierarchy", flush=True)
    H = vk.Hierarchy(6, 2, 3).bind().setup()
    OH, OV = solve.setup(2, 6, 2, 3, 1.0, fields.baseline_mms)
    return H, OH, OV


def _quad_fixture(k, n0, nl):
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print(f"[gpu] building Q{k}-Q{k - 1} {n0 << (nl - 1)}x{n0 << (nl - 1)} hierarchy", flush=True)
    H = vk.Hierarchy(k, n0, nl, family=vk.VK_TH_QUAD).bind().setup()
    OH, OV = solve.setup(2, k, n0, nl, 1.0, fields.baseline_mms, family="qk")
    return H, OH, OV


@pytest.fixture(scope="module")
def q2q1():
    """Q2-Q1 on 16x16 squares, levels 4/8/16: vertex patches of 51 DoFs."""
    return _quad_fixture(2, 4, 3)


@pytest.fixture(scope="module")
def q4q3():
    """Q4-Q3 on 8x8 squares, levels 2/4/8: vertex (163), edge and cell patches."""
    return _quad_fixture(4, 2, 3)


@pytest.fixture(scope="module")
def q7q6():
    """Q7-Q6 on 4x4 squares, levels 2/4: vertex stars of 451 DoFs (global-memory inversion)."""
    return _quad_fixture(7, 2, 2)


@pytest.fixture(scope="module")
def q8q7():
    """Q8-Q7 on 4x4 squares, levels 2/4: vertex stars of 579 DoFs (global-memory inversion in blocks
    of 8 columns, the 768-DoF size class)."""
    return _quad_fixture(8, 2, 2)


def _bdm_fixture(k, n0, nl):
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print(f"[gpu] building BDM{k}-dP{k - 1} {n0 << (nl - 1)}x{n0 << (nl - 1)} hierarchy", flush=True)
    H = vk.Hierarchy(k, n0, nl, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS).bind().setup()
    OH, OV = solve.setup(2, k, n0, nl, 1.0, fields.paper_mms, family="bdm")
    return H, OH, OV


@pytest.fixture(scope="module")
def bdm1():
    """BDM1-dP0 with interior penalty on 8x8, levels 2/4/8: extended cell patches of up to 19 DoFs."""
    return _bdm_fixture(1, 2, 3)


@pytest.fixture(scope="module")
def bdm2():
    """BDM2-dP1 on 8x8, levels 2/4/8: extended cell patches of up to 42 DoFs."""
    return _bdm_fixture(2, 2, 3)


@pytest.fixture(scope="module")
def bdm4():
    """BDM4-dP3 on 8x8, levels 2/4/8: extended cell patches of up to 115 DoFs."""
    return _bdm_fixture(4, 2, 3)


@pytest.fixture(scope="module")
def bdm6():
    """BDM6-dP5 on 4x4, levels 1/2/4: interior extended patches of exactly 224 DoFs, the largest
    size held in the symmetric tiled storage and inverted in registers."""
    return _bdm_fixture(6, 1, 3)


@pytest.fixture(scope="module")
def bdm8():
    """BDM8-dP7 on 2x2, levels 1/2: extended cell patches of up to 333 DoFs (global-memory inversion)."""
    return _bdm_fixture(8, 1, 2)


# relative solution difference allowed between two 1e-10-residual solves: Taylor-Hood 1e-8;
# Scott-Vogelius 1e-6, since a relative rhs perturbation of 1e-11 moves the SV 16x16 solution by
# 1.5e-6 (its small nonzero singular values), measured with a sparse direct solve.  High orders:
# a random relative rhs perturbation of 1e-10 moves the P6-P5 8x8 solution by up to 1.7e-5 and the
# P8-P7 4x4 solution by up to 7.3e-5 (sparse direct solves), so two 1e-10-residual solutions may
# differ by twice that; iteration counts and residual histories are still compared tightly.
# Quadrilaterals, measured the same way: Q2-Q1 16x16 1.4e-7, Q4-Q3 8x8 9.0e-7, Q7-Q6 4x4 1.1e-5,
# Q8-Q7 4x4 2.9e-5
# BDM with interior penalty, the same way: BDM1 8x8 2.6e-9, BDM2 8x8 2.1e-8, BDM4 8x8 1.4e-7,
# BDM6 4x4 4.6e-7, BDM8 2x2 9.9e-7
XTOL = {"p2p1": 1e-8, "p4p3": 1e-8, "p2p1_3d": 1e-8, "p3dp2_sv": 1e-6, "p6p5": 4e-5, "p8p7": 1.5e-4,
        "q2q1": 3e-7, "q4q3": 2e-6, "q7q6": 2.2e-5, "q8q7": 6e-5, "bdm1": 1e-8, "bdm2": 5e-8, "bdm4": 3e-7,
        "bdm6": 1e-6, "bdm8": 2e-6}
# the GPU and oracle FP64 solves follow one Krylov trajectory (equal counts, histories checked), so their
# solutions agree far more closely than two arbitrary 1e-10-residual solutions: 1e-9 for every fixture
TRAJ_TOL = 1e-9
ALL = ["p2p1", "p4p3", "p2p1_3d", "p3dp2_sv", "p6p5", "p8p7", "q2q1", "q4q3", "q7q6", "q8q7", "bdm1", "bdm2",
       "bdm4", "bdm6", "bdm8"]


def _assembly_terms(L):
    """Roundings by which two independent assemblies of one entry may differ, in units of eps: the
    (k + 3)^dim quadrature terms, and for BDM levels the dual-basis inversions (growing like k^2)."""
    if getattr(L, "family", "") == "bdm":
        return 2 * (L.k + 3) ** 2 + 50 * L.k ** 2
    return 2 * (L.k + 3) ** L.dim


def _cond_bound(S):
    """max_i n_i * cond(K_i): scale of the explicit-inverse vs LU-solve difference."""
    return max(len(I) * np.linalg.cond(S.patch_matrix(i)) for i, I in enumerate(S.patches))


@pytest.mark.parametrize("fx", ALL)
def test_spmv_and_transfers(fx, request):
    H, OH, OV = request.getfixturevalue(fx)
    for l in range(len(OH.levels)):
        L = OH.levels[l]
        x = synth.vector(L.N, 100 + l)
        y = torch.empty(L.N, dtype=torch.float64, device="cuda")
        H.spmv(l, _dev(x), y)
        ref = L.K @ x
        # elementwise: summation roundoff (2 nnz_i eps) plus the assembly difference of two
        # independent assemblers (2 (k + 3)^dim eps, the quadrature sums of an entry)
        cV = _assembly_terms(L)
        absK = abs(L.K)
        bound = (cV + 2 * np.diff(L.K.indptr)) * EPS * (absK @ np.abs(x))
        assert np.all(np.abs(_host(y) - ref) <= bound)
        if l > 0:
            P = OH.P[l]
            xc = synth.vector(P.shape[1], 200 + l)
            ef = _dev(x)
            H.prolong_add(l, _dev(xc), ef)
            # the SV pressure transfer is an L^2 projection computed independently on each side
            # (clipped-polygon quadrature, local mass solves): entries agree to 2.5e-13 absolute
            # BDM transfers apply independently computed dual bases: entries agree to 1e-13 k absolute
            ptol = 2.5e-13 if fx == "p3dp2_sv" else (1e-13 * L.k if fx.startswith("bdm") else 0.0)
            pat = abs(P).sign()
            assert np.all(np.abs(_host(ef) - (x + P @ xc)) <=
                          1e-13 * (abs(P) @ np.abs(xc) + np.abs(x)) + ptol * (pat @ np.abs(xc)))
            rc = torch.empty(P.shape[1], dtype=torch.float64, device="cuda")
            H.restrict(l, _dev(x), rc)
            assert np.all(np.abs(_host(rc) - P.T @ x) <= 1e-13 * (abs(P.T) @ np.abs(x)) + ptol * (pat.T @ np.abs(x)))


@pytest.mark.parametrize("fx", ALL)
def test_patch_gather_matches_csr_and_oracle(fx, request):
    H, OH, OV = request.getfixturevalue(fx)
    l = len(OH.levels) - 1
    S = OV.smoothers[l]
    rp, col, val = H.csr(l)
    import scipy.sparse as sp
    Klib = sp.csr_matrix((val, col, rp), shape=(len(rp) - 1,) * 2).toarray()
    ptr, dofs = H.patches(l)
    J = len(ptr) - 1
    sizes = np.diff(ptr)
    out = torch.empty(int((sizes.astype(np.int64) ** 2).sum()), dtype=torch.float64, device="cuda")
    H.patch_gather(l, 0, J, out)
    flat = _host(out)
    off = 0
    for i in range(J):
        n = sizes[i]
        Ki = flat[off:off + n * n].reshape(n, n, order="F")
        off += n * n
        I = dofs[ptr[i]:ptr[i + 1]]
        assert np.array_equal(Ki, Klib[np.ix_(I, I)])          # bitwise: a pure copy of the library's CSR
        Ko = S.patch_matrix(i)
        assert np.abs(Ki - Ko).max() <= 1e-12 * np.abs(Ko).max()  # oracle: within assembly roundoff


@pytest.mark.parametrize("fx", ALL)
def test_patch_inverses(fx, request):
    H, OH, OV = request.getfixturevalue(fx)
    l = len(OH.levels) - 1
    S = OV.smoothers[l]
    rng = np.random.default_rng(5)
    picks = sorted(set(rng.integers(0, len(S.patches), 40).tolist()) | {0, len(S.patches) - 1})
    for i in picks:
        n = len(S.patches[i])
        out = torch.empty(n * n, dtype=torch.float64, device="cuda")
        H.patch_inverse(l, i, out)
        X = _host(out).reshape(n, n, order="F")
        Ki = S.patch_matrix(i)
        Xo = sla.lu_solve(S.lu[i], np.eye(n))
        c = np.linalg.cond(Ki)
        assert np.abs(Ki @ X - np.eye(n)).max() <= 8 * n * EPS * c
        assert np.abs(X - Xo).max() <= 8 * n * EPS * c * np.abs(Xo).max()


# one sweep and one V-cycle, measured on the correction (the change of x, or e from zero): the
# survey's parity protocol asks 1e-13 per sweep and 1e-12 per V-cycle, relative to the largest
# entry of the oracle's correction
SWEEP_TOL = 1e-13
VCYCLE_TOL = 1e-12


@pytest.mark.parametrize("fx", ALL)
def test_one_sweep(fx, request):
    H, OH, OV = request.getfixturevalue(fx)
    for l in range(1, len(OH.levels)):
        L, S = OH.levels[l], OV.smoothers[l]
        b, x0 = synth.vector(L.N, 300 + l), synth.vector(L.N, 400 + l)
        x = _dev(x0)
        H.smooth(l, _dev(b), x, 1)
        d_ref = S.sweep(b, x0) - x0
        err = _rel(_host(x) - x0, d_ref)
        # two sweeps in a row
        x = _dev(x0)
        H.smooth(l, _dev(b), x, 2)
        d2_ref = S.sweep(b, S.sweep(b, x0)) - x0
        err2 = _rel(_host(x) - x0, d2_ref)
        print(f"[measure] {fx} level {l}: sweep correction rel err {err:.2e}, two sweeps {err2:.2e}")
        assert err <= SWEEP_TOL
        assert err2 <= 2 * SWEEP_TOL


def test_coarse_solve(p4p3):
    H, OH, OV = p4p3
    r = synth.vector(OH.levels[0].N, 500)
    e = torch.empty_like(_dev(r))
    H.coarse_solve(_dev(r), e)
    ref = OV.coarse_solve(r)
    L0 = OH.levels[0]
    z = L0.nullvec()
    Kb = np.block([[L0.K.toarray(), z[:, None]], [z[None, :], np.zeros((1, 1))]])
    tol = 8 * Kb.shape[0] * EPS * np.linalg.cond(Kb)
    err = _rel(_host(e), ref)
    print(f"[gpu] coarse solve rel err {err:.2e} (tol {tol:.1e})")
    assert err <= tol


@pytest.mark.parametrize("fx", ALL)
def test_vcycle(fx, request):
    H, OH, OV = request.getfixturevalue(fx)
    L = OH.finest
    r = synth.vector(L.N, 600)
    e = torch.empty(L.N, dtype=torch.float64, device="cuda")
    H.vcycle(_dev(r), e, 2, 2)
    ref = OV.apply(r)
    err = _rel(_host(e), ref)
    print(f"[measure] {fx}: V-cycle rel err {err:.2e}")
    assert err <= VCYCLE_TOL
    # deterministic: a second application is bitwise identical
    e2 = torch.empty_like(e)
    H.vcycle(_dev(r), e2, 2, 2)
    assert torch.equal(e, e2)


@pytest.mark.parametrize("fx", ALL)
def test_solve_matches_oracle(fx, request):
    from oracle import solve
    H, OH, OV = request.getfixturevalue(fx)
    L = OH.finest
    b = H.rhs()
    ob = solve.consistent_rhs(L)
    x = torch.empty(L.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(b), x, history=True)
    xo, its, hist, conv = solve.solve(OH, OV)
    xg = _host(x)
    print(f"[gpu] {fx}: its gpu {res['iterations']} oracle {its}, rel res gpu {res['rel_residual']:.2e}, "
          f"solution diff {np.linalg.norm(xg - xo) / np.linalg.norm(xo):.2e}")
    assert res["converged"] and conv
    oracle_history.check_count(fx, res["iterations"], its, L, OV.apply)
    # the library's own residual is <= 1e-10; measured with the oracle's independently assembled K
    # it may move by the assembly difference (~1e-13 relative to |K||x|)
    true_res = np.linalg.norm(ob - L.K @ xg) / np.linalg.norm(ob)
    assert res["rel_residual"] <= 1e-10
    assert true_res <= 1.05e-10
    diff = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"[measure] {fx}: solution diff {diff:.2e} (trajectory bound {TRAJ_TOL:.0e}; any two 1e-10 solutions "
          f"may differ by {XTOL[fx]:.1e})")
    assert diff <= TRAJ_TOL
    # residual histories, every iteration: relative 1e-6 plus 1e-9 of the initial residual, or the
    # oracle's own sensitivity to 1e-13 perturbations where that is larger (P8-P7)
    oracle_history.check(fx, res["history"][: its + 1], hist, L, OV.apply)
    # bitwise reproducible
    x2 = torch.empty_like(x)
    H.solve(_dev(b), x2)
    assert torch.equal(x, x2)


def test_mixed_precision_solve(p4p3):
    """FP64 factorisation, FP32 stored/applied inverses: the FP64 FGMRES still reaches 1e-10."""
    import paper_2409_14222_amd as vk
    from oracle import solve
    H64, OH, OV = p4p3
    H = vk.Hierarchy(4, 4, 3, store=vk.VK_STORE_FP32).bind().setup()
    L = OH.finest
    b = H.rhs()
    x = torch.empty(L.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(b), x)
    xo, its, _, _ = solve.solve(OH, OV)
    xg = _host(x)
    ob = solve.consistent_rhs(L)
    print(f"[gpu] mixed: its {res['iterations']} (fp64 oracle {its}), diff {np.linalg.norm(xg - xo) / np.linalg.norm(xo):.2e}")
    assert res["converged"]
    assert res["iterations"] == its
    assert res["rel_residual"] <= 1e-10
    assert np.linalg.norm(ob - L.K @ xg) <= 1.05e-10 * np.linalg.norm(ob)
    assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("fx", ALL)
def test_launch_shapes_do_not_change_results(fx, request):
    """The autotuner may pick any lanes-per-row / waves-per-patch: results stay bitwise equal."""
    H, OH, OV = request.getfixturevalue(fx)
    L = OH.finest
    r = _dev(synth.vector(L.N, 700))
    saved = [H.tuning(l) for l in range(len(OH.levels))]
    ref = torch.empty_like(r)
    H.vcycle(r, ref, 2, 2)
    for lanes, waves, depth, merged in ((4, 1, 2, 0), (8, 2, 4, 1), (16, 4, 2, 0), (64, 1, 4, 1), (32, 4, 4, 1),
                                        (16, 8, 2, 1), (8, 16, 4, 0)):
        for l in range(len(OH.levels)):
            # 8 and 16 waves exist for the tiled storage only (patches of at most 224 DoFs, one RHS)
            w = waves if (waves <= 4 or (l > 0 and H.level_info(l).max_n <= 224)) else 4
            H.set_tuning(l, k_lanes=lanes, p_lanes=lanes, pt_lanes=lanes, apply_waves_large=w,
                         apply_waves_small=w, apply_depth_large=depth, apply_depth_small=depth,
                         apply_merged=merged)
        e = torch.empty_like(r)
        H.vcycle(r, e, 2, 2)
        assert torch.equal(e, ref), (lanes, waves)
    H.autotune(reps=2)
    e = torch.empty_like(r)
    H.vcycle(r, e, 2, 2)
    assert torch.equal(e, ref)
    for l, t in enumerate(saved):
        H.set_tuning(l, **t)


@pytest.mark.parametrize("k,n0,nl", [(2, 4, 3), (4, 2, 3)])
def test_graph_replays_match_eager(k, n0, nl):
    """Arnoldi steps replayed from captured HIP graphs give bitwise the eager result; replays
    are interleaved with eager solves and host synchronisations and every one is checked."""
    import paper_2409_14222_amd as vk
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        H = vk.Hierarchy(k, n0, nl).bind().setup()
        b = _dev(H.rhs())
        x_eager = torch.empty_like(b)
        ref = H.solve(b, x_eager)
        for rep in range(3):
            x = torch.empty_like(b)
            res = H.solve(b, x, graphs=True)
            side.synchronize()
            assert res["iterations"] == ref["iterations"] and res["converged"]
            assert torch.equal(x, x_eager), rep
            x2 = torch.empty_like(b)
            H.solve(b, x2)                      # eager work between replays
            side.synchronize()
            assert torch.equal(x2, x_eager)


def test_mixed_precision_solve_3d(p2p1_3d):
    """3D workload pattern: FP64 factorisation, FP32 inverses, FP64 FGMRES reaches 1e-10."""
    import paper_2409_14222_amd as vk
    from oracle import solve
    H64, OH, OV = p2p1_3d
    H = vk.Hierarchy(2, 2, 3, dim=3, forcing=vk.VK_F_CUBE_MMS, store=vk.VK_STORE_FP32).bind().setup()
    L = OH.finest
    x = torch.empty(L.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(H.rhs()), x)
    xo, its, _, _ = solve.solve(OH, OV)
    xg = _host(x)
    ob = solve.consistent_rhs(L)
    print(f"[gpu] 3D mixed: its {res['iterations']} (fp64 oracle {its}), diff {np.linalg.norm(xg - xo) / np.linalg.norm(xo):.2e}")
    assert res["converged"] and res["iterations"] == its
    assert res["rel_residual"] <= 1e-10
    assert np.linalg.norm(ob - L.K @ xg) <= 1.05e-10 * np.linalg.norm(ob)


def test_coarse_solve_sv(p3dp2_sv):
    H, OH, OV = p3dp2_sv
    r = synth.vector(OH.levels[0].N, 501)
    e = torch.empty_like(_dev(r))
    H.coarse_solve(_dev(r), e)
    L0 = OH.levels[0]
    z = L0.nullvec()
    Kb = np.block([[L0.K.toarray(), z[:, None]], [z[None, :], np.zeros((1, 1))]])
    tol = 8 * Kb.shape[0] * EPS * np.linalg.cond(Kb)
    err = _rel(_host(e), OV.coarse_solve(r))
    print(f"[gpu] SV coarse solve rel err {err:.2e} (tol {tol:.1e})")
    assert err <= tol


def test_mixed_precision_solve_sv(p3dp2_sv):
    """FP32-stored macro-patch inverses on the non-nested SV hierarchy: FP64 FGMRES reaches 1e-10."""
    import paper_2409_14222_amd as vk
    from oracle import solve
    _, OH, OV = p3dp2_sv
    H = vk.Hierarchy(3, 4, 3, family=vk.VK_SV, store=vk.VK_STORE_FP32).bind().setup()
    L = OH.finest
    b = H.rhs()
    x = torch.empty(L.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(b), x)
    xo, its, _, _ = solve.solve(OH, OV)
    xg = _host(x)
    ob = solve.consistent_rhs(L)
    print(f"[gpu] SV mixed: its {res['iterations']} (fp64 oracle {its}), "
          f"diff {np.linalg.norm(xg - xo) / np.linalg.norm(xo):.2e}")
    assert res["converged"] and res["iterations"] == its
    assert np.linalg.norm(ob - L.K @ xg) <= 1.05e-10 * np.linalg.norm(ob)
    assert np.linalg.norm(xg - xo) <= XTOL["p3dp2_sv"] * np.linalg.norm(xo)


@pytest.mark.parametrize("fx", ["bdm2", "bdm8"])
def test_bdm_many_rhs_and_fp32_inverses(fx, request):
    """BDM levels through the many-right-hand-side path (FP64 patch GEMMs; FP32 matrix-core GEMMs with
    FP32 inverses, including the column-major storage of patches above 224 DoFs for BDM8).  FP64
    inverses with many right-hand sides are limited to patches of 128 DoFs: BDM8 reports that."""
    import paper_2409_14222_amd as vk
    from oracle import solve
    H64, OH, OV = request.getfixturevalue(fx)
    L = OH.finest
    b = solve.consistent_rhs(L)
    xo, its, _, _ = solve.solve(OH, OV)
    R = 3
    Bm = np.stack([b * (c + 1) for c in range(R)], axis=1)
    k, n0, nl = L.k, OH.levels[0].n, len(OH.levels)
    for store in (vk.VK_STORE_FP64, vk.VK_STORE_FP32):
        H = vk.Hierarchy(k, n0, nl, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS, store=store)
        H.bind(max_rhs=R).setup()
        X = torch.zeros((L.N, R), dtype=torch.float64, device="cuda")
        if store == vk.VK_STORE_FP64 and H.level_info(nl - 1).max_n > 128:
            with pytest.raises(vk.VkError) as e:
                H.solve_multi(_dev(Bm), X, R)
            assert e.value.code == vk.VK_EINVAL
            del H
            continue
        _, res = H.solve_multi(_dev(Bm), X, R)
        Xh = _host(X)
        for c in range(R):
            rel = np.linalg.norm(Xh[:, c] - (c + 1) * xo) / ((c + 1) * np.linalg.norm(xo))
            print(f"[gpu] {fx} store {store} column {c}: its {res[c]['iterations']} (oracle {its}) diff {rel:.2e}")
            assert res[c]["converged"] and res[c]["rel_residual"] <= 1e-10
            # FP32-stored inverses change the preconditioner, by up to eps32 cond(K_i) in a local solve;
            # the BDM8 patches have cond(K_i) = 1.6e9, so that change is O(1) in some directions and
            # costs one FGMRES iteration (14 against 13); every other FP32 case keeps the FP64 count
            allowed = 1 if (store == vk.VK_STORE_FP32 and fx == "bdm8") else 0
            assert abs(res[c]["iterations"] - its) <= allowed
            assert rel <= XTOL[fx]
        del H


@pytest.mark.parametrize("fx", ["bdm2", "bdm4"])
def test_bdm_gpu_velocity_is_divergence_free(fx, request):
    """The H(div)-L2 pair's defining property (Sec. 2, the theorem on the H(div)-conforming
    discretisation): the discrete velocity the GPU solve returns is pointwise divergence-free,
    evaluated cell by cell with the oracle's basis."""
    from oracle import quad
    H, OH, OV = request.getfixturevalue(fx)
    L = OH.finest
    x = torch.empty(L.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(H.rhs()), x)
    assert res["converged"]
    xg = _host(x)
    qp, _ = quad.simplex_rule(2, 3)
    worst = scale = 0.0
    for ci, cell in enumerate(L.cells):
        v0, J = L.cell_geometry(cell)
        _, G = L.velocity(ci, xg, v0 + qp @ J.T)
        worst = max(worst, np.abs(G[:, 0, 0] + G[:, 1, 1]).max())
        scale = max(scale, np.abs(G).max())
    print(f"[gpu] {fx}: max |div u_h| {worst:.2e} (max |grad u_h| {scale:.2e})")
    assert worst <= 1e-9 * scale


def test_bdm_mixed_precision_and_graphs(bdm4):
    """BDM4-dP3 with FP32-stored inverses (factored in FP64): the FP64 FGMRES reaches 1e-10 against
    the oracle's matrix in the FP64 oracle's iteration count; and graph replay of the Arnoldi
    steps reproduces the eager FP64 solve bit for bit."""
    import paper_2409_14222_amd as vk
    from oracle import solve
    H64, OH, OV = bdm4
    L = OH.finest
    ob = solve.consistent_rhs(L)
    xo, its, _, _ = solve.solve(OH, OV)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        H = vk.Hierarchy(4, 2, 3, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS, store=vk.VK_STORE_FP32).bind().setup()
        G = vk.Hierarchy(4, 2, 3, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS).bind().setup()
    b = H.rhs()
    x = torch.empty(L.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(b), x)
    xg = _host(x)
    print(f"[gpu] bdm4 fp32 inverses: its {res['iterations']} (fp64 oracle {its}), "
          f"diff {np.linalg.norm(xg - xo) / np.linalg.norm(xo):.2e}")
    assert res["converged"] and res["iterations"] == its
    assert np.linalg.norm(ob - L.K @ xg) <= 1.05e-10 * np.linalg.norm(ob)
    assert np.linalg.norm(xg - xo) <= XTOL["bdm4"] * np.linalg.norm(xo)
    xe = torch.empty(L.N, dtype=torch.float64, device="cuda")
    G.solve(_dev(b), xe)
    for rep in range(2):
        xr = torch.empty_like(xe)
        G.solve(_dev(b), xr, graphs=True)
        side.synchronize()
        assert torch.equal(xr, xe), rep
