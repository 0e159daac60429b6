"""GPU parity of the many-right-hand-side path (lockstep FGMRES, SpMM, patch GEMMs).

Every column is compared with the oracle run on that column alone.  The FP32
matrix-core patch GEMM is checked against an elementwise bound computed by
the oracle from FP32 rounding of the inverse, the inputs and the
accumulation.  Columns must not interact: a right-hand side solved alone, or
at another position of the batch, gives the same bits.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps
EPS32 = float(np.finfo(np.float32).eps)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def hier():
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print("[gpu-multi] building P2-P1 and P4-P3 16x16 hierarchies (FP64 and FP32 inverses)", flush=True)
    out = {}
    for k in (2, 4):
        OH, OV = solve.setup(2, k, 4, 3, 1.0, fields.baseline_mms)
        H64 = vk.Hierarchy(k, 4, 3).bind(max_rhs=16).setup()
        H32 = vk.Hierarchy(k, 4, 3, store=vk.VK_STORE_FP32).bind(max_rhs=16).setup()
        out[k] = (H64, H32, OH, OV)
    print("[gpu-multi] building SV P3-dP2 16x16 hierarchies", flush=True)
    OH, OV = solve.setup(2, 3, 4, 3, 1.0, fields.baseline_mms, family="sv")
    H64 = vk.Hierarchy(3, 4, 3, family=vk.VK_SV).bind(max_rhs=16).setup()
    H32 = vk.Hierarchy(3, 4, 3, family=vk.VK_SV, store=vk.VK_STORE_FP32).bind(max_rhs=16).setup()
    out["sv"] = (H64, H32, OH, OV)
    print("[gpu-multi] building P8-P7 4x4 hierarchies (patches of 435 DoFs)", flush=True)
    OH, OV = solve.setup(2, 8, 2, 2, 1.0, fields.baseline_mms)
    H64 = vk.Hierarchy(8, 2, 2).bind(max_rhs=16).setup()
    H32 = vk.Hierarchy(8, 2, 2, store=vk.VK_STORE_FP32).bind(max_rhs=16).setup()
    out[8] = (H64, H32, OH, OV)
    return out


@pytest.mark.parametrize("k", [2, 4, "sv"])
def test_smooth_multi_fp64(hier, k):
    H64, _, OH, OV = hier[k]
    R = 7
    for l in (1, 2):
        L, S = OH.levels[l], OV.smoothers[l]
        B = synth.vector(L.N * R, 800 + l).reshape(L.N, R)
        X0 = synth.vector(L.N * R, 900 + l).reshape(L.N, R)
        X = _dev(X0)
        H64.smooth_multi(l, _dev(B), X, R, 1)
        got = _host(X)
        cb = max(len(I) * np.linalg.cond(S.patch_matrix(i)) for i, I in enumerate(S.patches))
        for c in range(R):
            ref = S.sweep(B[:, c], X0[:, c])
            assert np.abs(got[:, c] - ref).max() <= 8 * EPS * cb * np.abs(ref).max()


@pytest.mark.parametrize("k", [2, 4, "sv", 8])
def test_smooth_multi_fp32_matrix_cores(hier, k):
    """FP32 inverses on the matrix cores: error within the FP32 rounding bound (k = 8: 8-wave
    workgroups for the 435-DoF patches)."""
    _, H32, OH, OV = hier[k]
    _check_fp32_sweep_from_zero(H32, OH, OV, 16, 1000)


@pytest.mark.parametrize("R", [64, 40])
def test_smooth_multi_fp32_matrix_cores_wide_p4p3(hier, R):
    """P4-P3 patches of up to 64 DoFs on 4 waves and of 65..123 DoFs on 8 (one 16-row tile per
    wave), with all four 16-column tiles holding right-hand sides (R = 64) or the fourth empty
    (R = 40): every column within the FP32 rounding bound."""
    import paper_2409_14222_amd as vk
    _, _, OH, OV = hier[4]
    H32 = vk.Hierarchy(4, 4, 3, store=vk.VK_STORE_FP32).bind(max_rhs=64).setup()
    assert H32.level_info(2).max_n > 64
    _check_fp32_sweep_from_zero(H32, OH, OV, R, 1100 + R)


def _check_fp32_sweep_from_zero(H32, OH, OV, R, seed):
    l = len(OH.levels) - 1
    L, S = OH.levels[l], OV.smoothers[l]
    B = synth.vector(L.N * R, seed).reshape(L.N, R)
    X = _dev(np.zeros((L.N, R)))
    H32.smooth_multi(l, _dev(B), X, R, 1)    # x = 0 + omega W sum_i R_i^T K_i^{-1} R_i b
    got = _host(X)
    # elementwise bound: |delta_i - K_i^{-1} b_i| <= (n_i + 2) eps32 |K_i^{-1}| |b_i| per patch,
    # then the weighted scatter of those bounds
    bound = np.zeros((L.N, R))
    ref = np.zeros((L.N, R))
    for i, I in enumerate(S.patches):
        Ainv = sla.lu_solve(S.lu[i], np.eye(len(I)))
        ref[I] += Ainv @ B[I]
        bound[I] += (len(I) + 2) * EPS32 * (np.abs(Ainv) @ np.abs(B[I]))
    w = (S.omega * S.weight)[:, None]
    ref *= w
    bound = bound * w + 16 * EPS * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)
    # and the FP32 path is not just FP64 in disguise (it should differ at FP32 level somewhere)
    assert np.abs(got - ref).max() > 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("k", [2, 4, "sv"])
def test_vcycle_multi_fp64(hier, k):
    H64, _, OH, OV = hier[k]
    R = 5
    L = OH.finest
    Rv = synth.vector(L.N * R, 1100).reshape(L.N, R)
    E = torch.empty((L.N, R), dtype=torch.float64, device="cuda")
    H64.vcycle_multi(_dev(Rv), E, R)
    got = _host(E)
    cb = max(max(len(I) * np.linalg.cond(S.patch_matrix(i)) for i, I in enumerate(S.patches))
             for S in OV.smoothers[1:])
    for c in range(R):
        ref = OV.apply(Rv[:, c])
        assert np.abs(got[:, c] - ref).max() <= 32 * EPS * cb * np.abs(ref).max()


def _oracle_random_solve(k, g):
    from oracle import fields, solve
    if k == "sv":
        OH, OV = solve.setup(2, 3, 4, 3, 1.0, lambda nu: fields.random_sine_field(g, nu), family="sv")
    else:
        OH, OV = solve.setup(2, k, 4, 3, 1.0, lambda nu: fields.random_sine_field(g, nu))
    x, its, _, conv = solve.solve(OH, OV)
    return OH, x, its, conv


@pytest.mark.parametrize("k,store", [(2, "fp64"), (4, "fp64"), (2, "fp32"), (4, "fp32"), ("sv", "fp64"),
                                     ("sv", "fp32")])
def test_solve_multi_matches_single_oracle_solves(hier, k, store):
    from oracle import solve
    H64, H32, OH, OV = hier[k]
    H = H64 if store == "fp64" else H32
    R = 4 if k == "sv" else 6
    # SV: a 1e-11 relative rhs perturbation moves the 16x16 solution by ~1.5e-6 (see the parity tests)
    xtol = 1e-6 if k == "sv" else 1e-8
    gs = [synth.forcing_coeffs(20240922 + j) for j in range(R)]
    N = OH.finest.N
    B = np.stack([H.rhs_random(g) for g in gs], axis=1)
    X = torch.empty((N, R), dtype=torch.float64, device="cuda")
    status, infos = H.solve_multi(_dev(B), X, R)
    got = _host(X)
    for c in range(R):
        OHc, xo, its, conv = _oracle_random_solve(k, gs[c])
        Lc = OHc.finest
        bo = solve.consistent_rhs(Lc)
        assert np.abs(B[:, c] - bo).max() <= 1e-13 * np.abs(bo).max()
        res = np.linalg.norm(bo - Lc.K @ got[:, c]) / np.linalg.norm(bo)
        diff = np.linalg.norm(got[:, c] - xo) / np.linalg.norm(xo)
        print(f"[gpu-multi] k={k} {store} col {c}: its {infos[c]['iterations']} oracle {its} res {res:.2e} diff {diff:.2e}")
        assert infos[c]["converged"] and conv
        assert infos[c]["rel_residual"] <= 1e-10 and res <= 1.05e-10
        assert infos[c]["iterations"] == its
        assert diff <= xtol


@pytest.mark.parametrize("store", ["fp64", "fp32"])
def test_columns_are_independent(hier, store):
    """A right-hand side gives bitwise the same solution alone and at any position in a batch."""
    H64, H32, OH, OV = hier[4]
    H = H64 if store == "fp64" else H32
    R = 8
    N = OH.finest.N
    B = np.stack([H.rhs_random(synth.forcing_coeffs(77 + j)) for j in range(R)], axis=1)
    X = torch.empty((N, R), dtype=torch.float64, device="cuda")
    _, infos = H.solve_multi(_dev(B), X, R)
    batch = _host(X)
    perm = np.array([5, 2, 7, 0, 3, 6, 1, 4])
    Xp = torch.empty((N, R), dtype=torch.float64, device="cuda")
    _, infos_p = H.solve_multi(_dev(B[:, perm]), Xp, R)
    shuffled = _host(Xp)
    for c in (0, 3, 7):
        x1 = torch.empty((N, 1), dtype=torch.float64, device="cuda")
        _, i1 = H.solve_multi(_dev(B[:, c:c + 1]), x1, 1)
        alone = _host(x1)[:, 0]
        assert np.array_equal(alone, batch[:, c])
        assert i1[0]["iterations"] == infos[c]["iterations"]
    for pos, c in enumerate(perm):
        assert np.array_equal(shuffled[:, pos], batch[:, c])


@pytest.mark.parametrize("store,max_rhs,R", [("fp64", 6, 5), ("fp32", 6, 5), ("fp64", 16, 12)])
def test_multi_graph_replays_match_eager(store, max_rhs, R):
    """Many-RHS Arnoldi steps replayed from captured HIP graphs give bitwise the eager result,
    also with columns converging at different iterations (12 columns: the K products over union
    groups); replays are interleaved with eager solves and host synchronisations and every one
    is checked."""
    import paper_2409_14222_amd as vk
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        st = vk.VK_STORE_FP32 if store == "fp32" else vk.VK_STORE_FP64
        H = vk.Hierarchy(2, 4, 3, store=st).bind(max_rhs=max_rhs).setup()
        N = H.level_info(2).n_free
        B = np.stack([H.rhs_random(synth.forcing_coeffs(300 + j)) * (10.0 ** -(j % 6)) for j in range(R)], axis=1)
        B[:, 2] = 0.0  # a column that is done before the first iteration
        Bd = _dev(B)
        X_eager = torch.empty((N, R), dtype=torch.float64, device="cuda")
        _, ref = H.solve_multi(Bd, X_eager, R)
        for rep in range(3):
            X = torch.empty((N, R), dtype=torch.float64, device="cuda")
            _, res = H.solve_multi(Bd, X, R, graphs=True)
            side.synchronize()
            assert [r["iterations"] for r in res] == [r["iterations"] for r in ref]
            assert torch.equal(X, X_eager), rep
            X2 = torch.empty_like(X)
            H.solve_multi(Bd, X2, R)
            side.synchronize()
            assert torch.equal(X2, X_eager)


# ---------------------------------------------------------------- the 64-RHS shape at 16x16
# The Scott-Vogelius many-RHS workload solves 64 right-hand sides at once.  Batches of more than
# 32 columns take their own kernels (wave-per-row transfer SpMM, wave-per-DoF scatter) and more
# than 48 the full-width matrix-core GEMM; K products of more than 8 columns run over union
# groups on the FP64 matrix cores.  These cases run them at 16x16, where the oracle can follow
# sampled columns one by one.

@pytest.fixture(scope="module")
def sv_wide(hier):
    import paper_2409_14222_amd as vk
    _, _, OH, OV = hier["sv"]
    print("[gpu-multi] building SV P3-dP2 16x16 hierarchies for 64 right-hand sides", flush=True)
    H64 = vk.Hierarchy(3, 4, 3, family=vk.VK_SV).bind(max_rhs=64).setup()
    H32 = vk.Hierarchy(3, 4, 3, family=vk.VK_SV, store=vk.VK_STORE_FP32).bind(max_rhs=64).setup()
    return H64, H32, OH, OV


@pytest.mark.parametrize("R", [64, 49, 33, 32, 17, 16, 9])
def test_spmv_multi_wide_groups(sv_wide, R):
    """Y = K X for more than 8 columns (rows in groups sharing one column list, FP64 matrix cores,
    1, 2 or 4 tiles of 16 columns per wave) gives bitwise what products of at most 8 columns give
    (one run of identical rows at a time, FMAs in ascending column order), on every level; it lies
    within the FP64 summation bound of the exact product with the library's matrix, and within that
    plus the assembly rounding of the oracle's product."""
    import scipy.sparse as sp
    H64, _, OH, OV = sv_wide
    for l in range(len(OH.levels)):
        L = OH.levels[l]
        X = synth.vector(L.N * R, 2100 + R + l).reshape(L.N, R)
        Y = torch.empty((L.N, R), dtype=torch.float64, device="cuda")
        H64.spmv_multi(l, _dev(X), Y, R)
        slices = []
        for c0 in range(0, R, 8):
            c1 = min(R, c0 + 8)
            Yh = torch.empty((L.N, c1 - c0), dtype=torch.float64, device="cuda")
            H64.spmv_multi(l, _dev(X[:, c0:c1]), Yh, c1 - c0)
            slices.append(_host(Yh))
        got = _host(Y)
        assert np.array_equal(got, np.concatenate(slices, axis=1)), l
        rp, col, val = H64.csr(l)
        K = sp.csr_matrix((val, col, rp), shape=(L.N, L.N))
        m = np.diff(rp)[:, None]
        absKX = abs(K) @ np.abs(X)
        ratio = (np.abs(got - K @ X) / np.maximum(2 * (m + 2) * EPS * absKX, 1e-300)).max()
        # the oracle assembles K on its own: entries agree to the quadrature sums' rounding
        bound = (2 * (L.k + 3) ** 2 + 2 * m + 4) * EPS * absKX
        ratio_o = (np.abs(got - L.K @ X) / np.maximum(bound, 1e-300)).max()
        print(f"[gpu-multi] SV wide level {l} R={R}: K X worst error / bound {ratio:.2e} (library matrix), "
              f"{ratio_o:.2e} (oracle matrix)")
        assert ratio <= 1.0 and ratio_o <= 1.0


@pytest.mark.parametrize("case", ["p4p3", "p2p1_3d", "bdm3", "q3q2"])
def test_spmv_multi_groups_every_family(case):
    """The union-group K product of a hierarchy bound for 64 right-hand sides gives, for 64 and for
    16 columns, bitwise the <= 8-column run product on every level of each discretisation (rows of very different lengths:
    3D vertex stars, BDM interior-penalty rows, quadrilateral cells) and lies within the FP64
    summation bound of the exact product with the library's matrix."""
    import scipy.sparse as sp
    import paper_2409_14222_amd as vk
    k, n0, nl, kw = {"p4p3": (4, 4, 3, {}),
                     "p2p1_3d": (2, 2, 3, dict(dim=3, forcing=vk.VK_F_CUBE_MMS)),
                     "bdm3": (3, 2, 3, dict(family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS)),
                     "q3q2": (3, 2, 3, dict(family=vk.VK_TH_QUAD))}[case]
    print(f"[gpu-multi] {case}: hierarchy for 64 right-hand sides", flush=True)
    H = vk.Hierarchy(k, n0, nl, **kw).bind(max_rhs=64).setup()
    for R in (64, 16):
        for l in range(nl):
            rp, col, val = H.csr(l)
            N = len(rp) - 1
            X = synth.vector(N * R, 2300 + l).reshape(N, R)
            Y = torch.empty((N, R), dtype=torch.float64, device="cuda")
            H.spmv_multi(l, _dev(X), Y, R)
            slices = []
            for c0 in range(0, R, 8):
                Yh = torch.empty((N, 8), dtype=torch.float64, device="cuda")
                H.spmv_multi(l, _dev(X[:, c0:c0 + 8]), Yh, 8)
                slices.append(_host(Yh))
            got = _host(Y)
            assert np.array_equal(got, np.concatenate(slices, axis=1)), (case, R, l)
            K = sp.csr_matrix((val, col, rp), shape=(N, N))
            bound = 2 * (np.diff(rp)[:, None] + 2) * EPS * (abs(K) @ np.abs(X))
            ratio = (np.abs(got - K @ X) / np.maximum(bound, 1e-300)).max()
            print(f"[gpu-multi] {case} R={R} level {l}: K X worst error / bound {ratio:.2e}")
            assert ratio <= 1.0


@pytest.mark.parametrize("R", [64, 49])
def test_smooth_multi_wide_fp64(sv_wide, R):
    """One FP64 sweep on R columns from a random start: each column's correction against the
    oracle's sweep of that column alone."""
    H64, _, OH, OV = sv_wide
    l = 2
    L, S = OH.levels[l], OV.smoothers[l]
    B = synth.vector(L.N * R, 1500 + R).reshape(L.N, R)
    X0 = synth.vector(L.N * R, 1600 + R).reshape(L.N, R)
    X = _dev(X0)
    H64.smooth_multi(l, _dev(B), X, R, 1)
    got = _host(X)
    worst = 0.0
    for c in range(R):
        d_ref = S.sweep(B[:, c], X0[:, c]) - X0[:, c]
        err = np.abs((got[:, c] - X0[:, c]) - d_ref).max() / np.abs(d_ref).max()
        worst = max(worst, err)
    print(f"[gpu-multi] SV wide R={R} FP64 sweep: worst column correction rel err {worst:.2e}")
    assert worst <= 1e-13


@pytest.mark.parametrize("R", [64, 49])
def test_smooth_multi_wide_fp32(sv_wide, R):
    """One sweep with FP32 inverses on the matrix cores from a random start (FP64 SpMM residual,
    FP32 gather and GEMM, FP64 scatter): every column within the elementwise FP32 rounding bound."""
    _, H32, OH, OV = sv_wide
    l = 2
    L, S = OH.levels[l], OV.smoothers[l]
    B = synth.vector(L.N * R, 1700 + R).reshape(L.N, R)
    X0 = synth.vector(L.N * R, 1800 + R).reshape(L.N, R)
    X = _dev(X0)
    H32.smooth_multi(l, _dev(B), X, R, 1)
    got = _host(X)
    Rres = B - L.K @ X0
    # FP64 residual rounding (the SpMM's sums and the assembly difference), elementwise
    rbound = (2 * (L.k + 3) ** 2 + 2 * np.diff(L.K.indptr))[:, None] * EPS * (abs(L.K) @ np.abs(X0) + np.abs(B))
    corr = np.zeros((L.N, R))
    bound = np.zeros((L.N, R))
    for i, I in enumerate(S.patches):
        Ainv = sla.lu_solve(S.lu[i], np.eye(len(I)))
        corr[I] += Ainv @ Rres[I]
        bound[I] += (len(I) + 2) * EPS32 * (np.abs(Ainv) @ np.abs(Rres[I])) + np.abs(Ainv) @ rbound[I]
    w = (S.omega * S.weight)[:, None]
    ref = X0 + w * corr
    bound = w * bound + 4 * EPS * (np.abs(X0) + np.abs(ref))
    ratio = (np.abs(got - ref) / bound).max()
    print(f"[gpu-multi] SV wide R={R} FP32 sweep: worst error / bound {ratio:.2e}")
    assert ratio <= 1.0


def test_vcycle_multi_wide_fp64(sv_wide):
    H64, _, OH, OV = sv_wide
    R = 64
    L = OH.finest
    Rv = synth.vector(L.N * R, 1900).reshape(L.N, R)
    E = torch.empty((L.N, R), dtype=torch.float64, device="cuda")
    H64.vcycle_multi(_dev(Rv), E, R)
    got = _host(E)
    worst = 0.0
    for c in (0, 17, 33, 48, 49, 63):
        ref = OV.apply(Rv[:, c])
        worst = max(worst, np.abs(got[:, c] - ref).max() / np.abs(ref).max())
    print(f"[gpu-multi] SV wide V-cycle R=64: worst sampled column rel err {worst:.2e}")
    assert worst <= 1e-12


@pytest.mark.parametrize("R,store", [(64, "fp32"), (49, "fp32"), (64, "fp64")])
def test_solve_multi_wide_matches_oracle(sv_wide, R, store):
    """The 64-RHS workload at 16x16: R random forcings (seeds 20240922 + j) solved together; sampled
    columns against the oracle's solve of that column (its own load vector, equal iteration counts),
    every column against 1e-10 with the oracle's matrix."""
    from oracle import fields, solve, sv
    H64, H32, OH, OV = sv_wide
    H = H32 if store == "fp32" else H64
    L = OH.finest
    gs = [synth.forcing_coeffs(synth.SEED + j) for j in range(R)]
    B = np.stack([H.rhs_random(g) for g in gs], axis=1)
    X = torch.empty((L.N, R), dtype=torch.float64, device="cuda")
    _, infos = H.solve_multi(_dev(B), X, R)
    got = _host(X)
    for c in range(R):
        assert infos[c]["converged"] and infos[c]["rel_residual"] <= 1e-10
        bc = solve.consistent_rhs(L, B[:, c])
        assert np.linalg.norm(bc - L.K @ got[:, c]) <= 1.05e-10 * np.linalg.norm(bc)
    for c in (0, 21, 40, R - 1):
        Lc = sv.SVLevel(3, 16, 1.0, fields.random_sine_field(gs[c]))
        assert np.abs(B[:, c] - Lc.b).max() <= 1e-13 * np.abs(Lc.b).max()
        xo, its, _, conv = solve.solve(OH, OV, b=Lc.b)
        diff = np.linalg.norm(got[:, c] - xo) / np.linalg.norm(xo)
        print(f"[gpu-multi] SV wide R={R} {store} col {c}: its {infos[c]['iterations']} oracle {its}, diff {diff:.2e}")
        assert conv and infos[c]["iterations"] == its
        assert diff <= 1e-6
