"""GPU parity of the Chebyshev-accelerated additive Vanka smoother (Sec. 3) against the oracle.

Compared through the C ABI: the per-level eigenvalue estimate (same counter-based start vector,
same Arnoldi recurrence), nu Chebyshev steps on every level, one V-cycle, the FGMRES solve
(iteration counts equal) and the many-right-hand-side path column by column.

Tolerances: one application of W B differs from the oracle's LU solves by at most
8 eps max_i n_i cond(K_i) relative (explicit inverses); the estimate runs k such applications
through the Arnoldi recurrence, and its largest Ritz value moves by at most that perturbation times
its condition, which the test bounds by 1e3 (the printed values sit far below); nu Chebyshev steps
add nu applications and the coefficients' relative change, the estimate's error.
"""
import numpy as np
import pytest

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


def _cond_bound(S):
    return max(len(I) * np.linalg.cond(S.patch_matrix(i)) for i, I in enumerate(S.patches))


def _build(k, n0, nl, family="th", weighting="none", store=0, max_rhs=1, seed=0):
    import paper_2409_14222_amd as vk
    from oracle import fields, solve
    print(f"[gpu] chebyshev hierarchy k={k} n0={n0} levels={nl} {family} {weighting} store={store} "
          f"rhs={max_rhs}", flush=True)
    fam = {"sv": vk.VK_SV, "qk": vk.VK_TH_QUAD, "bdm": vk.VK_BDM}.get(family, vk.VK_TH)
    w = vk.VK_WEIGHT_NONE if weighting == "none" else vk.VK_WEIGHT_MULTIPLICITY
    dim = 3 if family == "3d" else 2
    bdm = family == "bdm"
    H = vk.Hierarchy(k, n0, nl, dim=dim, family=fam, store=store, smoother=vk.VK_SMOOTH_CHEBYSHEV, weighting=w,
                     est_seed=seed, forcing=vk.VK_F_CUBE_MMS if dim == 3 else (vk.VK_F_PAPER_MMS if bdm else
                                                                                vk.VK_F_BASELINE_MMS))
    H.bind(max_rhs=max_rhs).setup()
    field = fields.cube_mms if dim == 3 else (fields.paper_mms if bdm else fields.baseline_mms)
    OH, OV = solve.setup(dim, k, n0, nl, 1.0, field,
                         family="th" if family == "3d" else family, smoother="chebyshev", weighting=weighting,
                         est_seed=seed)
    return H, OH, OV


CASES = {
    "p2p1": (2, 4, 3, "th", "none"),
    "p4p3": (4, 4, 3, "th", "none"),
    "p2p1_mult": (2, 4, 3, "th", "multiplicity"),
    "p3dp2_sv": (3, 4, 3, "sv", "none"),
    "q3q2": (3, 4, 3, "qk", "none"),
    "p2p1_3d": (2, 2, 3, "3d", "none"),
    "bdm3": (3, 2, 3, "bdm", "none"),
}


@pytest.fixture(scope="module", params=list(CASES))
def cheb(request):
    k, n0, nl, fam, w = CASES[request.param]
    H, OH, OV = _build(k, n0, nl, fam, w, seed=3)
    bounds = [None] + [_cond_bound(OV.smoothers[l]) for l in range(1, nl)]
    return request.param, H, OH, OV, bounds


def test_eigenvalue_estimate(cheb):
    name, H, OH, OV, cb = cheb
    for l in range(1, len(OH.levels)):
        inf = H.level_info(l)
        ref = OV.cheb[l].lam
        err = abs(inf.cheb_lambda - ref) / ref
        tol = 1e3 * 10 * 8 * EPS * cb[l]
        print(f"[gpu] {name} level {l}: lambda gpu {inf.cheb_lambda:.12f} oracle {ref:.12f} "
              f"rel {err:.1e} (tol {tol:.1e}) steps {inf.cheb_steps}")
        assert inf.cheb_steps == 10
        assert err <= tol
    assert H.level_info(0).cheb_lambda == 0.0


def test_chebyshev_steps(cheb):
    name, H, OH, OV, cb = cheb
    for l in range(1, len(OH.levels)):
        L, C = OH.levels[l], OV.cheb[l]
        lam_err = abs(H.level_info(l).cheb_lambda - C.lam) / C.lam
        b, x0 = synth.vector(L.N, 700 + l), synth.vector(L.N, 800 + l)
        for nu in (1, 2, 4):
            x = _dev(x0)
            H.smooth(l, _dev(b), x, nu)
            ref = C.sweeps(b, x0.copy(), nu)
            tol = nu * (8 * EPS * cb[l] + 4 * lam_err) * 4
            err = _rel(_host(x), ref)
            print(f"[gpu] {name} level {l} nu {nu}: rel err {err:.2e} (tol {tol:.1e})")
            assert err <= tol
        x = torch.full((L.N,), 7.0, dtype=torch.float64, device="cuda")
        H.smooth(l, _dev(b), x, 0)  # zero steps leave x alone
        assert torch.all(x == 7.0)


def test_vcycle_and_solve(cheb):
    from oracle import solve
    name, H, OH, OV, cb = cheb
    L = OH.finest
    r = synth.vector(L.N, 900)
    e = torch.empty(L.N, dtype=torch.float64, device="cuda")
    H.vcycle(_dev(r), e, 2, 2)
    ref = OV.apply(r)
    lam_err = max(abs(H.level_info(l).cheb_lambda - OV.cheb[l].lam) / OV.cheb[l].lam for l in range(1, len(OH.levels)))
    # the protocol's 1e-12 per V-cycle, plus the Chebyshev coefficients' relative change from the
    # estimate's difference (amplified by at most 64 over nu = 2 steps on three levels)
    tol = 1e-12 + 64 * lam_err
    err = _rel(_host(e), ref)
    print(f"[measure] {name}: Chebyshev V-cycle rel err {err:.2e} (tol {tol:.1e}, lambda rel diff {lam_err:.1e})")
    assert err <= tol
    x = torch.empty(L.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(H.rhs()), x, history=True)
    xo, its, hist, conv = solve.solve(OH, OV)
    xg = _host(x)
    rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"[gpu] {name}: its gpu {res['iterations']} oracle {its}, solution diff {rel:.2e}")
    assert conv == bool(res["converged"])
    oracle_history.check_count(name, res["iterations"], its, L, OV.apply)
    if conv:
        # one Krylov trajectory: 1e-9; where the count sits on the threshold and differs by one, the two
        # 1e-10-residual solutions may differ by the problem's sensitivity (see test_gpu_parity.XTOL)
        tol = 1e-9 if res["iterations"] == its else {"p3dp2_sv": 1e-6, "q3q2": 1e-6, "bdm3": 1e-7}.get(name, 1e-8)
        assert rel <= tol
        n = min(res["iterations"], its) + 1
        oracle_history.check(name, res["history"][:n], hist[:n], L, OV.apply)


def test_many_rhs_columns_match_oracle():
    H, OH, OV = _build(2, 4, 3, max_rhs=5, seed=1)
    R = 5
    l = 2
    L, C = OH.levels[l], OV.cheb[l]
    B = np.stack([synth.vector(L.N, 1000 + c) for c in range(R)], axis=1)
    X0 = np.stack([synth.vector(L.N, 1100 + c) for c in range(R)], axis=1)
    X = _dev(X0)
    H.smooth_multi(l, _dev(B), X, R, 3)
    Xg = _host(X)
    cb = _cond_bound(OV.smoothers[l])
    lam_err = abs(H.level_info(l).cheb_lambda - C.lam) / C.lam
    for c in range(R):
        ref = C.sweeps(B[:, c], X0[:, c].copy(), 3)
        err = _rel(Xg[:, c], ref)
        print(f"[gpu] multi column {c}: rel err {err:.2e}")
        assert err <= 12 * (8 * EPS * cb + 4 * lam_err) * 4
    from oracle import solve
    Lf = OH.finest
    b = solve.consistent_rhs(Lf)
    Bm = np.stack([b * (c + 1) for c in range(3)], axis=1)
    Xm = torch.zeros((Lf.N, 3), dtype=torch.float64, device="cuda")
    _, res = H.solve_multi(_dev(Bm), Xm, 3)
    xo, its, hist, conv = solve.solve(OH, OV)
    Xh = _host(Xm)
    for c in range(3):
        assert res[c]["iterations"] == its
        assert np.linalg.norm(Xh[:, c] - (c + 1) * xo) <= 1e-9 * (c + 1) * np.linalg.norm(xo)


def test_fp32_store_estimate_and_solve():
    """FP32 stored inverses: lambda within the FP32 rounding of B, the FP64 FGMRES still reaches 1e-10."""
    import paper_2409_14222_amd as vk
    H, OH, OV = _build(4, 4, 3, store=vk.VK_STORE_FP32, seed=3)
    for l in range(1, 3):
        ref = OV.cheb[l].lam
        assert abs(H.level_info(l).cheb_lambda - ref) <= 1e-4 * ref
    x = torch.empty(OH.finest.N, dtype=torch.float64, device="cuda")
    res = H.solve(_dev(H.rhs()), x)
    print(f"[gpu] fp32 chebyshev: its {res['iterations']} rel res {res['rel_residual']:.2e}")
    assert res["converged"] and res["rel_residual"] <= 1e-10
