"""CPU tests of the HIP library's host side (no GPU needed).

The C ABI must load and export every function declared in include/vk.h; the
library's own host assembly (mesh, numbering, CSR, right-hand side,
prolongation, patches) must agree with the independent oracle.
"""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2409_14222_amd as vk
from oracle import fields, norms, patches, solve, th

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_function():
    hdr = open(os.path.join(ROOT, "include", "vk.h")).read()
    declared = set(re.findall(r"\b(vk_[a-z0-9_]+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    missing = [f for f in declared if not hasattr(vk.lib, f)]
    assert not missing
    assert declared == set(vk.EXPORTS)


def _asm_bound(ol):
    return 2 * (ol.k + 3) ** ol.dim


def _csr_matrix(rp, col, val, n, m):
    return sp.csr_matrix((val, col, rp), shape=(n, m))


@pytest.mark.parametrize("k,n0,nl", [(2, 4, 3), (3, 2, 2), (4, 2, 3), (6, 2, 2), (8, 2, 2)])
def test_host_assembly_matches_oracle(k, n0, nl):
    H = vk.Hierarchy(k, n0, nl)
    OH = th.THHierarchy(2, k, n0, nl, 1.0, fields.baseline_mms)
    for l in range(nl):
        ol = OH.levels[l]
        inf = H.level_info(l)
        assert (inf.n_free, inf.nnz, inf.n_velocity) == (ol.N, ol.K.nnz, ol.nu_free)
        X, kind = H.dof_coords(l)
        OX, okind = ol.dof_coords()
        assert np.array_equal(kind, okind) and np.abs(X - OX).max() < 1e-15
        rp, col, val = H.csr(l)
        assert np.array_equal(rp, ol.K.indptr) and np.array_equal(col, ol.K.indices)
        # two independent assemblers, each summing (k + 3)^dim quadrature terms per element entry:
        # entries agree to 2 (k + 3)^dim eps of the row maximum
        cV = _asm_bound(ol)
        rowmax = np.maximum.reduceat(np.abs(ol.K.data), ol.K.indptr[:-1])
        tol = cV * np.finfo(float).eps * np.repeat(rowmax, np.diff(ol.K.indptr))
        assert np.all(np.abs(val - ol.K.data) <= tol + 1e-300)
        if l > 0:
            prp, pcol, pval = H.prolongation(l)
            P = OH.P[l]
            assert np.array_equal(prp, P.indptr) and np.array_equal(pcol, P.indices)
            assert np.abs(pval - P.data).max() <= 1e-14
            ptr, dofs = H.patches(l)
            op = patches.build_patches(ol)
            assert len(op) == len(ptr) - 1
            for i, I in enumerate(op):
                assert list(dofs[ptr[i]:ptr[i + 1]]) == list(I)
    b = H.rhs()
    ob = solve.consistent_rhs(OH.finest)
    assert np.abs(b - ob).max() <= 1e-13 * np.abs(ob).max()


def test_random_forcing_rhs_matches_oracle():
    import synth
    g = synth.forcing_coeffs(7)
    H = vk.Hierarchy(2, 2, 2, forcing=vk.VK_F_RANDOM, coeffs=g)
    L = th.THLevel(2, 2, 4, 1.0, fields.random_sine_field(g))
    assert np.abs(H.rhs() - solve.consistent_rhs(L)).max() <= 1e-13 * np.abs(L.b).max()


def test_star_patches_match_oracle():
    H = vk.Hierarchy(3, 2, 2, construct=vk.VK_PATCH_STAR)
    ol = th.THLevel(2, 3, 4, 1.0, fields.baseline_mms(1.0))
    ptr, dofs = H.patches(1)
    op = patches.build_patches(ol, "star")
    assert [list(dofs[ptr[i]:ptr[i + 1]]) for i in range(len(op))] == [list(I) for I in op]


def test_p4p3_level_counts_of_the_64x64_hierarchy_coarse_levels():
    H = vk.Hierarchy(4, 4, 3)
    got = [(H.level_info(l).n_free, H.level_info(l).nnz) for l in range(3)]
    assert got == [(619, 29720), (2547, 137528), (10339, 590072)]
    inf = H.level_info(2)
    assert (inf.n_patches, inf.sum_n, inf.sum_n2, inf.max_n) == (1601, 83731, 5776697, 123)


def test_invalid_arguments_are_rejected():
    with pytest.raises(vk.VkError) as e:
        vk.Hierarchy(1, 4, 3)
    assert e.value.code == vk.VK_EINVAL
    with pytest.raises(vk.VkError) as e:
        vk.Hierarchy(2, 4, 3, viscosity=-1.0)
    assert e.value.code == vk.VK_EINVAL
    with pytest.raises(vk.VkError) as e:
        vk.Hierarchy(2, 4, 1)
    assert e.value.code == vk.VK_EINVAL
    H = vk.Hierarchy(2, 2, 2)
    with pytest.raises(vk.VkError) as e:
        H.level_info(5)
    assert e.value.code == vk.VK_EINVAL
    # device calls before bind are state errors, not crashes
    with pytest.raises(vk.VkError) as e:
        vk.check(vk.lib.vk_patches_setup(H.h))
    assert e.value.code == vk.VK_ESTATE
    # union groups exist on levels with patches only, and take all of their arrays or none
    with pytest.raises(vk.VkError) as e:
        H.union_groups(0)
    assert e.value.code == vk.VK_EINVAL
    sizes = np.zeros(4, np.int64)
    some = np.zeros(16, np.int32)
    with pytest.raises(vk.VkError) as e:
        vk.check(vk.lib.vk_level_union_groups(H.h, 1, vk._ptr(sizes), vk._ptr(some), None, None, None, None, None))
    assert e.value.code == vk.VK_EINVAL


def test_server_create_validates_streams():
    """The server runs on caller-owned streams: a missing array, a count out of 1..64 or a null stream
    is rejected before anything touches a device (these calls make no HIP call)."""
    import ctypes
    opts = vk.vk_server_opts(4, vk.VK_STORE_FP32, 0.5, 2, 30, 100, 1e-10, 16)
    pool = ctypes.c_void_p(1 << 20)           # never dereferenced: creation only records it
    out = ctypes.c_void_p()
    fake = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    null = (ctypes.c_void_p * 2)(0x1000, None)
    for arr, n in ((None, 1), (fake, 0), (fake, 65), (null, 2)):
        st = vk.lib.vk_server_create(ctypes.byref(opts), pool, 1 << 30, arr, n, ctypes.byref(out))
        assert st == vk.VK_EINVAL, (n, st)
    st = vk.lib.vk_server_create(ctypes.byref(opts), pool, 1 << 30, fake, 2, ctypes.byref(out))
    assert st == vk.VK_OK
    assert vk.lib.vk_server_destroy(out) == vk.VK_OK


def test_noalloc_smoothing_rejects_levels_beyond_its_scratch():
    """The allocation-free smoothing call holds 32 MiB of sweep scratch per GPU: the P4-P3 128x128
    finest level (670,211 DoFs, 5.5 M patch slots: 49.6 MB) is refused with VK_EINVAL before any
    device work; a level that fits gets past the size check to the state check (not bound)."""
    H = vk.Hierarchy(4, 4, 6)
    st = vk.lib.vk_smooth_noalloc(H.h, 5, 1 << 20, 1 << 21, 1)
    assert st == vk.VK_EINVAL
    assert "needs" in vk.lib.vk_last_error().decode()
    assert vk.lib.vk_smooth_noalloc(H.h, 4, 1 << 20, 1 << 21, 1) == vk.VK_ESTATE


def test_tuning_cache_needs_a_set_up_hierarchy():
    """vk_autotune_cached times kernels: before bind/setup it is a state error, whatever the path."""
    import ctypes
    H = vk.Hierarchy(2, 2, 2)
    hit = ctypes.c_int(7)
    assert vk.lib.vk_autotune_cached(H.h, 2, b"/nonexistent/dir/cache.txt", ctypes.byref(hit)) == vk.VK_ESTATE
    assert hit.value == 7


def test_host_assembly_3d_matches_oracle():
    """3D P2-P1 on Kuhn tetrahedra (levels 2, 4 cubes per direction)."""
    H = vk.Hierarchy(2, 2, 2, dim=3, forcing=vk.VK_F_CUBE_MMS)
    OH = th.THHierarchy(3, 2, 2, 2, 1.0, fields.cube_mms)
    for l in range(2):
        ol = OH.levels[l]
        inf = H.level_info(l)
        assert (inf.n_free, inf.nnz) == (ol.N, ol.K.nnz)
        X, kind = H.dof_coords(l)
        OX, okind = ol.dof_coords()
        assert np.array_equal(kind, okind) and np.abs(X - OX).max() < 1e-15
        rp, col, val = H.csr(l)
        assert np.array_equal(rp, ol.K.indptr) and np.array_equal(col, ol.K.indices)
        cV = _asm_bound(ol)
        rowmax = np.maximum.reduceat(np.abs(ol.K.data), ol.K.indptr[:-1])
        assert np.all(np.abs(val - ol.K.data) <= cV * np.finfo(float).eps * np.repeat(rowmax, np.diff(ol.K.indptr)))
        if l > 0:
            prp, pcol, pval = H.prolongation(l)
            P = OH.P[l]
            assert np.array_equal(prp, P.indptr) and np.array_equal(pcol, P.indices)
            assert np.abs(pval - P.data).max() <= 1e-14
            ptr, dofs = H.patches(l)
            op = patches.build_patches(ol)
            assert [list(dofs[ptr[i]:ptr[i + 1]]) for i in range(len(op))] == [list(I) for I in op]
    assert np.abs(H.rhs() - solve.consistent_rhs(OH.finest)).max() <= 1e-13 * np.abs(OH.finest.b).max()


def test_3d_counts_of_the_16_cube_hierarchy():
    """Free DoFs and patch statistics of P2-P1 on 4^3 / 8^3 / 16^3 Kuhn meshes."""
    H = vk.Hierarchy(2, 4, 3, dim=3, forcing=vk.VK_F_CUBE_MMS)
    for l, n in enumerate((4, 8, 16)):
        inf = H.level_info(l)
        assert inf.n_free == 3 * (2 * n - 1) ** 3 + (n + 1) ** 3
    inf = H.level_info(2)
    assert (inf.n_patches, inf.max_n) == (17 ** 3, 196)     # interior vertex star: 65 P2 nodes x 3 + 1


def test_singular_coarsest_level_is_reported():
    """A single Kuhn cube has spurious P1 pressure modes: the bordered coarsest system is
    singular beyond the constant and the library must refuse it."""
    with pytest.raises(vk.VkError) as e:
        vk.Hierarchy(2, 1, 2, dim=3, forcing=vk.VK_F_CUBE_MMS)
    assert e.value.code == vk.VK_ESINGULAR


# ---------------------------------------------------------------- Scott-Vogelius (barycentric) levels
@pytest.mark.parametrize("k", [2, 3])
def test_host_assembly_sv_matches_oracle(k):
    """P_k-dP_{k-1} on barycentric refinements of 2x2 / 4x4 / 8x8: numbering, CSR, non-nested
    transfers (nodal velocity, exact L^2 pressure projection), macro patches and the rhs."""
    from oracle import sv
    H = vk.Hierarchy(k, 2, 3, family=vk.VK_SV)
    OH = sv.SVHierarchy(k, 2, 3, 1.0, fields.baseline_mms)
    for l in range(3):
        ol = OH.levels[l]
        inf = H.level_info(l)
        assert (inf.n_free, inf.nnz, inf.n_velocity) == (ol.N, ol.K.nnz, ol.nu_free)
        X, kind = H.dof_coords(l)
        OX, okind = ol.dof_coords()
        assert np.array_equal(kind, okind) and np.abs(X - OX).max() < 1e-15
        rp, col, val = H.csr(l)
        assert np.array_equal(rp, ol.K.indptr) and np.array_equal(col, ol.K.indices)
        cV = _asm_bound(ol)
        rowmax = np.maximum.reduceat(np.abs(ol.K.data), ol.K.indptr[:-1])
        assert np.all(np.abs(val - ol.K.data) <= cV * np.finfo(float).eps * np.repeat(rowmax, np.diff(ol.K.indptr)))
        if l > 0:
            prp, pcol, pval = H.prolongation(l)
            P = OH.P[l]
            assert np.array_equal(prp, P.indptr) and np.array_equal(pcol, P.indices)
            # the pressure rows come from clipped-polygon quadrature and a 3x3 / 6x6 mass solve on
            # both sides (values up to ~2): a few hundred roundings
            assert np.abs(pval - P.data).max() <= 1e-13
            ptr, dofs = H.patches(l)
            op = patches.build_patches(ol, "macro")
            assert [list(dofs[ptr[i]:ptr[i + 1]]) for i in range(len(op))] == [list(I) for I in op]
    assert np.abs(H.rhs() - solve.consistent_rhs(OH.finest)).max() <= 1e-13 * np.abs(OH.finest.b).max()


def test_sv_counts_and_random_rhs():
    import synth
    from oracle import sv
    H = vk.Hierarchy(3, 4, 3, family=vk.VK_SV)
    for l, n in enumerate((4, 8, 16)):
        inf = H.level_info(l)
        assert inf.n_free == 90 * n * n - 12 * n + 2
    inf = H.level_info(2)
    assert (inf.nnz, inf.n_patches, inf.sum_n, inf.sum_n2, inf.max_n) == (802292, 512, 28044, 1539784, 56)
    g = synth.forcing_coeffs(7)
    Hs = vk.Hierarchy(3, 2, 2, family=vk.VK_SV)
    L = sv.SVLevel(3, 4, 1.0, fields.random_sine_field(g))
    assert np.abs(Hs.rhs_random(g) - solve.consistent_rhs(L)).max() <= 1e-13 * np.abs(L.b).max()


def test_sv_invalid_combinations_are_rejected():
    for kw in (dict(family=vk.VK_SV, construct=vk.VK_PATCH_COMPOSITE), dict(construct=vk.VK_PATCH_MACRO),
               dict(family=vk.VK_SV, dim=3, forcing=vk.VK_F_CUBE_MMS)):
        with pytest.raises(vk.VkError) as e:
            vk.Hierarchy(3, 2, 2, **kw)
        assert e.value.code == vk.VK_EINVAL
    with pytest.raises(vk.VkError) as e:
        vk.Hierarchy(5, 2, 2, family=vk.VK_SV)
    assert e.value.code == vk.VK_EINVAL


def test_symmetric_tiled_storage_size():
    """The stored inverse of a patch of n DoFs in the tiled layout is the nb (nb + 1) / 2 tiles of
    8 x 8 on and below the diagonal, nb = ceil(n / 8), the nb tiles of the last block row cut to
    the 2-double row chunks below n; the column-major layout rounds n up to 2."""
    for H, levels in ((vk.Hierarchy(4, 2, 3), (1, 2)), (vk.Hierarchy(3, 2, 2, family=vk.VK_SV), (1,)),
                      (vk.Hierarchy(2, 2, 2, dim=3, forcing=vk.VK_F_CUBE_MMS), (1,))):
        for l in levels:
            ptr, _ = H.patches(l)
            n = np.diff(ptr).astype(np.int64)
            nb = (n + 7) // 8
            inf = H.level_info(l)
            nvr = (n - 8 * (nb - 1) + 1) // 2  # 2-double chunks of the last block row's n - 8 (nb - 1) rows
            assert inf.inv_elems_tri == int(((nb - 1) * nb // 2 * 64 + nb * 8 * 2 * nvr).sum())
            assert inf.inv_elems_tri < inf.sum_n2 or n.max() <= 8


def _match_eigs(a, b, tol):
    """Each of a matched to a distinct nearest entry of b (greedy on sorted distance)."""
    a, b = list(a), list(b)
    assert len(a) == len(b)
    for z in a:
        i = int(np.argmin([abs(z - w) for w in b]))
        assert abs(z - b[i]) <= tol, (z, b[i])
        b.pop(i)


def test_hessenberg_eigenvalues_match_dense_eigensolver():
    """The library's QR iteration against LAPACK's on Hessenberg matrices with real and complex
    spectra, a zero subdiagonal (split matrix), a 1 x 1 and a 2 x 2 rotation, and the Hessenberg
    matrices of Arnoldi on nonsymmetric operators; for a tight cluster under a non-normal part, whose
    eigenvalues no two backward-stable methods need to agree on, only the backward error."""
    rng = np.random.default_rng(11)
    cases = [np.array([[3.5]]), np.array([[0.0, -2.0], [2.0, 0.0]])]
    for n in (3, 5, 10, 30, 60):
        cases.append(np.triu(rng.standard_normal((n, n)), -1))
    S = np.triu(rng.standard_normal((8, 8)), -1)
    S[4, 3] = 0.0
    cases.append(S)
    arnoldi = []
    for n, spread in ((10, 1.0), (40, 1.0), (40, 0.0)):
        # spread 0: a tight cluster under a non-normal upper part (ill-conditioned eigenvalues)
        d = np.linspace(0.2, 2.0, n) if spread else 1.0 + 0.01 * rng.standard_normal(n)
        A = np.diag(d) + 0.3 / np.sqrt(n) * np.triu(rng.standard_normal((n, n)), 1)
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        A = Q @ A @ Q.T
        V = np.zeros((n, n + 1)); Hm = np.zeros((n + 1, n))
        v = rng.standard_normal(n); V[:, 0] = v / np.linalg.norm(v)
        for j in range(n):
            w = A @ V[:, j]
            for _ in range(2):
                h = V[:, : j + 1].T @ w
                w -= V[:, : j + 1] @ h
                Hm[: j + 1, j] += h
            Hm[j + 1, j] = np.linalg.norm(w)
            V[:, j + 1] = w / Hm[j + 1, j]
        (cases if spread else arnoldi).append(Hm[:n, :n])
    for H in cases + arnoldi:
        got = vk.hessenberg_eigenvalues(H)
        nrm = np.linalg.norm(H, 2)
        # backward error: each value is an exact eigenvalue of a matrix within a few ulps of H
        for z in got:
            assert np.linalg.svd(H - z * np.eye(H.shape[0]), compute_uv=False)[-1] <= 1e-13 * nrm * H.shape[0]
        assert abs(got.sum() - np.trace(H)) <= 1e-13 * nrm * H.shape[0]
    for H in cases:
        got = vk.hessenberg_eigenvalues(H)
        want = np.linalg.eigvals(H)
        _match_eigs(got, want, 1e-9 * max(1.0, np.abs(H).max()) * H.shape[0])
        assert abs(got.real.max() - want.real.max()) <= 1e-10 * max(1.0, np.abs(H).max()) * H.shape[0]


def test_hessenberg_eigenvalues_reject_bad_input():
    with pytest.raises(vk.VkError) as e:
        vk.hessenberg_eigenvalues(np.array([[1.0, np.nan], [1.0, 2.0]]))
    assert e.value.code == vk.VK_ENAN
    re = np.empty(1)
    assert vk.lib.vk_hessenberg_eigenvalues(0, re.ctypes.data, re.ctypes.data, re.ctypes.data) == vk.VK_EINVAL


def test_chebyshev_options_are_validated():
    for kw in ({"smoother": 2}, {"weighting": 5}, {"smoother": vk.VK_SMOOTH_CHEBYSHEV, "est_steps": 201},
               {"est_steps": -1}):
        with pytest.raises(vk.VkError) as e:
            vk.Hierarchy(2, 2, 3, **kw)
        assert e.value.code == vk.VK_EINVAL, kw
    H = vk.Hierarchy(2, 2, 3, smoother=vk.VK_SMOOTH_CHEBYSHEV, weighting=vk.VK_WEIGHT_NONE)
    assert H.level_info(1).cheb_lambda == 0.0  # no estimate before vk_patches_setup


@pytest.mark.parametrize("k,n0", [(2, 4), (4, 4), (8, 2)])
def test_coarse_inverse_matches_dense_inverse(k, n0):
    """The blocked Gauss-Jordan of the coarsest bordered matrix against LAPACK's inverse of the
    oracle's bordered matrix (several 32-pivot panels and a ragged last one at every size here)."""
    H = vk.Hierarchy(k, n0, 2)
    OH = th.THHierarchy(2, k, n0, 2, 1.0, fields.baseline_mms)
    L0 = OH.levels[0]
    z = L0.nullvec()
    Kb = np.block([[L0.K.toarray(), z[:, None]], [z[None, :], np.zeros((1, 1))]])
    ref = np.linalg.inv(Kb)[: L0.N, : L0.N]
    got = H.coarse_inverse()
    c = np.linalg.cond(Kb)
    print(f"k={k}: N0={L0.N} cond {c:.1e} err {np.abs(got - ref).max() / np.abs(ref).max():.1e}")
    assert np.abs(got - ref).max() <= 8 * Kb.shape[0] * np.finfo(float).eps * c * np.abs(ref).max()


@pytest.mark.parametrize("case", ["p2p1", "p4p3_paper", "p3p2_3d", "sv"])
def test_solution_errors_match_oracle_norms(case):
    """The library's discretisation-error norms against the oracle's, on the discrete solution
    (errors near the discretisation level) and on a perturbed vector (large errors, both terms)."""
    import scipy.sparse.linalg as spla
    from oracle import sv
    if case == "p2p1":
        H = vk.Hierarchy(2, 4, 2); OH = th.THHierarchy(2, 2, 4, 2, 1.0, fields.baseline_mms); ferr = norms.errors
    elif case == "p4p3_paper":
        H = vk.Hierarchy(4, 2, 2, forcing=vk.VK_F_PAPER_MMS); OH = th.THHierarchy(2, 4, 2, 2, 1.0, fields.paper_mms)
        ferr = norms.errors
    elif case == "p3p2_3d":
        H = vk.Hierarchy(2, 2, 2, dim=3, forcing=vk.VK_F_CUBE_MMS)
        OH = th.THHierarchy(3, 2, 2, 2, 1.0, fields.cube_mms); ferr = norms.errors
    else:
        H = vk.Hierarchy(3, 2, 2, family=vk.VK_SV); OH = sv.SVHierarchy(3, 2, 2, 1.0, fields.baseline_mms)
        ferr = lambda L, x: sv.errors(L, x)[:2]
    L = OH.finest
    z = L.nullvec()
    b = solve.consistent_rhs(L)
    Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    x = spla.spsolve(Kb, np.concatenate([b, [0.0]]))[: L.N]
    rng = np.random.default_rng(2)
    for v in (x, x + 0.05 * rng.standard_normal(L.N)):
        got = H.solution_errors(v)
        ref = ferr(L, v)
        print(case, got, ref)
        assert abs(got[0] - ref[0]) <= 1e-11 * ref[0] + 1e-15
        assert abs(got[1] - ref[1]) <= 1e-11 * ref[1] + 1e-15
    with pytest.raises(vk.VkError):
        vk.Hierarchy(2, 2, 2, forcing=vk.VK_F_RANDOM, coeffs=np.ones((2, 2, 2))).solution_errors(np.zeros(10))


@pytest.mark.parametrize("k,n0,nl", [(2, 4, 3), (3, 2, 3), (5, 2, 2), (7, 2, 2), (8, 2, 2)])
def test_host_assembly_quad_matches_oracle(k, n0, nl):
    """Quadrilateral Taylor-Hood: the library's host assembly, transfers and patches against the
    oracle's (independent tensor bases and point location)."""
    from oracle import qk
    H = vk.Hierarchy(k, n0, nl, family=vk.VK_TH_QUAD)
    OH = qk.QKHierarchy(k, n0, nl, 1.0, fields.baseline_mms)
    for l in range(nl):
        ol = OH.levels[l]
        inf = H.level_info(l)
        assert (inf.n_free, inf.nnz, inf.n_velocity) == (ol.N, ol.K.nnz, ol.nu_free)
        X, kind = H.dof_coords(l)
        OX, okind = ol.dof_coords()
        assert np.array_equal(kind, okind) and np.abs(X - OX).max() < 1e-15
        rp, col, val = H.csr(l)
        assert np.array_equal(rp, ol.K.indptr) and np.array_equal(col, ol.K.indices)
        rowmax = np.maximum.reduceat(np.abs(ol.K.data), ol.K.indptr[:-1])
        assert np.all(np.abs(val - ol.K.data) <= _asm_bound(ol) * np.finfo(float).eps * np.repeat(rowmax, np.diff(ol.K.indptr)))
        if l > 0:
            prp, pcol, pval = H.prolongation(l)
            P = OH.P[l]
            assert np.array_equal(prp, P.indptr) and np.array_equal(pcol, P.indices)
            assert np.abs(pval - P.data).max() <= 1e-14
            ptr, dofs = H.patches(l)
            op = patches.build_patches(ol)
            assert [list(dofs[ptr[i]:ptr[i + 1]]) for i in range(len(op))] == [list(I) for I in op]
    b = H.rhs()
    ob = solve.consistent_rhs(OH.finest)
    assert np.abs(b - ob).max() <= 1e-13 * np.abs(ob).max()


def test_quad_errors_and_limits():
    from oracle import qk
    H = vk.Hierarchy(3, 2, 2, family=vk.VK_TH_QUAD, forcing=vk.VK_F_PAPER_MMS)
    OH = qk.QKHierarchy(3, 2, 2, 1.0, fields.paper_mms)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(OH.finest.N) * 0.01
    got, ref = H.solution_errors(x), norms.errors(OH.finest, x)
    assert abs(got[0] - ref[0]) <= 1e-11 * ref[0] and abs(got[1] - ref[1]) <= 1e-11 * ref[1]
    for kw in ({"k": 9}, {"k": 2, "dim": 3}, {"k": 3, "construct": vk.VK_PATCH_STAR}):
        k = kw.pop("k")
        with pytest.raises(vk.VkError) as e:
            vk.Hierarchy(k, 2, 2, family=vk.VK_TH_QUAD, **kw)
        assert e.value.code == vk.VK_EINVAL


@pytest.mark.parametrize("k,n0,nl", [(1, 2, 3), (2, 2, 3), (4, 2, 2), (8, 1, 2)])
def test_host_assembly_bdm_matches_oracle(k, n0, nl):
    """(BDM_k, dP_{k-1}) with interior penalty: the library's dual bases, edge terms, transfers and
    extended patches against the oracle's (independent dual-basis construction: Gauss-Jordan on a
    Lagrange local space versus numpy's inverse, and its own Gram-Schmidt of the interior tests)."""
    from oracle import bdm
    H = vk.Hierarchy(k, n0, nl, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS)
    OH = bdm.BDMHierarchy(k, n0, nl, 1.0, fields.paper_mms)
    # entries carry the rounding of two dual-basis inversions (condition growing with k)
    tol = 1e-14 * k * k
    for l in range(nl):
        ol = OH.levels[l]
        inf = H.level_info(l)
        assert (inf.n_free, inf.nnz, inf.n_velocity) == (ol.N, ol.K.nnz, ol.nu_free)
        rp, col, val = H.csr(l)
        assert np.array_equal(rp, ol.K.indptr) and np.array_equal(col, ol.K.indices)
        rowmax = np.maximum.reduceat(np.abs(ol.K.data), ol.K.indptr[:-1])
        assert np.all(np.abs(val - ol.K.data) <= tol * np.repeat(rowmax, np.diff(ol.K.indptr)))
        X, kind = H.dof_coords(l)
        assert np.array_equal(kind, np.where(np.arange(ol.N) < ol.nu_free, 0, 2))
        if l > 0:
            prp, pcol, pval = H.prolongation(l)
            P = OH.P[l]
            assert np.array_equal(prp, P.indptr) and np.array_equal(pcol, P.indices)
            assert np.abs(pval - P.data).max() <= tol
            ptr, dofs = H.patches(l)
            op = patches.build_patches(ol)
            assert [list(dofs[ptr[i]:ptr[i + 1]]) for i in range(len(op))] == [list(I) for I in op]
    b = H.rhs()
    ob = solve.consistent_rhs(OH.finest)
    assert np.abs(b - ob).max() <= tol * np.abs(ob).max()
    rng = np.random.default_rng(k)
    x = rng.standard_normal(OH.finest.N) * 0.01
    got, ref = H.solution_errors(x), bdm.errors(OH.finest, x)
    assert abs(got[0] - ref[0]) <= 1e-11 * ref[0] and abs(got[1] - ref[1]) <= 1e-11 * ref[1]


def test_bdm_invalid_combinations_are_rejected():
    for kw in ({"k": 9}, {"k": 0}, {"k": 2, "forcing": vk.VK_F_BASELINE_MMS},
               {"k": 2, "construct": vk.VK_PATCH_COMPOSITE}, {"k": 2, "dim": 3}, {"k": 2, "penalty": -1.0}):
        k = kw.pop("k")
        kw.setdefault("forcing", vk.VK_F_PAPER_MMS)
        with pytest.raises(vk.VkError) as e:
            vk.Hierarchy(k, 2, 2, family=vk.VK_BDM, **kw)
        assert e.value.code == vk.VK_EINVAL
    with pytest.raises(vk.VkError):
        vk.Hierarchy(2, 2, 2, construct=vk.VK_PATCH_EXTENDED)
    # an explicit penalty reaches the edge terms: K changes, the volume-only pressure rows do not
    H0 = vk.Hierarchy(2, 2, 2, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS)
    H1 = vk.Hierarchy(2, 2, 2, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS, penalty=40.0)
    from oracle import bdm
    O1 = bdm.BDMLevel(2, 4, 1.0, fields.paper_mms(1.0), alpha=40.0)
    rp, col, val = H1.csr(1)
    assert np.abs(val - O1.K.data).max() <= 1e-12 * np.abs(O1.K.data).max()
    assert np.abs(H0.csr(1)[2] - val).max() > 1.0


@pytest.mark.parametrize("case", ["p4p3", "sv", "bdm2", "p2p1_3d"])
def test_union_groups_hold_k_exactly(case):
    """K's union groups (the layout of the K products of more than 8 right-hand sides): every row
    in exactly one group of at most 16 rows, the rows of a group in blocks of consecutive rows with
    identical column lists, the listed columns the ascending union of the rows' columns padded to
    a multiple of 16 by its last column, at most 96 of them unless the group is one block, at most
    twice the group's nonzeros stored, and the dense [step][row][4] blocks holding exactly K's
    entries with zeros elsewhere, so that the blocks reproduce K X."""
    kw = {"p4p3": dict(k=4, n0=2, nl=3), "sv": dict(k=3, n0=2, nl=3, family=vk.VK_SV),
          "bdm2": dict(k=2, n0=2, nl=3, family=vk.VK_BDM, forcing=vk.VK_F_PAPER_MMS),
          "p2p1_3d": dict(k=2, n0=2, nl=2, dim=3, forcing=vk.VK_F_CUBE_MMS)}[case]
    k, n0, nl = kw.pop("k"), kw.pop("n0"), kw.pop("nl")
    H = vk.Hierarchy(k, n0, nl, **kw)
    rng = np.random.default_rng(7)
    for l in range(1, nl):
        rp, col, val = H.csr(l)
        N = len(rp) - 1
        K = _csr_matrix(rp, col, val, N, N)
        gptr, grow, uptr, ucol, voff, gval = H.union_groups(l)
        assert np.array_equal(np.sort(grow), np.arange(N))
        X = rng.standard_normal((N, 3))
        Y = np.zeros((N, 3))
        off = 0
        for g in range(len(gptr) - 1):
            rows = grow[gptr[g]:gptr[g + 1]]
            G = len(rows)
            u = ucol[uptr[g]:uptr[g + 1]]
            assert 1 <= G <= 16 and len(u) % 16 == 0 and voff[g] == off
            U = len(np.unique(u))
            assert np.all(np.diff(u[:U]) > 0) and np.all(u[U:] == u[U - 1])
            cols = [col[rp[r]:rp[r + 1]] for r in rows]
            assert np.array_equal(u[:U], np.unique(np.concatenate(cols)))
            # blocks of consecutive rows with identical column lists
            blocks = 1 + sum(1 for a, b, ca, cb in zip(rows, rows[1:], cols, cols[1:])
                             if b != a + 1 or not np.array_equal(ca, cb))
            assert U <= 96 or blocks == 1
            nnz = sum(len(c) for c in cols)
            assert G * U <= 2 * nnz
            blk = gval[off:off + G * len(u)].reshape(len(u) // 4, G, 4)
            dense = blk.transpose(1, 0, 2).reshape(G, len(u))
            ref = np.zeros((G, len(u)))
            for t, r in enumerate(rows):
                pos = np.searchsorted(u[:U], col[rp[r]:rp[r + 1]])
                ref[t, pos] = val[rp[r]:rp[r + 1]]
            assert np.array_equal(dense, ref)
            Y[rows] = dense @ X[u]
            off += G * len(u)
        assert off == len(gval)
        m = np.diff(rp)[:, None]
        assert np.all(np.abs(Y - K @ X) <= 2 * (m + 2) * np.finfo(float).eps * (abs(K) @ np.abs(X)))
