"""Pins for the oracle's manufactured fields and random forcing (CPU only).

The fields are checked against the mathematics rather than against a retyped
copy of their formulas: gradients against central differences of u, the
divergence-free property pointwise, the forcing against -nu times a
finite-difference Laplacian (Sec. 2, the strain-rate Stokes system with p = 0),
the sine-series forcing against the orthogonality of the sine basis, and the
3D field through the O(h^2) convergence of the P2-P1 discretisation it drives
(Sec. 2, Taylor-Hood approximation order).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import fields, norms, th

H_FD = 1e-4


def _points(dim, n=200, seed=7):
    return np.random.default_rng(seed).uniform(0.05, 0.95, (n, dim))


def _fd_grad(F, x):
    """Central differences of u: g[:, c, d] = du_c / dx_d, error O(H_FD^2)."""
    g = np.empty((len(x), F.dim, F.dim))
    for d in range(F.dim):
        e = np.zeros(F.dim)
        e[d] = H_FD
        g[:, :, d] = (F.u(x + e) - F.u(x - e)) / (2 * H_FD)
    return g


def _fd_laplace(F, x, h=1e-3):
    lap = np.zeros((len(x), F.dim))
    for d in range(F.dim):
        e = np.zeros(F.dim)
        e[d] = h
        lap += (F.u(x + e) - 2 * F.u(x) + F.u(x - e)) / (h * h)
    return lap


FIELDS = [fields.baseline_mms, fields.paper_mms, fields.cube_mms]


@pytest.mark.parametrize("fac", FIELDS)
def test_gradient_matches_finite_differences(fac):
    F = fac(1.0)
    x = _points(F.dim)
    assert np.abs(F.grad_u(x) - _fd_grad(F, x)).max() <= 1e-6


@pytest.mark.parametrize("fac", FIELDS)
def test_field_is_divergence_free(fac):
    """div u = 0 pointwise, from finite differences of u (independent of grad_u) and from grad_u."""
    F = fac(1.0)
    x = _points(F.dim)
    assert np.abs(np.trace(_fd_grad(F, x), axis1=1, axis2=2)).max() <= 1e-6
    assert np.abs(np.trace(F.grad_u(x), axis1=1, axis2=2)).max() <= 1e-13


@pytest.mark.parametrize("fac", FIELDS)
@pytest.mark.parametrize("nu", [1.0, 0.3])
def test_forcing_is_minus_nu_laplacian(fac, nu):
    """With div u = 0 and p = 0: f = -div(2 nu eps(u)) = -nu Laplace(u)."""
    F = fac(nu)
    x = _points(F.dim)
    assert np.abs(F.p(x)).max() == 0.0
    ref = -nu * _fd_laplace(F, x)
    assert np.abs(F.f(x) - ref).max() <= 1e-4 * nu


def test_cube_field_has_nonzero_boundary_data_and_no_rigid_part():
    """The Dirichlet data of the 3D field is not trivial (a sign slip making u vanish on a face or
    everywhere would otherwise go unnoticed by the rate test's relative norm)."""
    F = fields.cube_mms(1.0)
    t = np.linspace(0.1, 0.9, 9)
    face = np.stack(np.meshgrid(t, t, indexing="ij"), -1).reshape(-1, 2)
    for d in range(3):
        for side in (0.0, 1.0):
            x = np.insert(face, d, side, axis=1)
            assert np.abs(F.u(x)).max() > 0.1


def _direct(L):
    z = L.nullvec()
    b = L.b - (z @ L.b) * z
    Kb = sp.bmat([[L.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[: L.N]


def test_cube_field_convergence_rate_3d():
    """3D P2-P1 on Kuhn meshes n = 4, 8 driven by the cube field: velocity H^1 error O(h^2), pressure
    L^2 error at least O(h^2) (it is still pre-asymptotic at these sizes, order 2.7). A sign slip in
    any term of u, grad u or f breaks the divergence-free forcing/solution pair and the rates."""
    errs = []
    for n in (4, 8):
        L = th.THLevel(3, 2, n, 1.0, fields.cube_mms(1.0))
        errs.append(norms.errors(L, _direct(L)))
    ru = np.log2(errs[0][0] / errs[1][0])
    rp = np.log2(errs[0][1] / errs[1][1])
    print(f"cube field: velocity H1 {errs[0][0]:.3e} -> {errs[1][0]:.3e} (order {ru:.2f}), "
          f"pressure L2 {errs[0][1]:.3e} -> {errs[1][1]:.3e} (order {rp:.2f})")
    assert abs(ru - 2) <= 0.25
    assert rp >= 1.75
    assert errs[1][0] <= 0.02 and errs[1][1] <= 0.03


def _sine_coefficients(F, M, nq=48):
    """c[c, a-1, b-1] = 4 (a^2 + b^2) int_0^1 int_0^1 f_c sin(a pi x) sin(b pi y): by the orthogonality
    of the sine basis this recovers the generating coefficients exactly (tensor Gauss-Legendre with
    nq points per direction integrates the trigonometric polynomials of degree <= 2M far below 1e-13)."""
    t, w = np.polynomial.legendre.leggauss(nq)
    t, w = 0.5 * (t + 1), 0.5 * w
    X, Y = np.meshgrid(t, t, indexing="ij")
    W = np.outer(w, w).ravel()
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    f = F.f(pts)
    out = np.empty((2, M, M))
    for a in range(1, M + 1):
        for b in range(1, M + 1):
            s = np.sin(a * np.pi * pts[:, 0]) * np.sin(b * np.pi * pts[:, 1])
            out[:, a - 1, b - 1] = 4 * (a * a + b * b) * (W * s) @ f
    return out


def test_random_sine_field_recovers_its_coefficients():
    """Non-symmetric random coefficients: a transposed (a, b), a swapped component or a wrong
    denominator changes the recovered coefficients."""
    g = synth.forcing_coeffs(31)
    F = fields.random_sine_field(g)
    assert np.abs(_sine_coefficients(F, 8) - g).max() <= 1e-12
    assert np.abs(F.u(_points(2))).max() == 0.0 and F.homogeneous


def test_random_sine_field_single_mode_closed_form():
    """One mode g[1, a-1, b-1] = 1 with (a, b) = (3, 2): f = (0, sin(3 pi x) sin(2 pi y) / 13), checked
    at the points where the sines are +-1 and 0, and its integral over the unit square,
    (1 - cos 3pi)(1 - cos 2pi) / (6 pi^2 13) = 0."""
    g = np.zeros((2, 8, 8))
    g[1, 2, 1] = 1.0
    F = fields.random_sine_field(g)
    x = np.array([[1 / 6, 1 / 4], [1 / 2, 1 / 4], [1 / 6, 3 / 4], [1 / 3, 1 / 4], [0.3, 0.0]])
    ref = np.array([1.0, -1.0, -1.0, 0.0, 0.0]) / 13.0
    assert np.abs(F.f(x)[:, 0]).max() == 0.0
    assert np.abs(F.f(x)[:, 1] - ref).max() <= 1e-15
    # odd-odd mode: nonzero integral 4 / (a b pi^2 (a^2 + b^2)) for (a, b) = (3, 1)
    g = np.zeros((2, 8, 8))
    g[0, 2, 0] = 1.0
    F = fields.random_sine_field(g)
    t, w = np.polynomial.legendre.leggauss(40)
    t, w = 0.5 * (t + 1), 0.5 * w
    X, Y = np.meshgrid(t, t, indexing="ij")
    integral = np.outer(w, w).ravel() @ F.f(np.stack([X.ravel(), Y.ravel()], 1))[:, 0]
    assert abs(integral - 4 / (3 * np.pi ** 2 * 10)) <= 1e-14


def test_random_forcing_load_sums_to_the_integral():
    """The velocity basis is a partition of unity, so the load entries of component c summed over all
    velocity nodes equal int f_c exactly.  The free (interior) nodes miss only the boundary-node
    functions, whose support is a strip of width O(h) where the sine forcing is itself O(h): the sum
    over free entries converges to the closed-form integral at O(h^2)."""
    g = np.zeros((2, 8, 8))
    g[0, 0, 0] = 1.0   # f_x = sin(pi x) sin(pi y) / 2, integral 2 / pi^2
    g[1, 2, 0] = 1.0   # f_y = sin(3 pi x) sin(pi y) / 10, integral 4 / (3 pi^2 10)
    exact = np.array([4 / np.pi ** 2 / 2, 4 / (3 * np.pi ** 2 * 10)])
    prev = None
    for n in (8, 16, 32):
        L = th.THLevel(2, 2, n, 1.0, fields.random_sine_field(g))
        X, kind = L.dof_coords()
        sums = np.array([L.b[kind == c].sum() for c in range(2)])
        err = np.abs(sums - exact).max()
        if prev is not None:
            assert err <= prev / 3.0
        prev = err
    assert prev <= 2e-3
