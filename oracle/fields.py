"""Exact solutions and forcing fields used by the oracle.

For a divergence-free u whose components are eigenfunctions of -Laplace
with eigenvalue lam and p = 0, the Stokes momentum equation (Sec. 2, the
strain-rate form) gives f = -div(2 nu eps(u)) = -nu Laplace(u) = nu lam u.
"""
import numpy as np

PI = np.pi


class Field:
    """u(x) -> (npts, dim), p(x) -> (npts,), f(x) -> (npts, dim), grad_u(x) -> (npts, dim, dim)."""

    def __init__(self, dim, u, p, f, grad_u, homogeneous=False):
        self.dim, self.u, self.p, self.f, self.grad_u = dim, u, p, f, grad_u
        self.homogeneous = homogeneous


def baseline_mms(nu):
    """u = (sin(pi x) sin(pi y), cos(pi x) cos(pi y)), p = 0, f = 2 nu pi^2 u."""
    def u(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([np.sin(PI * X) * np.sin(PI * Y), np.cos(PI * X) * np.cos(PI * Y)], 1)

    def gu(x):
        X, Y = x[:, 0], x[:, 1]
        g = np.empty((len(X), 2, 2))
        g[:, 0, 0] = PI * np.cos(PI * X) * np.sin(PI * Y)
        g[:, 0, 1] = PI * np.sin(PI * X) * np.cos(PI * Y)
        g[:, 1, 0] = -PI * np.sin(PI * X) * np.cos(PI * Y)
        g[:, 1, 1] = -PI * np.cos(PI * X) * np.sin(PI * Y)
        return g

    return Field(2, u, lambda x: np.zeros(len(x)), lambda x: 2.0 * nu * PI * PI * u(x), gu)


def paper_mms(nu):
    """The paper's field (Sec. 4, model problem): u = (sin(pi x) cos(pi y), -cos(pi x) sin(pi y)), p = 0."""
    def u(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([np.sin(PI * X) * np.cos(PI * Y), -np.cos(PI * X) * np.sin(PI * Y)], 1)

    def gu(x):
        X, Y = x[:, 0], x[:, 1]
        g = np.empty((len(X), 2, 2))
        g[:, 0, 0] = PI * np.cos(PI * X) * np.cos(PI * Y)
        g[:, 0, 1] = -PI * np.sin(PI * X) * np.sin(PI * Y)
        g[:, 1, 0] = PI * np.sin(PI * X) * np.sin(PI * Y)
        g[:, 1, 1] = -PI * np.cos(PI * X) * np.cos(PI * Y)
        return g

    return Field(2, u, lambda x: np.zeros(len(x)), lambda x: 2.0 * nu * PI * PI * u(x), gu)


def cube_mms(nu):
    """3D divergence-free field built from terms sin(pi a) cos(pi b), p = 0."""
    def u(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        s, c = np.sin, np.cos
        return np.stack([
            s(PI * X) * c(PI * Y) - s(PI * X) * c(PI * Z),
            s(PI * Y) * c(PI * Z) - c(PI * X) * s(PI * Y),
            s(PI * Z) * c(PI * X) - c(PI * Y) * s(PI * Z)], 1)

    def gu(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        s, c = np.sin, np.cos
        g = np.empty((len(X), 3, 3))
        g[:, 0, 0] = PI * c(PI * X) * c(PI * Y) - PI * c(PI * X) * c(PI * Z)
        g[:, 0, 1] = -PI * s(PI * X) * s(PI * Y)
        g[:, 0, 2] = PI * s(PI * X) * s(PI * Z)
        g[:, 1, 0] = PI * s(PI * X) * s(PI * Y)
        g[:, 1, 1] = PI * c(PI * Y) * c(PI * Z) - PI * c(PI * X) * c(PI * Y)
        g[:, 1, 2] = -PI * s(PI * Y) * s(PI * Z)
        g[:, 2, 0] = -PI * s(PI * Z) * s(PI * X)
        g[:, 2, 1] = PI * s(PI * Y) * s(PI * Z)
        g[:, 2, 2] = PI * c(PI * Z) * c(PI * X) - PI * c(PI * Y) * c(PI * Z)
        return g

    return Field(3, u, lambda x: np.zeros(len(x)), lambda x: 2.0 * nu * PI * PI * u(x), gu)


def poly_k2(nu):
    """u = (x^2, -2xy), p = x + y - 1: lies in (P2, P1), f = (1 - 2 nu, 1)."""
    def u(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([X * X, -2 * X * Y], 1)

    def gu(x):
        X, Y = x[:, 0], x[:, 1]
        g = np.zeros((len(X), 2, 2))
        g[:, 0, 0] = 2 * X
        g[:, 1, 0] = -2 * Y
        g[:, 1, 1] = -2 * X
        return g

    return Field(2, u, lambda x: x[:, 0] + x[:, 1] - 1.0,
                 lambda x: np.stack([np.full(len(x), 1 - 2 * nu), np.ones(len(x))], 1), gu)


def poly_k3(nu):
    """u = (2x^2 y + x^3, -2 x y^2 - 3 x^2 y) (the curl of x^2 y^2 + x^3 y), p = x^2 + x y - 7/12:
    lies in (P3, P2) and in (P3, dP2); f = -nu Laplace(u) + grad p."""
    def u(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([2 * X * X * Y + X ** 3, -2 * X * Y * Y - 3 * X * X * Y], 1)

    def gu(x):
        X, Y = x[:, 0], x[:, 1]
        g = np.zeros((len(X), 2, 2))
        g[:, 0, 0] = 4 * X * Y + 3 * X * X
        g[:, 0, 1] = 2 * X * X
        g[:, 1, 0] = -2 * Y * Y - 6 * X * Y
        g[:, 1, 1] = -4 * X * Y - 3 * X * X
        return g

    def f(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([(2 - 6 * nu) * X + (1 - 4 * nu) * Y, (1 + 4 * nu) * X + 6 * nu * Y], 1)

    return Field(2, u, lambda x: x[:, 0] ** 2 + x[:, 0] * x[:, 1] - 7.0 / 12.0, f, gu)


def with_gradient(field, psi, grad_psi):
    """The same velocity with the pressure p + psi: f gains grad psi (Sec. 2, pressure robustness)."""
    return Field(field.dim, field.u, lambda x: field.p(x) + psi(x), lambda x: field.f(x) + grad_psi(x),
                 field.grad_u, field.homogeneous)


def poly_k4(nu):
    """u = (2 x^3 y, -3 x^2 y^2), p = x^3 - 1/4: lies in (P4, P3)."""
    def u(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([2 * X ** 3 * Y, -3 * X ** 2 * Y ** 2], 1)

    def gu(x):
        X, Y = x[:, 0], x[:, 1]
        g = np.zeros((len(X), 2, 2))
        g[:, 0, 0] = 6 * X ** 2 * Y
        g[:, 0, 1] = 2 * X ** 3
        g[:, 1, 0] = -6 * X * Y ** 2
        g[:, 1, 1] = -6 * X ** 2 * Y
        return g

    def f(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([-12 * nu * X * Y + 3 * X ** 2, 6 * nu * (X ** 2 + Y ** 2)], 1)

    return Field(2, u, lambda x: x[:, 0] ** 3 - 0.25, f, gu)


def poly_3d_k2(nu):
    """u = (x^2, -2xy, 0), p = x + y + z - 3/2: lies in (P2, P1) in 3D, f = (1 - 2 nu, 1, 1)."""
    def u(x):
        X, Y = x[:, 0], x[:, 1]
        return np.stack([X * X, -2 * X * Y, np.zeros(len(X))], 1)

    def gu(x):
        X, Y = x[:, 0], x[:, 1]
        g = np.zeros((len(X), 3, 3))
        g[:, 0, 0] = 2 * X
        g[:, 1, 0] = -2 * Y
        g[:, 1, 1] = -2 * X
        return g

    return Field(3, u, lambda x: x[:, 0] + x[:, 1] + x[:, 2] - 1.5,
                 lambda x: np.stack([np.full(len(x), 1 - 2 * nu), np.ones(len(x)), np.ones(len(x))], 1), gu)


def random_sine_field(coeffs, nu=1.0):
    """Smooth random forcing f_c = sum_{a,b=1..M} g[c,a-1,b-1] sin(a pi x) sin(b pi y) / (a^2 + b^2).

    ``coeffs`` has shape (2, M, M) and is drawn by the seeded input generator
    (the oracle draws no random numbers itself).  Homogeneous Dirichlet data;
    the exact solution is unknown (u, p, grad_u return None).
    """
    coeffs = np.asarray(coeffs, dtype=float)
    M = coeffs.shape[1]

    def f(x):
        X, Y = x[:, 0], x[:, 1]
        out = np.zeros((len(X), 2))
        for c in range(2):
            for a in range(1, M + 1):
                for b in range(1, M + 1):
                    out[:, c] += coeffs[c, a - 1, b - 1] * np.sin(a * PI * X) * np.sin(b * PI * Y) / (a * a + b * b)
        return out

    zero_u = lambda x: np.zeros((len(x), 2))
    return Field(2, zero_u, lambda x: np.zeros(len(x)), f, None, homogeneous=True)
