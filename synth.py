"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds none of the solver's arithmetic: only random draws.  Anything random that
the method consumes (test vectors, forcing coefficients) is drawn here and
handed, as plain arrays, to both the oracle and the GPU library.
"""
import numpy as np

SEED = 20240922


def vector(n, seed=SEED):
    """Standard-normal float64 vector of length n."""
    return np.random.default_rng(seed).standard_normal(n)


def forcing_coeffs(seed=SEED, modes=8, dim=2):
    """Coefficients g[c, a, b] ~ N(0, 1) of the smooth random forcing
    f_c = sum_{a,b=1..modes} g[c, a-1, b-1] sin(a pi x) sin(b pi y) / (a^2 + b^2)."""
    return np.random.default_rng(seed).standard_normal((dim, modes, modes))
