"""Chebyshev-accelerated additive Vanka relaxation (oracle), Sec. 3.

Sec. 3 (the relaxation component of the V-cycle) accelerates the additive
Vanka sweeps with the Chebyshev iteration.  The interval is [lambda / 4,
1.1 lambda], lambda an estimate of the largest eigenvalue of the
relaxation-preconditioned operator B K on the level, obtained from GMRES:
the lower bound leaves the lowest quarter of the spectrum to the coarse-grid
correction, the factor 1.1 is a safety margin.

Readings (the paper leaves them open):
* B = W sum_i R_i^T K_i^{-1} R_i, the additive patch sum with the weights of
  the damped sweep (1 / multiplicity, or none); the damping omega plays no role.
* lambda = the largest real part of the Ritz values of `steps` (10) Arnoldi
  steps (CGS2) on B K from a pseudo-random start vector: entry i of level l is
  2 u - 1 with u the 53-bit uniform from the counter-based SplitMix64 value
  mix(seed + l * 0xD1B54A32D192ED03 + (i + 1) * 0x9E3779B97F4A7C15), where mix
  is the SplitMix64 output function (Steele, Lea and Flood 2014; the constants
  of Vigna's reference splitmix64).
* One Chebyshev sweep sequence of nu steps for K x = b (Saad, Iterative
  Methods for Sparse Linear Systems, the preconditioned Chebyshev iteration):
    theta = (a + c) / 2, delta = (c - a) / 2, sigma = theta / delta, rho = 1 / sigma
    r = b - K x;  d = B r / theta;  x += d
    repeat nu - 1 times:
      rho' = 1 / (2 sigma - rho);  r = b - K x
      d = rho' rho d + (2 rho' / delta) B r;  x += d;  rho = rho'
  so the error after nu steps is T_nu((theta - B K) / delta) / T_nu(theta / delta)
  applied to the initial error (T_nu the Chebyshev polynomial of the first kind).
"""
import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
LEVEL_STRIDE = 0xD1B54A32D192ED03


def splitmix64_mix(z):
    """The SplitMix64 output function of a 64-bit state (Python integers)."""
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def start_vector(n, seed, level):
    """Entries 2 u - 1, u = (mix(seed + level * S + (i + 1) * GAMMA) >> 11) / 2^53."""
    base = (seed + level * LEVEL_STRIDE) & MASK
    out = np.empty(n)
    for i in range(n):
        u = (splitmix64_mix(base + (i + 1) * GAMMA) >> 11) * 2.0 ** -53
        out[i] = 2.0 * u - 1.0
    return out


def arnoldi_lambda(K, B, v0, steps=10):
    """Largest real part of the Ritz values of `steps` Arnoldi steps on B K (CGS2)."""
    V = [v0 / np.linalg.norm(v0)]
    H = np.zeros((steps + 1, steps))
    k = steps
    for j in range(steps):
        w = B(K @ V[j])
        for _ in range(2):
            h = np.array([v @ w for v in V])
            w = w - sum(hh * v for hh, v in zip(h, V))
            H[: j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= 1e-14 * np.abs(H[: j + 1, j]).max():
            k = j + 1
            break
        V.append(w / H[j + 1, j])
    return float(np.linalg.eigvals(H[:k, :k]).real.max())


class ChebyshevVanka:
    """nu Chebyshev steps on [lam / 4, 1.1 lam] preconditioned by the additive patch sum."""

    def __init__(self, vanka, lam):
        self.v, self.K, self.lam = vanka, vanka.K, lam
        a, c = lam / 4.0, 1.1 * lam
        self.theta, self.delta = (a + c) / 2.0, (c - a) / 2.0

    def B(self, r):
        return self.v.weight * self.v.correction(r)

    def sweeps(self, b, x, nu):
        if nu == 0:
            return x
        theta, delta = self.theta, self.delta
        sigma = theta / delta
        rho = 1.0 / sigma
        d = self.B(b - self.K @ x) / theta
        x = x + d
        for _ in range(nu - 1):
            rho_n = 1.0 / (2.0 * sigma - rho)
            d = rho_n * rho * d + (2.0 * rho_n / delta) * self.B(b - self.K @ x)
            x = x + d
            rho = rho_n
        return x
