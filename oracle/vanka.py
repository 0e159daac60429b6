"""Additive Vanka relaxation (oracle): Algorithm 1 of Sec. 3.1 used as a smoother.

Algorithm 1 (additive / parallel subspace correction) solves, for every
patch i, the local saddle-point problem restricted to the patch's subspace
with the current global residual as data, and then adds the weighted sum of
all local corrections to the iterate.  In matrix form, with R_i the 0/1
restriction to the DoF list I_i and K_i = R_i K R_i^T the patch submatrix
taken from the assembled global matrix (the matrix-full approach of Sec. 3.1):

    r = b - K x
    x <- x + omega * sum_i w_i R_i^T K_i^{-1} R_i r

Reading of the weighting operators w_i, gamma_i (the paper lists them as
inputs of Algorithm 1 but never states them): every DoF d is scaled by
1 / mult(d), where mult(d) is the number of patches that contain d
("multiplicity" weighting, a diagonal operator restricted to each patch), and
a single global damping omega (0.5 by default) multiplies the sum:

    x <- x + omega * W * sum_i R_i^T K_i^{-1} R_i r,   W = diag(1 / mult).

With the identity weights ("none") and omega = 0.5 the largest eigenvalue of
omega M^{-1} K is close to 4 for P2-P1 vertex patches (velocity DoFs lie in up
to seven patches), so the unweighted sweep amplifies error; the multiplicity
weights bring the spectrum of W M^{-1} K into (0, 2].  The sum runs over
patches in ascending order.  K_i^{-1} is applied through an
LU factorisation with partial pivoting (K_i is symmetric indefinite with a
zero pressure block).
"""
import numpy as np
import scipy.linalg as sla


class AdditiveVanka:
    def __init__(self, K, patches, omega=0.5, weighting="multiplicity"):
        self.K = K
        self.patches = [np.asarray(I, dtype=np.int64) for I in patches]
        self.omega = omega
        mult = np.zeros(K.shape[0])
        for I in self.patches:
            mult[I] += 1.0
        self.mult = mult
        if weighting == "multiplicity":
            if np.any(mult == 0):
                raise ValueError("the patches do not cover every DoF")
            self.weight = 1.0 / mult
        elif weighting == "none":
            self.weight = np.ones_like(mult)
        else:
            raise ValueError(weighting)
        self.lu = []
        for I in self.patches:
            Ki = K[I][:, I].toarray()          # matrix-full extraction K[I_i, I_i]
            self.lu.append(sla.lu_factor(Ki, check_finite=True))

    def patch_matrix(self, i):
        I = self.patches[i]
        return self.K[I][:, I].toarray()

    def correction(self, r):
        """sum_i R_i^T K_i^{-1} R_i r, accumulated in ascending patch order."""
        delta = np.zeros_like(r)
        for I, lu in zip(self.patches, self.lu):
            delta[I] += sla.lu_solve(lu, r[I])
        return delta

    def sweep(self, b, x):
        r = b - self.K @ x
        return x + (self.omega * self.weight) * self.correction(r)

    def dense_operator(self):
        """sum_i R_i^T K_i^{-1} R_i as a dense matrix (small problems only; no W, no omega)."""
        N = self.K.shape[0]
        M = np.zeros((N, N))
        for I, lu in zip(self.patches, self.lu):
            Kinv = sla.lu_solve(lu, np.eye(len(I)))
            M[np.ix_(I, I)] += Kinv
        return M
