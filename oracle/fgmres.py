"""Right-preconditioned flexible GMRES (oracle), Sec. 3 and Sec. 4.

The paper uses FGMRES because it stores the preconditioned Arnoldi vectors
z_j = M(v_j), so the update x += Z y needs no extra preconditioner
application.  Settings of Sec. 4: x_0 = 0, stop when the Euclidean norm of
the residual has dropped by 1e10 relative to the initial one, at most 100
iterations.  The restart length is a parameter (30 for the workloads here,
"unrestarted" = restart >= maxit).

Orthogonalisation (not specified in the paper): classical Gram-Schmidt
applied twice (CGS2).  The least-squares problem is updated by Givens
rotations; |g_{j+1}| is the residual-norm estimate used as stopping test.
At a restart the true residual b - K x is recomputed.  On exit the constant
pressure component is removed from x (x <- x - (z.x) z; K z = 0) and the
true residual is checked again; if it is above tolerance and iterations
remain, the method restarts.
"""
import numpy as np


def fgmres(K, b, precond, restart=30, rtol=1e-10, maxit=100, nullvec=None):
    N = len(b)
    x = np.zeros(N)
    bnorm = np.linalg.norm(b)
    its = 0
    history = [bnorm]
    if bnorm == 0.0:
        return x, 0, history, True
    r = b.copy()
    converged = False
    while True:
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            converged = True
            break
        if its >= maxit:
            break
        m = restart
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        jlast = -1
        for j in range(m):
            Z[j] = precond(V[j])
            w = K @ Z[j]
            h = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0.0:
                V[j + 1] = w / hn
            for i in range(j):
                a, c_ = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c_
                H[i + 1, j] = -sn[i] * a + cs[i] * c_
            a, c_ = H[j, j], H[j + 1, j]
            den = np.hypot(a, c_)
            cs[j], sn[j] = a / den, c_ / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            jlast = j
            history.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * bnorm or its >= maxit or hn == 0.0:
                break
        n = jlast + 1
        y = np.zeros(n)
        for i in reversed(range(n)):
            y[i] = (g[i] - H[i, i + 1:n] @ y[i + 1:n]) / H[i, i]
        x = x + Z[:n].T @ y
        if nullvec is not None:
            x = x - (nullvec @ x) * nullvec
        r = b - K @ x
    return x, its, history, converged
