"""Taylor-Hood (Q_k, Q_{k-1}) on quadrilaterals (oracle), Sec. 2 and Sec. 3.1.

The quadrilateral Taylor-Hood pair: continuous vector Q_k velocities and
continuous Q_{k-1} pressures on the uniform n x n mesh of squares of the unit
square (Sec. 4 uses quadrilateral meshes next to the triangular ones; the
coarsest mesh is the same n0 x n0 grid, without the diagonal cut).  The
weak form, the Dirichlet lifting, the matrix pattern (the element closure
without pressure-pressure pairs) and the free-DoF numbering are those of the
triangular pair (oracle.th): the Q_k nodes of the square grid are exactly the
points of the P_k lattice of spacing 1/(k n), so both numberings coincide.

Basis: the tensor product of the 1D equispaced Lagrange polynomials of degree
kk on [0, 1],  l_a(t) = prod_{m != a} (kk t - m) / (a - m),  node (a, b) at
(a / kk, b / kk), ordered with a fastest.  Quadrature: the tensor
Gauss-Legendre rule of q points per direction (k + 3 for assembly).

Transfers (Sec. 3, grid transfers): nodal interpolation of the coarse Q_k /
Q_{k-1} functions at the fine nodes (the spaces are nested).

Patches (Sec. 3.1, composite Vanka): one patch per topological entity that
carries pressure DoFs of Q_{k-1} (vertices for every k >= 2; edge interiors,
k - 2 DoFs each, and cell interiors, (k - 2)^2 DoFs each, for k >= 3), with
every free velocity DoF on the closure of the entity's star: the up to four
squares around a vertex, the one or two squares of an edge, the square
itself.  DoF lists ascending, patches ordered by their smallest pressure DoF.
"""
import numpy as np
import scipy.sparse as sp

from . import quad, th


class TensorBasis:
    """Q_kk nodal basis on [0, 1]^2, the tensor product of 1D equispaced Lagrange polynomials."""

    def __init__(self, kk):
        self.k = kk
        self.lattice = [(a, b) for b in range(kk + 1) for a in range(kk + 1)]
        self.nodes = np.array(self.lattice, dtype=float) / kk

    def _1d(self, t):
        """Values and derivatives of l_0..l_kk at the points t: arrays (npts, kk + 1)."""
        kk = self.k
        t = np.asarray(t, dtype=float)
        V = np.ones((len(t), kk + 1))
        D = np.zeros((len(t), kk + 1))
        for a in range(kk + 1):
            for m in range(kk + 1):
                if m == a:
                    continue
                f = (kk * t - m) / (a - m)
                D[:, a] = D[:, a] * f + V[:, a] * (kk / (a - m))
                V[:, a] = V[:, a] * f
        return V, D

    def eval(self, x):
        x = np.atleast_2d(np.asarray(x, dtype=float))
        Vx, _ = self._1d(x[:, 0])
        Vy, _ = self._1d(x[:, 1])
        return np.stack([Vx[:, a] * Vy[:, b] for a, b in self.lattice], axis=1)

    def grad(self, x):
        x = np.atleast_2d(np.asarray(x, dtype=float))
        Vx, Dx = self._1d(x[:, 0])
        Vy, Dy = self._1d(x[:, 1])
        g = np.empty((x.shape[0], len(self.lattice), 2))
        for j, (a, b) in enumerate(self.lattice):
            g[:, j, 0] = Dx[:, a] * Vy[:, b]
            g[:, j, 1] = Vx[:, a] * Dy[:, b]
        return g


def square_rule(q):
    """Tensor Gauss-Legendre rule on [0, 1]^2: points (q*q, 2), weights summing to 1."""
    g, w = quad.gauss_legendre01(q)
    pts = np.array([(g[i], g[j]) for j in range(q) for i in range(q)])
    wts = np.array([w[i] * w[j] for j in range(q) for i in range(q)])
    return pts, wts


class QKLevel(th.THLevel):
    cell_type = "quad"

    def __init__(self, k, n, nu, field):
        self.dim, self.k, self.n, self.nu = 2, k, n, nu
        self.cells = [(i, j) for j in range(n) for i in range(n)]  # lower-left corner of each square
        self.vb = TensorBasis(k)
        self.pb = TensorBasis(k - 1)
        self.Mv = k * n
        self.Mp = (k - 1) * n
        self.n_vel_nodes_int = (self.Mv - 1) ** 2
        self.nu_free = 2 * self.n_vel_nodes_int
        self.np_ = (self.Mp + 1) ** 2
        self.N = self.nu_free + self.np_
        self.field = field
        self._assemble()

    def quad_rule(self, q):
        return square_rule(q)

    def cell_nodes(self, cell, kk):
        i, j = cell
        return [(kk * i + a, kk * j + b) for b in range(kk + 1) for a in range(kk + 1)]

    def cell_geometry(self, cell):
        i, j = cell
        return np.array([i, j], dtype=float) / self.n, np.eye(2) / self.n


def prolongation(coarse, fine):
    """P = diag(P^V, P^Q): the coarse basis of the square containing each fine node, evaluated there.

    A fine node on a coarse cell boundary takes the first square (in cell order) whose closure holds it;
    the continuous coarse functions agree there.  Exact zeros of the weights are dropped (|w| < 1e-12).
    """
    rows, cols, vals = [], [], []
    for kind, kk, cb, fM in (("v", coarse.k, coarse.vb, fine.Mv), ("p", coarse.k - 1, coarse.pb, fine.Mp)):
        filled = set()
        for cell in coarse.cells:
            v0, _ = coarse.cell_geometry(cell)
            cnodes = coarse.cell_nodes(cell, kk)
            r = fM // coarse.n  # fine lattice steps per coarse cell side
            lo = (cell[0] * r, cell[1] * r)
            pts = [(lo[0] + a, lo[1] + b) for b in range(r + 1) for a in range(r + 1)]
            xi = np.array([((G[0] / fM - v0[0]) * coarse.n, (G[1] / fM - v0[1]) * coarse.n) for G in pts])
            phi = cb.eval(xi)
            for p_i, G in enumerate(pts):
                if G in filled:
                    continue
                if kind == "v":
                    fidx = fine.vel_index(G)
                    if fidx < 0:
                        continue
                else:
                    fdof = fine.p_dof(G)
                filled.add(G)
                for j, CG in enumerate(cnodes):
                    val = phi[p_i, j]
                    if abs(val) < 1e-12:
                        continue
                    if kind == "v":
                        cidx = coarse.vel_index(CG)
                        if cidx < 0:
                            continue
                        for c in range(2):
                            rows.append(2 * fidx + c); cols.append(2 * cidx + c); vals.append(val)
                    else:
                        rows.append(fdof); cols.append(coarse.p_dof(CG)); vals.append(val)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(fine.N, coarse.N)).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    return P


class QKHierarchy:
    """Levels 0 (coarsest, n0) .. L-1 (finest, n0 * 2^(L-1)), rediscretised on every level."""

    def __init__(self, k, n0, nlevels, nu, field_factory):
        self.dim, self.k = 2, k
        self.levels = [QKLevel(k, n0 * 2 ** l, nu, field_factory(nu)) for l in range(nlevels)]
        self.P = [None] + [prolongation(self.levels[l - 1], self.levels[l]) for l in range(1, nlevels)]

    @property
    def finest(self):
        return self.levels[-1]


def build_patches(level):
    """Composite Vanka patches of a quadrilateral level (see the module docstring)."""
    k, n, kp = level.k, level.n, level.k - 1
    ent_pdofs = {}
    for gy in range(level.Mp + 1):
        for gx in range(level.Mp + 1):
            ix, rx = divmod(gx, kp)
            iy, ry = divmod(gy, kp)
            if rx == 0 and ry == 0:
                ent = ("v", ix, iy)
            elif ry == 0:
                ent = ("ex", ix, iy)  # horizontal edge: cell column ix on grid line iy
            elif rx == 0:
                ent = ("ey", ix, iy)  # vertical edge: grid line ix, cell row iy
            else:
                ent = ("c", ix, iy)
            ent_pdofs.setdefault(ent, []).append(level.p_dof((gx, gy)))

    def star_cells(ent):
        t, a, b = ent
        if t == "v":
            cand = [(a - 1, b - 1), (a, b - 1), (a - 1, b), (a, b)]
        elif t == "ex":
            cand = [(a, b - 1), (a, b)]
        elif t == "ey":
            cand = [(a - 1, b), (a, b)]
        else:
            cand = [(a, b)]
        return [c for c in cand if 0 <= c[0] < n and 0 <= c[1] < n]

    patches = []
    for ent, pd in ent_pdofs.items():
        vd = set()
        for cell in star_cells(ent):
            for G in level.cell_nodes(cell, k):
                idx = level.vel_index(G)
                if idx >= 0:
                    vd.update((2 * idx, 2 * idx + 1))
        patches.append(sorted(vd | set(pd)))
    patches.sort(key=lambda I: min(d for d in I if d >= level.nu_free))
    return patches
