"""Taylor-Hood (P_k, P_{k-1}) discretisation of the Stokes problem (oracle).

What is assembled (Sec. 2, the variational formulation and its discrete
form; Sec. 3, the per-level saddle-point matrix):

  a(u, v) = 2 nu int eps(u) : eps(v),   b(v, q) = - int (div v) q,
  <f, v>  = int f . v,

  K = [[A, B^T], [B, 0]] on the free (non-Dirichlet) DoFs, symmetric.

For u = phi_j e_d (trial) and v = phi_i e_c (test) the strain-rate form
reduces to  A[(i,c),(j,d)] = nu int (delta_cd grad phi_i . grad phi_j
+ d_d phi_i d_c phi_j),  and  B[q,(j,d)] = - int d_d phi_j psi_q.

Dirichlet data (the velocity on the boundary) are nodal interpolants of the
exact velocity; boundary velocity DoFs are eliminated and their coupling is
moved to the right-hand side (lifting).  The pressure is continuous with no
boundary condition; K has the constant pressure (0, 1) in its kernel.

DoF numbering of the free system (documented so that an independent
implementation can reproduce it): velocity lattice points (A, B[, C]) of the
P_k lattice of spacing 1/(k n), interior points only, lexicographic with x
fastest, components interleaved (dof = dim * idx + c); then all pressure
lattice points of the P_{k-1} lattice, lexicographic with x fastest.

The matrix pattern is the element closure: every pair of DoFs that share a
cell is stored (exact zeros included), except pressure-pressure pairs.
"""
import numpy as np
import scipy.sparse as sp

from . import lagrange, mesh, quad


class THLevel:
    def __init__(self, dim, k, n, nu, field):
        self.dim, self.k, self.n, self.nu = dim, k, n, nu
        self.cells = mesh.cells(dim, n)
        self.vb = lagrange.LagrangeBasis(dim, k)
        self.pb = lagrange.LagrangeBasis(dim, k - 1)
        self.Mv = k * n              # velocity lattice has Mv + 1 points per direction
        self.Mp = (k - 1) * n        # pressure lattice
        self.n_vel_nodes_int = (self.Mv - 1) ** dim
        self.nu_free = dim * self.n_vel_nodes_int
        self.np_ = (self.Mp + 1) ** dim
        self.N = self.nu_free + self.np_
        self.field = field
        self._assemble()

    # ---- numbering -------------------------------------------------------
    def vel_index(self, G):
        """Interior index of a velocity lattice point, or -1 on the boundary."""
        M = self.Mv
        if any(g <= 0 or g >= M for g in G):
            return -1
        idx = 0
        for d in reversed(range(self.dim)):
            idx = idx * (M - 1) + (G[d] - 1)
        return idx

    def p_dof(self, G):
        M = self.Mp
        idx = 0
        for d in reversed(range(self.dim)):
            idx = idx * (M + 1) + G[d]
        return self.nu_free + idx

    def cell_nodes(self, cell, kk):
        """Global lattice points (spacing 1/(kk n)) of the local P_kk nodes of a cell."""
        v0 = np.array(cell[0])
        E = [np.array(cell[d + 1]) - v0 for d in range(self.dim)]
        out = []
        for a in lagrange.lattice_nodes(self.dim, kk):
            G = kk * v0 + sum(a[d] * E[d] for d in range(self.dim))
            out.append(tuple(int(g) for g in G))
        return out

    def quad_rule(self, q):
        """Quadrature on the reference cell with q Gauss points per direction."""
        return quad.simplex_rule(self.dim, q)

    def cell_geometry(self, cell):
        v0 = np.array(cell[0], dtype=float) / self.n
        J = np.stack([np.array(cell[d + 1], dtype=float) / self.n - v0 for d in range(self.dim)], axis=1)
        return v0, J

    # ---- assembly --------------------------------------------------------
    def element_matrices(self, cell):
        """Local A (velocity, index i*dim + c), B (pressure x velocity) and load F of one cell."""
        dim, k, nu = self.dim, self.k, self.nu
        qp, qw = self._rule
        v0, J = self.cell_geometry(cell)
        detJ = abs(np.linalg.det(J))
        Jinv = np.linalg.inv(J)
        gphys = self._Gv @ Jinv          # (nq, nbv, dim): grad_x phi = grad_xi phi J^{-1}
        w = qw * detJ
        nbv, nbp = self._Pv.shape[1], self._Pp.shape[1]
        lap = np.einsum("q,qid,qjd->ij", w, gphys, gphys)
        Aloc = np.zeros((nbv * dim, nbv * dim))
        for c in range(dim):
            for d in range(dim):
                cross = np.einsum("q,qi,qj->ij", w, gphys[:, :, d], gphys[:, :, c])
                Aloc[c::dim, d::dim] = nu * (cross + (lap if c == d else 0.0))
        Bloc = np.zeros((nbp, nbv * dim))
        for d in range(dim):
            Bloc[:, d::dim] = -np.einsum("q,qp,qj->pj", w, self._Pp, gphys[:, :, d])
        xq = v0[None, :] + qp @ J.T
        fq = self.field.f(xq)
        Floc = np.zeros(nbv * dim)
        for c in range(dim):
            Floc[c::dim] = np.einsum("q,q,qi->i", w, fq[:, c], self._Pv)
        return Aloc, Bloc, Floc

    def _assemble(self):
        dim, k = self.dim, self.k
        self._rule = self.quad_rule(k + 3)
        qp = self._rule[0]
        self._Gv = self.vb.grad(qp)
        self._Pp = self.pb.eval(qp)
        self._Pv = self.vb.eval(qp)
        nbv = self._Pv.shape[1]
        rows, cols, vals = [], [], []
        rhs = np.zeros(self.N)
        for cell in self.cells:
            Aloc, Bloc, Floc = self.element_matrices(cell)
            vnodes = self.cell_nodes(cell, k)
            pnodes = self.cell_nodes(cell, k - 1)
            vdof = np.empty(nbv * dim, dtype=np.int64)
            uD = np.zeros(nbv * dim)
            for i, G in enumerate(vnodes):
                idx = self.vel_index(G)
                for c in range(dim):
                    vdof[i * dim + c] = dim * idx + c if idx >= 0 else -1
                if idx < 0:
                    x = np.array(G, dtype=float)[None, :] / self.Mv
                    uD[i * dim:(i + 1) * dim] = self.field.u(x)[0]
            pdof = np.array([self.p_dof(G) for G in pnodes], dtype=np.int64)
            free = vdof >= 0
            fv = vdof[free]
            rr, cc = np.meshgrid(fv, fv, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(Aloc[np.ix_(free, free)].ravel())
            rr, cc = np.meshgrid(pdof, fv, indexing="ij")
            Bf = Bloc[:, free]
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(Bf.ravel())
            rows.append(cc.ravel()); cols.append(rr.ravel()); vals.append(Bf.ravel())
            # right-hand side with Dirichlet lifting
            rhs[fv] += Floc[free] - Aloc[np.ix_(free, ~free)] @ uD[~free]
            rhs[pdof] += -Bloc[:, ~free] @ uD[~free]
        rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
        K = sp.coo_matrix((vals, (rows, cols)), shape=(self.N, self.N)).tocsr()
        K.sum_duplicates()
        K.sort_indices()
        self.K = K
        self.b = rhs

    # ---- geometry of the free DoFs ----------------------------------------
    def dof_coords(self):
        """(N, dim) coordinates and (N,) kind (0..dim-1 velocity component, dim = pressure)."""
        X = np.zeros((self.N, self.dim))
        kind = np.zeros(self.N, dtype=np.int64)
        M = self.Mv
        for idx in range(self.n_vel_nodes_int):
            G, r = [], idx
            for d in range(self.dim):
                G.append(r % (M - 1) + 1)
                r //= (M - 1)
            for c in range(self.dim):
                X[self.dim * idx + c] = np.array(G, dtype=float) / M
                kind[self.dim * idx + c] = c
        Mp = self.Mp
        for idx in range(self.np_):
            G, r = [], idx
            for d in range(self.dim):
                G.append(r % (Mp + 1))
                r //= (Mp + 1)
            X[self.nu_free + idx] = np.array(G, dtype=float) / Mp
            kind[self.nu_free + idx] = self.dim
        return X, kind

    def nullvec(self):
        """z = (0, 1_p) / sqrt(m): the normalised constant pressure."""
        z = np.zeros(self.N)
        z[self.nu_free:] = 1.0 / np.sqrt(self.np_)
        return z


def prolongation(coarse, fine):
    """P = diag(P^V, P^Q): nodal interpolation of the coarse basis at fine nodes (Sec. 3, grid transfers).

    Row r (fine free DoF), column s (coarse free DoF): phi_s^coarse(x_r).
    Point location is generic: for each coarse cell, every fine lattice point
    inside its closure is evaluated there; a row is filled by the first cell
    that contains the point.  Entries with |value| < 1e-12 are exact zeros of
    the rational interpolation weights and are dropped.
    """
    dim = fine.dim
    rows, cols, vals = [], [], []
    for kind, kk, cb, fM in (("v", coarse.k, coarse.vb, fine.Mv), ("p", coarse.k - 1, coarse.pb, fine.Mp)):
        filled = set()
        for cell in coarse.cells:
            v0, J = coarse.cell_geometry(cell)
            Jinv = np.linalg.inv(J)
            cnodes = coarse.cell_nodes(cell, kk)
            verts = np.array(cell, dtype=float) / coarse.n
            lo = np.floor(verts.min(0) * fM + 1e-9).astype(int)
            hi = np.ceil(verts.max(0) * fM - 1e-9).astype(int)
            grids = np.meshgrid(*[np.arange(lo[d], hi[d] + 1) for d in range(dim)], indexing="ij")
            pts = np.stack([g.ravel() for g in grids], 1)
            xi = (pts / fM - v0[None, :]) @ Jinv.T
            lam = np.concatenate([1.0 - xi.sum(1, keepdims=True), xi], 1)
            inside = np.all(lam >= -1e-12, axis=1)
            pts, xi = pts[inside], xi[inside]
            phi = cb.eval(xi)
            for p_i, G in enumerate(pts):
                G = tuple(int(g) for g in G)
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
                        for c in range(dim):
                            rows.append(dim * fidx + c); cols.append(dim * cidx + c); vals.append(val)
                    else:
                        rows.append(fdof); cols.append(coarse.p_dof(CG)); vals.append(val)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(fine.N, coarse.N)).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    return P


class THHierarchy:
    """Levels 0 (coarsest, n0) .. L-1 (finest, n0 * 2^(L-1)), rediscretised on every level (Sec. 3)."""

    def __init__(self, dim, k, n0, nlevels, nu, field_factory):
        self.dim, self.k = dim, k
        self.levels = []
        for l in range(nlevels):
            n = n0 * 2 ** l
            self.levels.append(THLevel(dim, k, n, nu, field_factory(nu)))
        self.P = [None] + [prolongation(self.levels[l - 1], self.levels[l]) for l in range(1, nlevels)]

    @property
    def finest(self):
        return self.levels[-1]
