"""Scott-Vogelius (P_k, dP_{k-1}) on barycentrically refined meshes (oracle).

The paper names the Scott-Vogelius pair in Sec. 2 (velocity continuous P_k,
pressure discontinuous piecewise P_{k-1}) and notes that in 2D it is
inf-sup stable for k >= 2 on meshes obtained by one barycentric refinement
of a triangulation; it does not run experiments with it.  This module builds
that discretisation with the forms of Sec. 2 (the same as for Taylor-Hood):

  a(u, v) = 2 nu int eps(u) : eps(v),   b(v, q) = - int (div v) q,
  <f, v>  = int f . v,   K = [[A, B^T], [B, 0]] on the free DoFs.

Mesh.  The macro mesh is the n x n two-triangle mesh of the unit square
(top-left to bottom-right diagonals).  Macro triangle (v0, v1, v2) with
barycentre c is split into the three sub-cells
  s = 0: (v0, v1, c),  s = 1: (v1, v2, c),  s = 2: (v2, v0, c),
and the finite-element spaces live on these sub-cells.  Coordinates are
integers in units of 1/(3n) (a barycentre (v0 + v1 + v2)/3 of lattice
vertices is on that lattice).

DoF numbering of the free system:
  velocity: every P_k node of the sub-cell mesh (a point of the lattice of
    spacing 1/(3 k n)) that is not on the boundary of the square, in
    lexicographic order of its lattice coordinates with x fastest, the two
    components interleaved (dof = 2 idx + c);
  pressure: sub-cell by sub-cell (macro triangle in mesh order, then s), and
    inside a sub-cell the P_{k-1} nodes in the order of their lattice
    multi-index (a1, a2) relative to (V0; V1 - V0, V2 - V0) of the sub-cell's
    vertex order above: dof = n_vel + (3 m + s) * nbp + j.

Matrix pattern: the sub-cell closure (every velocity-velocity and
velocity-pressure pair that shares a sub-cell; no pressure-pressure block).

Hierarchy.  Level l is the barycentric refinement of the uniformly refined
macro mesh n0 2^l.  These meshes are not nested (a fine sub-cell can cross
a coarse sub-cell's edge), so the transfers are defined pointwise:
  velocity: the coarse (continuous) P_k function evaluated at each fine
    velocity node, in a coarse sub-cell that contains the node;
  pressure: the L^2 projection of the coarse (discontinuous) pressure onto
    the fine dP_{k-1} space, which is local to each fine sub-cell.  For nested
    spaces the natural embedding used by the paper's transfers (Sec. 3) is
    this projection; here it is computed exactly by clipping the fine
    sub-cell against the coarse sub-cells it overlaps.
Restriction is the transpose; the operators are rediscretised per level.
"""
import numpy as np
import scipy.sparse as sp

from . import lagrange, mesh, quad
from .th import THLevel


def macro_subcells(n):
    """Sub-cells of the barycentric refinement, in units of 1/(3n), with their macro index and s."""
    out = []
    for m, tri in enumerate(mesh.triangle_cells(n)):
        V = [(3 * v[0], 3 * v[1]) for v in tri]
        c = (sum(v[0] for v in tri), sum(v[1] for v in tri))
        for s in range(3):
            out.append(((V[s], V[(s + 1) % 3], c), m, s))
    return out


class SVLevel(THLevel):
    family = "sv"

    def __init__(self, k, n, nu, field):
        self.dim, self.k, self.n, self.nu = 2, k, n, nu
        sub = macro_subcells(n)
        self.cells = [c for c, _, _ in sub]
        self.macro = np.array([m for _, m, _ in sub])
        self.n3 = 3 * n
        self.vb = lagrange.LagrangeBasis(2, k)
        self.pb = lagrange.LagrangeBasis(2, k - 1)
        self.Mv = k * self.n3
        self.Mp = (k - 1) * self.n3
        self.nbp = len(lagrange.lattice_nodes(2, k - 1))
        # velocity nodes of the sub-cell mesh
        nodes = set()
        for cell in self.cells:
            nodes.update(self.cell_nodes(cell, k))
        M = self.Mv
        interior = [G for G in nodes if 0 < G[0] < M and 0 < G[1] < M]
        interior.sort(key=lambda G: (G[1], G[0]))
        self._vidx = {G: i for i, G in enumerate(interior)}
        self.vel_nodes = interior
        self.n_vel_nodes_int = len(interior)
        self.n_vel_nodes_all = len(nodes)
        self.nu_free = 2 * len(interior)
        self.np_ = len(self.cells) * self.nbp
        self.N = self.nu_free + self.np_
        self.field = field
        self._assemble()

    # ---- numbering ------------------------------------------------------------
    def vel_index(self, G):
        return self._vidx.get(tuple(G), -1)

    def cell_pdofs(self, ci):
        base = self.nu_free + ci * self.nbp
        return list(range(base, base + self.nbp))

    def cell_nodes(self, cell, kk):
        """Lattice points (spacing 1/(3 kk n)) of the local P_kk nodes of a sub-cell."""
        v0 = np.array(cell[0])
        E = [np.array(cell[1]) - v0, np.array(cell[2]) - v0]
        return [tuple(int(g) for g in kk * v0 + a[0] * E[0] + a[1] * E[1])
                for a in lagrange.lattice_nodes(2, kk)]

    def cell_geometry(self, cell):
        v0 = np.array(cell[0], dtype=float) / self.n3
        J = np.stack([np.array(cell[d + 1], dtype=float) / self.n3 - v0 for d in range(2)], axis=1)
        return v0, J

    # ---- assembly ---------------------------------------------------------------
    def _assemble(self):
        k = self.k
        self._rule = quad.simplex_rule(2, k + 3)
        qp = self._rule[0]
        self._Gv = self.vb.grad(qp)
        self._Pp = self.pb.eval(qp)
        self._Pv = self.vb.eval(qp)
        nbv = self._Pv.shape[1]
        rows, cols, vals = [], [], []
        rhs = np.zeros(self.N)
        for ci, cell in enumerate(self.cells):
            Aloc, Bloc, Floc = self.element_matrices(cell)
            vdof = np.empty(nbv * 2, dtype=np.int64)
            uD = np.zeros(nbv * 2)
            for i, G in enumerate(self.cell_nodes(cell, k)):
                idx = self.vel_index(G)
                for c in range(2):
                    vdof[2 * i + c] = 2 * idx + c if idx >= 0 else -1
                if idx < 0:
                    uD[2 * i:2 * i + 2] = self.field.u(np.array(G, dtype=float)[None, :] / self.Mv)[0]
            pdof = np.array(self.cell_pdofs(ci), dtype=np.int64)
            free = vdof >= 0
            fv = vdof[free]
            rr, cc = np.meshgrid(fv, fv, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(Aloc[np.ix_(free, free)].ravel())
            rr, cc = np.meshgrid(pdof, fv, indexing="ij")
            Bf = Bloc[:, free]
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(Bf.ravel())
            rows.append(cc.ravel()); cols.append(rr.ravel()); vals.append(Bf.ravel())
            rhs[fv] += Floc[free] - Aloc[np.ix_(free, ~free)] @ uD[~free]
            rhs[pdof] += -Bloc[:, ~free] @ uD[~free]
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.N, self.N)).tocsr()
        K.sum_duplicates()
        K.sort_indices()
        self.K = K
        self.b = rhs

    def dof_coords(self):
        """(N, 2) node positions and (N,) kind: 0/1 velocity component, 2 pressure.

        Pressure nodes on a shared sub-cell edge appear once per sub-cell.
        """
        X = np.zeros((self.N, 2))
        kind = np.zeros(self.N, dtype=np.int64)
        for i, G in enumerate(self.vel_nodes):
            X[2 * i:2 * i + 2] = np.array(G, dtype=float) / self.Mv
            kind[2 * i] = 0
            kind[2 * i + 1] = 1
        for ci, cell in enumerate(self.cells):
            for j, G in zip(self.cell_pdofs(ci), self.cell_nodes(cell, self.k - 1)):
                X[j] = np.array(G, dtype=float) / self.Mp
                kind[j] = 2
        return X, kind

    # ---- evaluation of a discrete solution ------------------------------------
    def cell_values(self, ci, x):
        """Nodal velocity (nbv, 2) with Dirichlet data, and pressure coefficients (nbp,) of one sub-cell."""
        cell = self.cells[ci]
        U = np.zeros((self._Pv.shape[1], 2))
        for i, G in enumerate(self.cell_nodes(cell, self.k)):
            idx = self.vel_index(G)
            if idx >= 0:
                U[i] = x[2 * idx:2 * idx + 2]
            else:
                U[i] = self.field.u(np.array(G, dtype=float)[None, :] / self.Mv)[0]
        return U, x[self.cell_pdofs(ci)]


def errors(level, x, qdeg=None):
    """Relative H^1 velocity error, L^2 pressure error (mean removed) and ||div u_h||_{L^2}."""
    k = level.k
    qp, qw = quad.simplex_rule(2, qdeg or k + 6)
    Pv, Gv, Pp = level.vb.eval(qp), level.vb.grad(qp), level.pb.eval(qp)
    F = level.field
    e1 = n1 = div2 = 0.0
    ep_int = ep2 = area = 0.0
    for ci, cell in enumerate(level.cells):
        v0, J = level.cell_geometry(cell)
        g = Gv @ np.linalg.inv(J)
        w = qw * abs(np.linalg.det(J))
        xq = v0[None, :] + qp @ J.T
        U, pl = level.cell_values(ci, x)
        uh = Pv @ U
        guh = np.einsum("qid,ic->qcd", g, U)
        div2 += w @ (guh[:, 0, 0] + guh[:, 1, 1]) ** 2
        if F.grad_u is not None:
            ue, gue = F.u(xq), F.grad_u(xq)
            e1 += w @ (np.sum((ue - uh) ** 2, 1) + np.sum((gue - guh) ** 2, (1, 2)))
            n1 += w @ (np.sum(ue ** 2, 1) + np.sum(gue ** 2, (1, 2)))
        dp = F.p(xq) - Pp @ pl
        ep_int += w @ dp
        ep2 += w @ dp ** 2
        area += w.sum()
    mean = ep_int / area
    ev = np.sqrt(e1 / n1) if n1 > 0 else float("nan")
    return ev, np.sqrt(max(ep2 - 2 * mean * ep_int + mean * mean * area, 0.0)), np.sqrt(div2)


def _bary(cell, pts, unit):
    """Barycentric coordinates (npts, 3) of points (npts, 2) w.r.t. a sub-cell given in lattice units."""
    V = np.array(cell, dtype=float) / unit
    T = np.stack([V[1] - V[0], V[2] - V[0]], axis=1)
    xi = np.linalg.solve(T, (pts - V[0]).T).T
    return np.concatenate([1.0 - xi.sum(1, keepdims=True), xi], 1), xi


def _coarse_candidates(coarse, pts):
    """For each point, the coarse sub-cell indices of the macro squares whose closure holds the point."""
    n = coarse.n
    out = []
    for p in pts:
        cand = []
        for i in range(max(0, int(np.floor(p[0] * n - 1e-9))), min(n - 1, int(np.floor(p[0] * n + 1e-9))) + 1):
            for j in range(max(0, int(np.floor(p[1] * n - 1e-9))), min(n - 1, int(np.floor(p[1] * n + 1e-9))) + 1):
                base = 6 * (j * n + i)         # two macro triangles per square, three sub-cells each
                cand.extend(range(base, base + 6))
        out.append(sorted(cand))
    return out


def _clip(poly, tri):
    """Sutherland-Hodgman: the part of a convex polygon (list of 2D points) inside a triangle."""
    T = [np.asarray(v, dtype=float) for v in tri]
    orient = np.sign((T[1][0] - T[0][0]) * (T[2][1] - T[0][1]) - (T[1][1] - T[0][1]) * (T[2][0] - T[0][0]))
    for e in range(3):
        a, b = T[e], T[(e + 1) % 3]
        side = lambda p: orient * ((b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0]))
        out = []
        for i in range(len(poly)):
            p, q = poly[i], poly[(i + 1) % len(poly)]
            sp_, sq = side(p), side(q)
            if sp_ >= 0:
                out.append(p)
            if (sp_ >= 0) != (sq >= 0):
                t = sp_ / (sp_ - sq)
                out.append(p + t * (q - p))
        poly = out
        if not poly:
            break
    return poly


def _area(poly):
    return 0.5 * abs(sum(poly[i][0] * poly[(i + 1) % len(poly)][1] - poly[(i + 1) % len(poly)][0] * poly[i][1]
                         for i in range(len(poly))))


def _pressure_l2(coarse, fine, fc, cand, qp, qw):
    """Local L^2 projection onto the fine sub-cell fc of each coarse pressure basis function:
    (nbp_f, np_c) block and the overlapping coarse sub-cells, exact (the intersections with the coarse sub-cells are clipped polygons,
    integrated piece by piece with a rule exact for the degree-2(k-1) integrands)."""
    fcell = fine.cells[fc]
    Vf = [np.array(v, dtype=float) / fine.n3 for v in fcell]
    _, Jf = fine.cell_geometry(fcell)
    areaf = 0.5 * abs(np.linalg.det(Jf))
    G = np.zeros((fine.nbp, coarse.np_))
    hit = []
    for cc in cand:
        Vc = [np.array(v, dtype=float) / coarse.n3 for v in coarse.cells[cc]]
        poly = _clip(list(Vf), Vc)
        if len(poly) < 3 or _area(poly) <= 1e-10 * areaf:
            continue
        cols = np.array(coarse.cell_pdofs(cc)) - coarse.nu_free
        hit.append(cc)
        for i in range(1, len(poly) - 1):
            a, b, c = poly[0], poly[i], poly[i + 1]
            Jt = np.stack([b - a, c - a], 1)
            w = qw * abs(np.linalg.det(Jt))
            x = a[None, :] + qp @ Jt.T
            _, xif = _bary(fcell, x, fine.n3)
            _, xic = _bary(coarse.cells[cc], x, coarse.n3)
            G[:, cols] += np.einsum("q,qa,qj->aj", w, fine.pb.eval(xif), coarse.pb.eval(xic))
    Mf = np.einsum("q,qa,qb->ab", qw * 2.0 * areaf, fine.pb.eval(qp), fine.pb.eval(qp))
    return np.linalg.solve(Mf, G), hit


def prolongation(coarse, fine, drop=1e-12):
    """P = diag(P^V, P^Q) between non-nested barycentric levels (see the module docstring).

    Velocity rows: nodal interpolation in the first coarse sub-cell (in
    sub-cell order) among those of the macro squares around the node whose
    closure contains it (barycentric coordinates >= -1e-12); entries below
    `drop` in magnitude are exact zeros of the rational weights and are dropped.
    Pressure rows: the fine sub-cell's block of the local L^2 projection; its
    pattern is every coarse pressure DoF of every coarse sub-cell that overlaps
    the fine sub-cell with positive area (stored even where a value is zero).
    """
    rows, cols, vals = [], [], []
    # velocity
    pts = np.array(fine.vel_nodes, dtype=float) / fine.Mv
    cands = _coarse_candidates(coarse, pts)
    for fi, (p, cand) in enumerate(zip(pts, cands)):
        for cc in cand:
            lam, xi = _bary(coarse.cells[cc], p[None, :], coarse.n3)
            if lam.min() >= -1e-12:
                break
        else:
            raise AssertionError("fine velocity node outside the coarse mesh")
        phi = coarse.vb.eval(xi)[0]
        for j, CG in enumerate(coarse.cell_nodes(coarse.cells[cc], coarse.k)):
            cidx = coarse.vel_index(CG)
            if cidx < 0 or abs(phi[j]) < drop:
                continue
            for c in range(2):
                rows.append(2 * fi + c); cols.append(2 * cidx + c); vals.append(phi[j])
    # pressure
    qp, qw = quad.simplex_rule(2, fine.k + 1)
    cents = np.array([np.mean(np.array(cell, dtype=float), 0) / fine.n3 for cell in fine.cells])
    cands = _coarse_candidates(coarse, cents)
    for fc, cand in enumerate(cands):
        loc, hit = _pressure_l2(coarse, fine, fc, cand, qp, qw)
        pat = sorted(c - coarse.nu_free for cc in hit for c in coarse.cell_pdofs(cc))
        for a, r in enumerate(fine.cell_pdofs(fc)):
            for c in pat:
                rows.append(r); cols.append(coarse.nu_free + c); vals.append(loc[a, c])
    P = sp.coo_matrix((vals, (rows, cols)), shape=(fine.N, coarse.N)).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    return P


def macro_patches(level):
    """One patch per macro triangle: the pressure DoFs of its three sub-cells and every free
    velocity DoF on the closure of the macro triangle; ascending DoF lists, macro order."""
    patches = []
    for m in range(len(level.cells) // 3):
        vd, pd = set(), []
        for ci in range(3 * m, 3 * m + 3):
            pd.extend(level.cell_pdofs(ci))
            for G in level.cell_nodes(level.cells[ci], level.k):
                idx = level.vel_index(G)
                if idx >= 0:
                    vd.update((2 * idx, 2 * idx + 1))
        patches.append(sorted(vd | set(pd)))
    return patches


class SVHierarchy:
    """Levels 0 (coarsest, n0) .. L-1 (finest, n0 2^(L-1)), each the barycentric refinement of the
    uniform macro mesh, rediscretised on every level."""

    def __init__(self, k, n0, nlevels, nu, field_factory):
        self.dim, self.k = 2, k
        self.levels = [SVLevel(k, n0 * 2 ** l, nu, field_factory(nu)) for l in range(nlevels)]
        self.P = [None] + [prolongation(self.levels[l - 1], self.levels[l]) for l in range(1, nlevels)]

    @property
    def finest(self):
        return self.levels[-1]
