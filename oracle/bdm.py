"""(BDM_k, dP_{k-1}) with symmetric interior penalty on triangles (oracle), Sec. 2-3.

Test infrastructure: only the tests, the smoke check and the CPU baseline of the
benchmark use this module.

Discretisation (Sec. 2, the H(div)-L2 formulation, Case 3 of Sec. 3):
  * mesh: the two-triangle split of the n x n grid of the unit square (oracle.mesh);
  * velocity: BDM_k, vector P_k on each triangle with continuous normal component,
    v.n = 0 imposed strongly on the boundary (boundary edge DoFs dropped);
  * pressure: dP_{k-1}, discontinuous P_{k-1} (a constant per cell for k = 1);
  * a_h: the symmetric interior-penalty form (the equation labelled
    DiscontBilinearForm): 2 nu [ sum_T (eps(u), eps(v))_T - sum_e ({eps(u)}, [v]^t)_e
    - sum_e ([u]^t, {eps(v)})_e ] + 2 nu alpha sum_e h_e^{-1} ([u]^t, [v]^t)_e over
    interior edges e only (the boundary terms vanish by u.n = 0 and the natural
    tangential-stress condition);  b(v, q) = -(q, div v);  load (f, v).

With t the unit tangent and n1 the unit normal of e pointing out of T1 (T2 on the
other side), the symmetric jump of a vector with continuous normal component is
[v]^t = ((v1 - v2).t) (t (.) n1) with t (.) n1 = (t n1^T + n1 t^T) / 2, so that
  {eps(u)} : [v]^t = ((v1 - v2).t) t^T {eps(u)} n1,  [u]^t : [v]^t = ((u1 - u2).t)((v1 - v2).t) / 2.
The penalty alpha is not given in the paper; the default is 2 (k + 1)^2, between 2.3 (k = 8)
and 4.6 (k = 1) times the smallest value that keeps a_h coercive on these meshes.

Degrees of freedom (a dual basis of the following functionals on each cell T):
  * each edge e with endpoints a, b (global vertex index y (n + 1) + x of a smaller),
    t = (b - a) / |b - a|, n_e = (t_y, -t_x):  v -> |e|^{-1} int_e (v.n_e) L_j(s) ds,
    j = 0..k, L_j the Legendre polynomial of degree j shifted to s in [0, 1] (s = 0 at a);
  * the interior:  v -> |T|^{-1} int_T v.q dx for q in an orthonormal basis (inner
    product |T|^{-1} int_T) of the Nedelec space of the first kind
    ND_{k-1} = [P_{k-2}]^2 + x^perp P~_{k-2} (P~ the homogeneous polynomials): the
    Gram-Schmidt orthonormalisation, in order, of e_0 l_a, e_1 l_a (l_a the nodal P_{k-2}
    basis of the cell) and (-xi_2, xi_1) l_a for the nodes a on the edge opposite the
    first vertex, xi = n (x - x_c), x_c the centroid (see _interior_q).  Orthonormal tests
    keep the interior basis functions of unit size at every k.
  Normal moments against P_k(e) fix v.n on e, so a function whose edge functionals
  vanish on an edge has zero normal trace there, and the cell-wise dual bases glue into
  an H(div) basis.
Pressure: the nodal P_{k-1} basis of each cell at the lattice points of the cell's
  vertex order (oracle.lagrange), so the constant pressure has all coefficients one.

Numbering: free velocity DoFs are the interior edges in ascending (index(a), index(b))
order with their k + 1 moments, then the cells (in oracle.mesh order) with their
k^2 - 1 interior moments; the pressure DoFs follow, cell by cell.

Transfers (Sec. 3, grid transfers): the natural embedding of the nested spaces, i.e. the
fine functionals applied to the coarse basis functions (velocity) and the coarse pressure
basis evaluated at the fine nodes; restriction is the transpose.

Patches (Sec. 3.1, extended cell Vanka): for each cell T, the pressure DoFs of T and every
velocity DoF on the closure of T and of the cells sharing an edge with T.
"""
import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as _leg

from . import lagrange, mesh, quad


def default_alpha(k):
    return 2.0 * (k + 1) * (k + 1)


def _vid(n, G):
    return G[1] * (n + 1) + G[0]


def _edge_key(n, a, b):
    return (a, b) if _vid(n, a) < _vid(n, b) else (b, a)


def _shifted_legendre(j, s):
    c = np.zeros(j + 1)
    c[j] = 1.0
    return _leg.legval(2.0 * np.asarray(s) - 1.0, c)


def _interior_q(k, xh, xi):
    """Values (npts, k^2 - 1, 2) of the raw interior test functions q_m (before orthonormalisation).

    xh are the points in the cell's reference coordinates, xi = n (x - x_c) the scaled
    physical offsets from the centroid.  With l_a the nodal P_{k-2} basis of the cell
    (oracle.lagrange lattice order; the constant for k = 2): first e_0 l_a, then e_1 l_a,
    then (-xi_2, xi_1) l_a for the nodes a with a_1 + a_2 = k - 2 (the nodes on the edge
    opposite the first vertex, whose leading homogeneous parts span the degree k - 2 forms).
    Together they span ND_{k-1}(T) = [P_{k-2}]^2 + x^perp P~_{k-2}.
    """
    if k < 2:
        return np.zeros((len(xh), 0, 2))
    if k == 2:
        lat, La = [(0, 0)], np.ones((len(xh), 1))
    else:
        lb = lagrange.LagrangeBasis(2, k - 2)
        lat, La = lb.lattice, lb.eval(xh)
    out = []
    for c in range(2):
        for m in range(len(lat)):
            v = np.zeros((len(xh), 2))
            v[:, c] = La[:, m]
            out.append(v)
    for m, a in enumerate(lat):
        if sum(a) == k - 2:
            out.append(np.stack([-xi[:, 1] * La[:, m], xi[:, 0] * La[:, m]], 1))
    return np.stack(out, 1)


def _gram_schmidt(Q, w):
    """Coefficients T (ni x ni, lower triangular) with q'_i = sum_j T[i, j] q_j orthonormal.

    Q: (npts, ni, 2) raw test functions at quadrature points, w: weights of the inner
    product |T|^{-1} int_T u.v.  Classical Gram-Schmidt in the given order (positive
    leading coefficients), done twice for accuracy.
    """
    ni = Q.shape[1]
    T = np.zeros((ni, ni))
    for i in range(ni):
        c = np.zeros(ni)
        c[i] = 1.0
        for _ in range(2):
            v = np.einsum("j,pjc->pc", c, Q)
            for j in range(i):
                qj = np.einsum("m,pmc->pc", T[j], Q)
                c = c - (w @ np.sum(v * qj, 1)) * T[j]
        v = np.einsum("j,pjc->pc", c, Q)
        T[i] = c / np.sqrt(w @ np.sum(v * v, 1))
    return T


class _PressureBasis:
    """Nodal P_kk on the reference triangle; kk = 0 is the constant."""

    def __init__(self, kk):
        self.kk = kk
        self.lb = lagrange.LagrangeBasis(2, kk) if kk >= 1 else None

    def eval(self, xh):
        if self.lb is None:
            return np.ones((len(np.atleast_2d(xh)), 1))
        return self.lb.eval(xh)

    def lattice(self):
        return [(0, 0)] if self.lb is None else self.lb.lattice


class BDMLevel:
    cell_type = "bdm"
    family = "bdm"

    def __init__(self, k, n, nu, field, alpha=None):
        self.dim, self.k, self.n, self.nu = 2, k, n, nu
        self.alpha = default_alpha(k) if alpha is None else alpha
        self.field = field
        self.cells = mesh.triangle_cells(n)
        self.vb = lagrange.LagrangeBasis(2, k)     # local polynomial space used to build the dual basis
        self.pb = _PressureBasis(k - 1)
        self.ne_loc = k + 1
        self.ni_loc = k * k - 1
        self.nbv = 3 * self.ne_loc + self.ni_loc   # = (k + 1)(k + 2) = dim [P_k]^2
        self.nbp = k * (k + 1) // 2
        # edges
        self.cell_edges = []
        edge_cells = {}
        for ci, c in enumerate(self.cells):
            es = []
            for a, b in ((c[0], c[1]), (c[1], c[2]), (c[0], c[2])):
                key = _edge_key(n, a, b)
                es.append(key)
                edge_cells.setdefault(key, []).append(ci)
            self.cell_edges.append(es)
        self.edge_cells = edge_cells
        interior = sorted((e for e, cs in edge_cells.items() if len(cs) == 2),
                          key=lambda e: (_vid(n, e[0]), _vid(n, e[1])))
        self.edge_rank = {e: r for r, e in enumerate(interior)}
        self.interior_edges = interior
        self.nu_edges = len(interior) * self.ne_loc
        self.nu_free = self.nu_edges + len(self.cells) * self.ni_loc
        self.np_ = len(self.cells) * self.nbp
        self.N = self.nu_free + self.np_
        self._bases = [self._cell_basis(ci) for ci in range(len(self.cells))]
        self._assemble()

    # ---- geometry ------------------------------------------------------------
    def cell_geometry(self, cell):
        v0 = np.array(cell[0], dtype=float) / self.n
        J = np.stack([np.array(cell[d + 1], dtype=float) / self.n - v0 for d in range(2)], axis=1)
        return v0, J

    def quad_rule(self, q):
        return quad.simplex_rule(2, q)

    def edge_frame(self, e):
        a = np.array(e[0], dtype=float) / self.n
        b = np.array(e[1], dtype=float) / self.n
        L = np.linalg.norm(b - a)
        t = (b - a) / L
        return a, b, L, t, np.array([t[1], -t[0]])

    # ---- the dual basis of one cell ------------------------------------------
    def cell_vel_dofs(self, ci):
        """Global DoF (or -1 on the boundary) of each local basis function of cell ci."""
        out = []
        for e in self.cell_edges[ci]:
            r = self.edge_rank.get(e, -1)
            out += [r * self.ne_loc + j if r >= 0 else -1 for j in range(self.ne_loc)]
        base = self.nu_edges + ci * self.ni_loc
        out += list(range(base, base + self.ni_loc))
        return np.array(out, dtype=np.int64)

    def cell_pdofs(self, ci):
        base = self.nu_free + ci * self.nbp
        return np.arange(base, base + self.nbp)

    def _psi(self, ci, x):
        """Local polynomial space [P_k]^2 at physical points x: values (np, 2 nb, 2), grads (np, 2 nb, 2, 2)."""
        v0, J = self.cell_geometry(self.cells[ci])
        Jinv = np.linalg.inv(J)
        xh = (x - v0[None, :]) @ Jinv.T
        P = self.vb.eval(xh)
        G = self.vb.grad(xh) @ Jinv          # d/dx
        npts, nb = P.shape
        val = np.zeros((npts, 2 * nb, 2))
        grad = np.zeros((npts, 2 * nb, 2, 2))
        for c in range(2):
            val[:, c::2, c] = P
            grad[:, c::2, c, :] = G
        return val, grad

    def _cell_basis(self, ci):
        """Coefficients C (2 nb x nbv) of the dual basis phi_i = sum_j C[j, i] psi_j."""
        k, cell = self.k, self.cells[ci]
        v0, J = self.cell_geometry(cell)
        D = np.zeros((self.nbv, self.nbv))
        row = 0
        g, gw = quad.gauss_legendre01(k + 2)
        for e in self.cell_edges[ci]:
            a, b, L, t, ne = self.edge_frame(e)
            x = a[None, :] + g[:, None] * (b - a)[None, :]
            val, _ = self._psi(ci, x)
            vn = val @ ne                       # (np, 2 nb)
            for j in range(self.ne_loc):
                D[row] = (gw * _shifted_legendre(j, g)) @ vn
                row += 1
        x, w, qv = self.interior_tests(ci)
        val, _ = self._psi(ci, x)
        for m in range(self.ni_loc):
            D[row] = np.einsum("p,pc,pjc->j", w, qv[:, m, :], val)
            row += 1
        return np.linalg.inv(D)

    def interior_tests(self, ci):
        """Orthonormal interior test functions of cell ci at its quadrature points.

        Returns the physical points (np, 2), the weights of |T|^{-1} int_T, and the values
        (np, k^2 - 1, 2) of the Gram-Schmidt orthonormalisation of the raw tests in order.
        """
        k = self.k
        v0, J = self.cell_geometry(self.cells[ci])
        qp, qw = quad.simplex_rule(2, k + 2)
        x = v0[None, :] + qp @ J.T
        w = qw * 2.0                                     # |det J| / |T| = 2
        xc = v0 + J @ np.array([1.0, 1.0]) / 3.0
        Q = _interior_q(k, qp, (x - xc[None, :]) * self.n)
        if Q.shape[1] == 0:
            return x, w, Q
        T = _gram_schmidt(Q, w)
        return x, w, np.einsum("im,pmc->pic", T, Q)

    def phi(self, ci, x):
        """Dual basis of cell ci at physical points x: values (np, nbv, 2), grads (np, nbv, 2, 2)."""
        val, grad = self._psi(ci, x)
        C = self._bases[ci]
        return np.einsum("pjc,ji->pic", val, C), np.einsum("pjcd,ji->picd", grad, C)

    def pressure_eval(self, ci, x):
        v0, J = self.cell_geometry(self.cells[ci])
        xh = (x - v0[None, :]) @ np.linalg.inv(J).T
        return self.pb.eval(xh)

    # ---- assembly ------------------------------------------------------------
    def element_matrices(self, ci):
        """Volume parts of one cell: A (nbv x nbv), B (nbp x nbv), F (nbv)."""
        nu = self.nu
        v0, J = self.cell_geometry(self.cells[ci])
        qp, qw = self._rule
        w = qw * abs(np.linalg.det(J))
        x = v0[None, :] + qp @ J.T
        Phi, G = self.phi(ci, x)
        eps = 0.5 * (G + np.swapaxes(G, 2, 3))
        A = 2.0 * nu * np.einsum("p,picd,pjcd->ij", w, eps, eps)
        div = G[:, :, 0, 0] + G[:, :, 1, 1]
        Q = self.pressure_eval(ci, x)
        B = -np.einsum("p,pq,pi->qi", w, Q, div)
        F = np.einsum("p,pc,pic->i", w, self.field.f(x), Phi)
        return A, B, F

    def edge_matrix(self, e):
        """Interior-edge terms of a_h on edge e over the local DoFs of (T1, T2), stacked."""
        nu, alpha = self.nu, self.alpha
        a, b, L, t, ne = self.edge_frame(e)
        T = self.edge_cells[e]
        # T1 is the cell that n_e points out of
        c0 = self.cells[T[0]]
        centroid = np.array([sum(v[d] for v in c0) for d in range(2)], dtype=float) / (3.0 * self.n)
        if (centroid - 0.5 * (a + b)) @ ne > 0:
            T = [T[1], T[0]]
        n1 = ne
        g, gw = quad.gauss_legendre01(self.k + 2)
        x = a[None, :] + g[:, None] * (b - a)[None, :]
        w = gw * L
        jumps, avgs = [], []
        for side, ci in enumerate(T):
            Phi, G = self.phi(ci, x)
            eps = 0.5 * (G + np.swapaxes(G, 2, 3))
            sgn = 1.0 if side == 0 else -1.0
            jumps.append(sgn * (Phi @ t))                                  # (np, nbv)
            avgs.append(0.5 * np.einsum("c,picd,d->pi", t, eps, n1))
        jump = np.concatenate(jumps, 1)
        avg = np.concatenate(avgs, 1)
        A = -2.0 * nu * (np.einsum("p,pi,pj->ij", w, jump, avg) + np.einsum("p,pi,pj->ij", w, avg, jump))
        A += 2.0 * nu * alpha / L * 0.5 * np.einsum("p,pi,pj->ij", w, jump, jump)
        dofs = np.concatenate([self.cell_vel_dofs(T[0]), self.cell_vel_dofs(T[1])])
        return A, dofs

    def _assemble(self):
        self._rule = quad.simplex_rule(2, self.k + 3)
        rows, cols, vals = [], [], []
        rhs = np.zeros(self.N)

        def add(r, c, M):
            fr, fc = r >= 0, c >= 0
            rr, cc = np.meshgrid(r[fr], c[fc], indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(M[np.ix_(fr, fc)].ravel())

        for ci in range(len(self.cells)):
            A, B, F = self.element_matrices(ci)
            vd, pd = self.cell_vel_dofs(ci), self.cell_pdofs(ci)
            add(vd, vd, A)
            add(pd, vd, B)
            add(vd, pd, B.T)
            free = vd >= 0
            rhs[vd[free]] += F[free]
        for e in self.interior_edges:
            A, dofs = self.edge_matrix(e)
            add(dofs, dofs, A)
        rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
        K = sp.coo_matrix((vals, (rows, cols)), shape=(self.N, self.N)).tocsr()
        K.sum_duplicates()
        K.sort_indices()
        self.K = K
        self.b = rhs

    def nullvec(self):
        """z = (0, 1_p) / sqrt(m): the normalised constant pressure (nodal basis)."""
        z = np.zeros(self.N)
        z[self.nu_free:] = 1.0 / np.sqrt(self.np_)
        return z

    # ---- evaluation of a discrete solution -----------------------------------
    def velocity(self, ci, coef, x):
        """u_h and grad u_h on cell ci at physical points x for the free-DoF vector coef."""
        Phi, G = self.phi(ci, x)
        vd = self.cell_vel_dofs(ci)
        c = np.where(vd >= 0, coef[np.maximum(vd, 0)], 0.0)
        return Phi.transpose(0, 2, 1) @ c, np.einsum("picd,i->pcd", G, c)

    def locate(self, x):
        """Index of a cell of this mesh whose closure holds the point x (lower triangle on ties)."""
        X = np.asarray(x, dtype=float) * self.n
        i = min(int(np.floor(X[0])), self.n - 1)
        j = min(int(np.floor(X[1])), self.n - 1)
        u, v = X[0] - i, X[1] - j
        return 2 * (j * self.n + i) + (0 if u + v <= 1.0 else 1)


def prolongation(coarse, fine):
    """Natural embedding BDM_k(coarse) -> BDM_k(fine) and dP_{k-1}(coarse) -> dP_{k-1}(fine).

    Velocity: entry (f, c) is the fine functional f applied to the coarse basis function c,
    evaluated in one coarse cell holding the fine entity (a fine edge on a coarse edge sees
    the same normal trace from both sides).  Pressure: the coarse basis of the parent cell
    at the fine nodes.  Entries below 1e-12 in magnitude (exact zeros up to rounding) are dropped.
    """
    k = fine.k
    rows, cols, vals = [], [], []

    def put(r, cdofs, v):
        for c, val in zip(cdofs, v):
            if c >= 0 and abs(val) >= 1e-12:
                rows.append(r); cols.append(c); vals.append(val)

    g, gw = quad.gauss_legendre01(k + 2)
    for e in fine.interior_edges:
        a, b, L, t, ne = fine.edge_frame(e)
        cc = coarse.locate(0.5 * (a + b))
        x = a[None, :] + g[:, None] * (b - a)[None, :]
        Phi, _ = coarse.phi(cc, x)
        vn = Phi @ ne                                           # (np, nbv)
        cd = coarse.cell_vel_dofs(cc)
        r0 = fine.edge_rank[e] * fine.ne_loc
        for j in range(fine.ne_loc):
            put(r0 + j, cd, (gw * _shifted_legendre(j, g)) @ vn)
    for ci, cell in enumerate(fine.cells):
        v0, J = fine.cell_geometry(cell)
        xc = v0 + J @ np.array([1.0, 1.0]) / 3.0
        cc = coarse.locate(xc)
        x, w, qv = fine.interior_tests(ci)
        Phi, _ = coarse.phi(cc, x)
        cd = coarse.cell_vel_dofs(cc)
        base = fine.nu_edges + ci * fine.ni_loc
        for m in range(fine.ni_loc):
            put(base + m, cd, np.einsum("p,pc,pic->i", w, qv[:, m, :], Phi))
        # pressure: nodal values of the coarse pressure basis at the fine nodes
        kk = k - 1
        nodes = fine.pb.lattice()
        xn = np.array([v0 + (J @ np.array(a, dtype=float)) / max(kk, 1) if kk >= 1 else xc for a in nodes])
        Q = coarse.pressure_eval(cc, xn)
        cpd = coarse.cell_pdofs(cc)
        for p_i, r in enumerate(fine.cell_pdofs(ci)):
            put(int(r), cpd, Q[p_i])
    P = sp.coo_matrix((vals, (rows, cols)), shape=(fine.N, coarse.N)).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    return P


class BDMHierarchy:
    """Levels 0 (coarsest, n0) .. L-1 (finest, n0 * 2^(L-1)), rediscretised on every level (Sec. 3)."""

    def __init__(self, k, n0, nlevels, nu, field_factory, alpha=None):
        self.dim, self.k = 2, k
        self.levels = [BDMLevel(k, n0 * 2 ** l, nu, field_factory(nu), alpha) for l in range(nlevels)]
        self.P = [None] + [prolongation(self.levels[l - 1], self.levels[l]) for l in range(1, nlevels)]

    @property
    def finest(self):
        return self.levels[-1]


def build_patches(level):
    """Extended cell Vanka patches (Sec. 3.1), one per cell in cell order, DoF lists ascending."""
    patches = []
    for ci in range(len(level.cells)):
        group = {ci}
        for e in level.cell_edges[ci]:
            group.update(level.edge_cells[e])
        vd = set()
        for cj in group:
            vd.update(int(d) for d in level.cell_vel_dofs(cj) if d >= 0)
        patches.append(sorted(vd | set(int(p) for p in level.cell_pdofs(ci))))
    return patches


def errors(level, x, q=None):
    """Relative broken H^1 velocity error and mean-free L^2 pressure error (Sec. 4.4).

    The velocity norm is taken cell by cell (u_h is only H(div)); fixed collapsed Gauss
    rule with k + 6 points per direction.
    """
    k = level.k
    qp, qw = quad.simplex_rule(2, k + 6 if q is None else q)
    F = level.field
    e1 = n1 = 0.0
    ep_int = ep2 = area = 0.0
    for ci, cell in enumerate(level.cells):
        v0, J = level.cell_geometry(cell)
        w = qw * abs(np.linalg.det(J))
        xq = v0[None, :] + qp @ J.T
        uh, guh = level.velocity(ci, x, xq)
        ue, gue = F.u(xq), F.grad_u(xq)
        e1 += w @ (np.sum((ue - uh) ** 2, 1) + np.sum((gue - guh) ** 2, (1, 2)))
        n1 += w @ (np.sum(ue ** 2, 1) + np.sum(gue ** 2, (1, 2)))
        ph = level.pressure_eval(ci, xq) @ x[level.cell_pdofs(ci)]
        dp = F.p(xq) - ph
        ep_int += w @ dp
        ep2 += w @ dp ** 2
        area += w.sum()
    mean = ep_int / area
    return np.sqrt(e1 / n1), np.sqrt(max(ep2 - 2 * mean * ep_int + mean * mean * area, 0.0))
