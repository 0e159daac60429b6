"""Composite ("topological") Vanka patches for Taylor-Hood (oracle), Sec. 3.1.

The space decomposition (Sec. 3.1, eq. spacedecomp) is built from the mesh
topology:

* the star of an entity is the entity together with the interiors of all
  edges, faces and cells incident on it; its closure adds their boundaries;
* one patch per topological entity that carries pressure DoFs of P_{k-1}:
  vertices (every k >= 2), edge interiors (k >= 3: k - 2 DoFs per edge) and
  cell interiors (k >= 4 in 2D: (k-2)(k-3)/2 DoFs per cell);
* a patch holds the pressure DoFs of its entity and every free velocity DoF
  on the closure of the entity's star (for a vertex: all cells around it;
  for an edge: its one or two cells; for a cell: the cell itself).

For k = 2 this is the vertex-based Vanka patch (pressure at a vertex plus
velocity on the closure of the vertex star); for k >= 4 a patch can hold
several pressure DoFs.

Ordering convention: each patch's DoF list is ascending, and patches are
ordered by their smallest pressure DoF.

The "star" option (vertex patches only, with the pressure DoFs of the open
vertex star) is provided for comparison runs.  The "macro" option is the
macro-element patch of the barycentric Scott-Vogelius levels (oracle.sv).
"""
import numpy as np

from . import lagrange


def _entity_of(bary):
    """Topological entity of a local node from its barycentric lattice coordinates.

    Returns the tuple of local vertex indices whose barycentric coordinate is
    non-zero: one vertex -> vertex, two -> edge interior, three -> face/cell
    interior (2D) or face interior (3D), four -> cell interior (3D).
    """
    return tuple(i for i, a in enumerate(bary) if a > 0)


def build_patches(level, construct="composite"):
    if construct == "macro":
        from .sv import macro_patches
        return macro_patches(level)
    if getattr(level, "cell_type", "simplex") == "bdm":
        from .bdm import build_patches as extended_patches
        return extended_patches(level)
    if getattr(level, "cell_type", "simplex") == "quad":
        from .qk import build_patches as quad_patches
        return quad_patches(level)
    dim, k = level.dim, level.k
    # global entity key: frozenset of global vertex tuples
    ent_pdofs = {}          # entity -> set of pressure DoFs interior to it
    ent_cells = {}          # entity -> set of cell indices whose closure contains the entity
    cell_vdofs = []         # cell -> free velocity DoFs on its closure
    plat = lagrange.lattice_nodes(dim, k - 1)
    for ci, cell in enumerate(level.cells):
        pnodes = level.cell_nodes(cell, k - 1)
        for a, G in zip(plat, pnodes):
            bary = (k - 1 - sum(a),) + tuple(a)
            ent = frozenset(cell[i] for i in _entity_of(bary))
            ent_pdofs.setdefault(ent, set()).add(level.p_dof(G))
        # every sub-entity of the cell (all non-empty vertex subsets) is in its closure
        nv = dim + 1
        for mask in range(1, 1 << nv):
            ent = frozenset(cell[i] for i in range(nv) if mask >> i & 1)
            ent_cells.setdefault(ent, set()).add(ci)
        vd = []
        for G in level.cell_nodes(cell, k):
            idx = level.vel_index(G)
            if idx >= 0:
                vd.extend(dim * idx + c for c in range(dim))
        cell_vdofs.append(vd)

    patches = []
    if construct == "composite":
        for ent, pd in ent_pdofs.items():
            cells = ent_cells[ent]
            vd = set()
            for ci in cells:
                vd.update(cell_vdofs[ci])
            patches.append(sorted(vd | pd))
    elif construct == "star":
        # vertex patches with the pressure DoFs of the open star of the vertex
        for ent in ent_pdofs:
            if len(ent) != 1:
                continue
            (v,) = tuple(ent)
            cells = ent_cells[ent]
            vd, pd = set(), set()
            for ci in cells:
                vd.update(cell_vdofs[ci])
            for e2, pd2 in ent_pdofs.items():
                if v in e2:
                    pd.update(pd2)
            patches.append(sorted(vd | pd))
    else:
        raise ValueError(construct)
    nu = level.nu_free
    patches.sort(key=lambda I: min(d for d in I if d >= nu))
    return patches
