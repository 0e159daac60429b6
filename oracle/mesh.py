"""Structured simplicial meshes of the unit square and cube (oracle).

2D (Sec. 4): an n x n grid of squares, each square cut along the diagonal
from its top-left to its bottom-right corner into two triangles.  Uniform
refinement (each triangle into four by its edge midpoints) of this mesh is
again the same kind of mesh at 2n, so the hierarchy n0, 2 n0, 4 n0, ... is
nested (Sec. 3, the nested grid family T_1 subset ... subset T_L).

3D (not in the paper, which is 2D only): each cube is split into the six
Kuhn tetrahedra that share the cube's (0,0,0)-(1,1,1) diagonal.

Vertices are integer lattice points (i, j[, l]) with 0 <= i, j, l <= n; the
physical point is (i, j, l) / n.  A cell is a tuple of dim + 1 such vertices.
"""
import itertools


def triangle_cells(n):
    cells = []
    for j in range(n):
        for i in range(n):
            bl, br, tl, tr = (i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1)
            cells.append((bl, br, tl))   # below the TL-BR diagonal
            cells.append((tr, tl, br))   # above it
    return cells


def kuhn_cells(n):
    cells = []
    for l in range(n):
        for j in range(n):
            for i in range(n):
                o = (i, j, l)
                for perm in itertools.permutations(range(3)):
                    v = list(o)
                    verts = [tuple(v)]
                    for d in perm:
                        v[d] += 1
                        verts.append(tuple(v))
                    cells.append(tuple(verts))
    return cells


def cells(dim, n):
    return triangle_cells(n) if dim == 2 else kuhn_cells(n)
