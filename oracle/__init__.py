"""Plain FP64 CPU oracle for the monolithic multigrid / FGMRES Stokes solver
with matrix-full additive Vanka relaxation (Rafiei & MacLachlan,
"Achieving h- and p-robust monolithic multigrid solvers for the Stokes
equations").

TEST INFRASTRUCTURE ONLY.  This package exists so that the tests, the
``smoke()`` check and the CPU baseline leg of the benchmark have an
independent, slow, obviously correct statement of what the GPU path must
compute.  The product path (the HIP library and its Python binding) never
imports, calls or links anything here, and nothing here imports the product.

Everything is numpy / scipy in float64.  Library primitives (dense LU,
sparse matrix-vector products, Gauss-Legendre nodes) serve as single steps;
there is no blocking, fusion or reordering beyond what the paper states.

Modules
-------
quad      Gauss-Legendre rules and the collapsed (conical) rules on simplices
lagrange  equispaced P_k Lagrange bases on the reference simplex (barycentric product form)
mesh      structured simplicial meshes of the unit square / cube
fields    manufactured solutions and forcing fields
th        Taylor-Hood assembly: DoF numbering, K = [A B^T; B 0], rhs, transfers
qk        Taylor-Hood (Q_k, Q_{k-1}) on squares: tensor bases, transfers, composite patches
patches   composite ("topological") Vanka patches, Sec. 3.1
vanka     additive subspace correction (Algorithm 1) as a damped smoother
chebyshev its Chebyshev acceleration with a per-level Arnoldi eigenvalue estimate
mg        monolithic V-cycle with a bordered coarsest solve, Sec. 3
fgmres    right-preconditioned FGMRES with CGS2 orthogonalisation, Sec. 3
norms     H^1 / L^2 error norms (pressure mean removed), Sec. 4.4
"""
