"""Geometric coarse space of the two-grid preconditioner (paper Sec. 3,
Eq. coarse: R_0 from a coarser triangulation, A_c = R_0 A R_0^T; the
fine:coarse ratio study of the coarse-space tables in Sec. 5).  Test
infrastructure only.

The fine mesh is the structured N x N lattice of squares cut along "/"; the
coarse mesh is the same lattice with N/r cells per side (r >= 1, dividing
N), so every coarse triangle is the union of r^2 fine triangles of the same
orientation (the fine cells on a coarse diagonal are cut along it).
R_0^T = P_0 interpolates coarse P1 functions at the fine nodes: fine node
(i, j) lies in coarse cell (i // r, j // r) at local coordinates
(a, b) = ((i mod r) / r, (j mod r) / r); in the lower triangle (a >= b:
corners (0,0), (1,0), (1,1)) its weights are (1 - a, a - b, b), in the upper
one (corners (0,0), (1,1), (0,1)) they are (1 - b, a, b - a).  Coarse nodes
on the boundary carry the Dirichlet value 0 and are dropped, so P_0 is
[(N-1)^2 x (N/r - 1)^2] with unknowns numbered x-fastest on both meshes.

The coarse operator is A_c = P_0^T A P_0 = sum_i (P_0^T K_i P_0) (x) G_i
(coarse.coarse_blocks with Z = P_0), and the two-grid cycle is the one of
precond.TwoLevel with Z = P_0.  For a mesh whose vertices were moved
(jittered), the same topological P_0 defines the coarse space.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def prolongation(N: int, r: int) -> sp.csr_matrix:
    if r < 1 or N % r:
        raise ValueError("the ratio r must divide the number of cells N")
    Nc = N // r
    nf, nc = (N - 1) ** 2, (Nc - 1) ** 2
    rows, cols, vals = [], [], []

    def add(row, ci, cj, w):
        if w != 0.0 and 0 < ci < Nc and 0 < cj < Nc:
            rows.append(row)
            cols.append((cj - 1) * (Nc - 1) + (ci - 1))
            vals.append(w)

    for j in range(1, N):
        for i in range(1, N):
            row = (j - 1) * (N - 1) + (i - 1)
            ci, cj = i // r, j // r
            a, b = (i % r) / r, (j % r) / r
            if a >= b:
                add(row, ci, cj, 1.0 - a)
                add(row, ci + 1, cj, a - b)
                add(row, ci + 1, cj + 1, b)
            else:
                add(row, ci, cj, 1.0 - b)
                add(row, ci + 1, cj + 1, a)
                add(row, ci, cj + 1, b - a)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))
