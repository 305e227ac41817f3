"""P1 finite elements for the stochastic Galerkin system (paper Sec. 2.1,
Eq. Galerkin_L_exp and the vector-PDE form Eq. linearVecPDE; the paper
leaves the element unnamed, "finite element or finite difference", end of
Sec. 2).  Test infrastructure only.

Reading: linear triangles, coefficient taken at the element centroid
(one-point rule), Dirichlet data eliminated (unknowns are interior nodes).

K_i[a, b] = sum_T c_bar_i(x_T) |T| grad(phi_a) . grad(phi_b)
F[a]      = sum_T f |T| / 3
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
import scipy.sparse as sp


def element_geometry(xy: np.ndarray, tri: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Areas [n_tri] and P1 gradients [n_tri, 3, 2] of the hat functions."""
    p = xy[tri]                                # [T, 3, 2]
    x, y = p[..., 0], p[..., 1]
    det = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    area = 0.5 * det
    grad = np.empty((tri.shape[0], 3, 2))
    # grad phi_k = (y_{k+1} - y_{k+2}, x_{k+2} - x_{k+1}) / (2 |T|)
    for k in range(3):
        k1, k2 = (k + 1) % 3, (k + 2) % 3
        grad[:, k, 0] = (y[:, k1] - y[:, k2]) / det
        grad[:, k, 1] = (x[:, k2] - x[:, k1]) / det
    return area, grad


def local_stiffness(xy: np.ndarray, tri: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """|T| grad(phi_a).grad(phi_b) for the three vertices: [n_tri, 3, 3]."""
    area, grad = element_geometry(xy, tri)
    return area[:, None, None] * np.einsum("tad,tbd->tab", grad, grad), area


def assemble(xy: np.ndarray, tri: np.ndarray, dof: np.ndarray, n: int,
             coef: np.ndarray) -> List[sp.csr_matrix]:
    """One stiffness matrix per row of ``coef`` ([L, n_tri], centroid values
    of the input PCE coefficients c_bar_i)."""
    kloc, _ = local_stiffness(xy, tri)
    d = dof[tri]                                       # [T, 3]
    out = []
    for ci in coef:
        rows, cols, vals = [], [], []
        for a in range(3):
            for b in range(3):
                m = (d[:, a] >= 0) & (d[:, b] >= 0)
                rows.append(d[m, a]); cols.append(d[m, b])
                vals.append(ci[m] * kloc[m, a, b])
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n)).tocsr()
        K.sum_duplicates()
        out.append(K)
    return out


def load_vector(xy: np.ndarray, tri: np.ndarray, dof: np.ndarray, n: int,
                f: float = 1.0) -> np.ndarray:
    """F[a] = sum over elements touching a of f |T| / 3 (constant forcing)."""
    _, area = local_stiffness(xy, tri)
    F = np.zeros(n)
    d = dof[tri]
    for a in range(3):
        m = d[:, a] >= 0
        np.add.at(F, d[m, a], f * area[m] / 3.0)
    return F


def load_vector_nodal(xy: np.ndarray, tri: np.ndarray, dof: np.ndarray, n: int,
                      fvals: np.ndarray) -> np.ndarray:
    """Lumped load for a variable forcing given at the vertices."""
    _, area = local_stiffness(xy, tri)
    F = np.zeros(n)
    d = dof[tri]
    for a in range(3):
        m = d[:, a] >= 0
        np.add.at(F, d[m, a], fvals[tri[m, a]] * area[m] / 3.0)
    return F
