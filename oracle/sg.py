"""The coupled stochastic Galerkin system (paper Eq. Galerkin_L_exp and its
vector-PDE form, Eqs. linearVecPDE / Ajklinear).  Test infrastructure only.

Layout: an SG field is an [n, P] array U with U[a, j] = u_bar_j(x_a); in the
flat vector of the vector-PDE form, node a's P coefficients are contiguous
(row index a*P + k).  The operator is

    Y = sum_i K_i X G_i,      (G_i)[k, j] = m_ijk,

i.e. the Kronecker sum  sum_i K_i (x) G_i  acting on the row-major flattening.
The right-hand side is b_k = f <Psi_k> = f delta_k0, so only column 0 of B
is non-zero.
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def sg_matvec(K: List[sp.csr_matrix], G: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Y = sum_i K_i X G_i  (G_i symmetric)."""
    Y = np.zeros_like(X)
    for i, Ki in enumerate(K):
        Y += Ki @ (X @ G[i].T)
    return Y


def sg_rhs(F: np.ndarray, P: int) -> np.ndarray:
    B = np.zeros((F.shape[0], P))
    B[:, 0] = F
    return B


def sg_kron(K: List[sp.csr_matrix], G: np.ndarray) -> sp.csr_matrix:
    """Explicit sum_i K_i (x) G_i in the row-major (a*P + k) numbering."""
    A = None
    for i, Ki in enumerate(K):
        t = sp.kron(Ki, sp.csr_matrix(G[i]), format="csr")
        A = t if A is None else A + t
    return A.tocsr()


def sg_solve_direct(K: List[sp.csr_matrix], G: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Reference solution U* by a sparse direct solve of the Kronecker form."""
    A = sg_kron(K, G)
    u = spla.spsolve(A.tocsc(), B.ravel())
    return u.reshape(B.shape)
