"""Statistics of an SG solution and sampling-based cross-checks (paper
Sec. 4.1: the SG mean and standard deviation are verified against Monte
Carlo samples).  Test infrastructure only.

mean(u)     = u_bar_0
var(u)      = sum_{alpha != 0} alpha! u_bar_alpha^2     (orthogonality of Psi)
"""
from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .pce import psi_eval


def pce_mean_var(U: np.ndarray, alpha_fact: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    return U[:, 0].copy(), (U[:, 1:] ** 2 * alpha_fact[None, 1:]).sum(axis=1)


def sample_solve(K: List[sp.csr_matrix], alpha_in: np.ndarray, F: np.ndarray,
                 xi: np.ndarray) -> np.ndarray:
    """Deterministic solves for the truncated input c_L(x, xi) =
    sum_i c_bar_i(x) Psi_i(xi): K(xi) = sum_i Psi_i(xi) K_i (K is linear in
    the coefficient).  xi: [S, M] -> [S, n]."""
    psi = psi_eval(alpha_in, xi)
    out = np.empty((xi.shape[0], F.shape[0]))
    for s in range(xi.shape[0]):
        Ks = K[0] * psi[s, 0]
        for i in range(1, len(K)):
            Ks = Ks + K[i] * psi[s, i]
        out[s] = spla.spsolve(Ks.tocsc(), F)
    return out


def collocation_moments(K: List[sp.csr_matrix], alpha_in: np.ndarray, F: np.ndarray,
                        M: int, q: int) -> Tuple[np.ndarray, np.ndarray]:
    """Mean and variance of the solution of the truncated-input problem by a
    tensor Gauss-Hermite rule with q points per variable."""
    from numpy.polynomial.hermite_e import hermegauss
    x, w = hermegauss(q)
    w = w / w.sum()
    grids = np.meshgrid(*([x] * M), indexing="ij")
    wg = np.meshgrid(*([w] * M), indexing="ij")
    xi = np.stack([g.ravel() for g in grids], axis=1)
    wt = np.prod(np.stack([g.ravel() for g in wg], axis=1), axis=1)
    u = sample_solve(K, alpha_in, F, xi)
    mean = wt @ u
    var = wt @ (u - mean) ** 2
    return mean, var
