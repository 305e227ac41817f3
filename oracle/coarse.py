"""Coarse space of the two-grid preconditioner (paper Sec. 3, Eq. coarse:
A_c = R_0 A R_0^T).  Test infrastructure only.

Reading: the paper builds R_0 from a coarser triangulation; here the
coarse space is Nicolaides' -- one vector per subdomain and PCE mode,
Z_s = R_s^T D_s 1, i.e. the indicator of the nodes that subdomain s owns --
so R_0 = Z^T with Z = [Z_s (x) e_k].  Then

    A_c = Z^T A Z = sum_i (Z^T K_i Z) (x) G_i,   C_i := Z^T K_i Z,

has the same Kronecker-sum structure as the fine operator, on the graph of
subdomains.  Coarse vectors are [n_sub, P] arrays (index s*P + k).
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .sg import sg_kron


def nicolaides(owner: np.ndarray, n_sub: int) -> sp.csr_matrix:
    n = owner.shape[0]
    return sp.csr_matrix((np.ones(n), (np.arange(n), owner)), shape=(n, n_sub))


def coarse_blocks(K: List[sp.csr_matrix], Z: sp.csr_matrix) -> List[sp.csr_matrix]:
    """C_i = Z^T K_i Z, one [n_sub, n_sub] matrix per input PCE term."""
    return [(Z.T @ Ki @ Z).tocsr() for Ki in K]


def coarse_operator(C: List[sp.csr_matrix], G: np.ndarray) -> sp.csr_matrix:
    return sg_kron(C, G)


def restrict(Z: sp.csr_matrix, R: np.ndarray) -> np.ndarray:
    return np.asarray(Z.T @ R)


def prolong(Z: sp.csr_matrix, E: np.ndarray) -> np.ndarray:
    return np.asarray(Z @ E)


class MeanExactCoarse:
    """Mean-based coarse solve: (C_0 (x) G_0)^{-1}, exact.  This is the
    reading of a "mean-based coarse solve" for the smallest configuration."""

    def __init__(self, C: List[sp.csr_matrix], alpha_fact: np.ndarray):
        self.chol = sla.cho_factor(C[0].toarray(), lower=True)
        self.alpha_fact = alpha_fact

    def __call__(self, rc: np.ndarray) -> np.ndarray:
        return sla.cho_solve(self.chol, rc) / self.alpha_fact[None, :]


class ExactCoarse:
    """A_c^{-1} by a dense factorisation (for small problems and pins)."""

    def __init__(self, C: List[sp.csr_matrix], G: np.ndarray):
        self.P = G.shape[1]
        Ac = coarse_operator(C, G).toarray()
        self.lu = sla.lu_factor(Ac)

    def __call__(self, rc: np.ndarray) -> np.ndarray:
        return sla.lu_solve(self.lu, rc.ravel()).reshape(rc.shape)
