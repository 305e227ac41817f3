"""Conditioning of the SG operator against the deterministic one (paper
appendix, Tab. ss_cond).  Test infrastructure only.

kappa_SG is lambda_max / lambda_min of the SPD matrix sum_i K_i (x) G_i^
in the orthonormal chaos basis: G_i^ = D^{-1/2} G_i D^{-1/2} with
D = diag(<Psi_k^2>) = diag(alpha_k!), so that a rescaling of the basis
polynomials does not enter the figure.  kappa_det is that of K_0, the
stiffness matrix of the mean coefficient, which is the deterministic
problem the SG system reduces to at zero variance.  Both by dense symmetric
eigenvalues (small meshes only; the paper's table uses a 29-vertex mesh).

Reading: the paper does not say which deterministic problem or which basis
normalisation its ratios use; the mean-coefficient problem and the
orthonormal basis are the readings taken here.
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.sparse as sp


def sg_dense(K: List[sp.csr_matrix], G: np.ndarray, alpha_fact: np.ndarray) -> np.ndarray:
    """sum_i K_i (x) G_i^ as a dense (n P) x (n P) matrix, row a*P + k."""
    s = 1.0 / np.sqrt(np.asarray(alpha_fact, dtype=np.float64))
    A = None
    for i, Ki in enumerate(K):
        Gh = (s[:, None] * G[i]) * s[None, :]
        term = np.kron(Ki.toarray(), Gh)
        A = term if A is None else A + term
    return A


def condition(A: np.ndarray) -> float:
    w = np.linalg.eigvalsh(0.5 * (A + A.T))
    if not w[0] > 0:
        raise ValueError("matrix is not positive definite")
    return float(w[-1] / w[0])


def condition_ratio(K: List[sp.csr_matrix], G: np.ndarray, alpha_fact: np.ndarray):
    """(kappa_SG, kappa_det, kappa_SG / kappa_det)."""
    k_sg = condition(sg_dense(K, G, alpha_fact))
    k_det = condition(K[0].toarray() / float(alpha_fact[0]))
    return k_sg, k_det, k_sg / k_det
