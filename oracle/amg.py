"""Smoothed-aggregation AMG on the coarse SG operator.  Test infrastructure
only.

The paper solves its coarse problem with BoomerAMG inside an inner GMRES
(2GV3, Sec. 3) and gives no AMG parameters.  This restates the fixed
definition used instead -- one V-cycle of smoothed aggregation on the block
matrix A_c (P x P blocks, one block-node per subdomain):

* strength: block-nodes s != t are strongly connected when
  |S_st| >= theta sqrt(|S_ss S_tt|), theta = 0.08, where S is the mean-mode
  entry of each block, A[(s,0),(t,0)] (on the first level S = Z^T K_0 Z);
* aggregation: the three greedy passes of Vanek, Mandel and Brezina in node
  order (1: a node whose strong neighbourhood is untouched seeds an
  aggregate with it; 2: a left-over node joins the pass-1 aggregate of its
  most strongly connected neighbour, ties to the lower index; 3: left-overs
  seed aggregates with their still-free strong neighbours);
* tentative prolongator: aggregate indicator (x) I_P, columns scaled to unit
  norm;
* smoothed prolongator: (I - omega D^{-1} A) P_tent, D the block diagonal,
  omega = (4/3)/rho(D^{-1} A), rho from 15 power iterations started from
  the all-ones vector;
* Galerkin coarse levels P^T A P, until <= 8 block-nodes or 4 levels;
* coarsest level solved exactly (dense Cholesky);
* V(1,1) with damped block-Jacobi, omega_s = 2/3, zero initial guess.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

THETA = 0.08
OMEGA_S = 2.0 / 3.0
MAX_LEVELS = 4
MIN_NODES = 8
POWER_ITS = 15


def strength_matrix(A: sp.csr_matrix, P: int) -> np.ndarray:
    idx = np.arange(A.shape[0] // P) * P
    return A[idx][:, idx].toarray()


def aggregate(S: np.ndarray, theta: float = THETA) -> np.ndarray:
    nn = S.shape[0]
    diag = np.abs(np.diag(S))
    nbrs = []
    for i in range(nn):
        js = [j for j in range(nn) if j != i and S[i, j] != 0.0
              and abs(S[i, j]) >= theta * np.sqrt(diag[i] * diag[j])]
        nbrs.append(js)
    agg = np.full(nn, -1, dtype=np.int64)
    n_agg = 0
    # pass 1
    for i in range(nn):
        if agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j in nbrs[i]):
            agg[i] = n_agg
            for j in nbrs[i]:
                agg[j] = n_agg
            n_agg += 1
    # pass 2
    snap = agg.copy()
    for i in range(nn):
        if agg[i] >= 0:
            continue
        best, best_v = -1, -1.0
        for j in nbrs[i]:
            if snap[j] >= 0 and abs(S[i, j]) > best_v:
                best, best_v = j, abs(S[i, j])
        if best >= 0:
            agg[i] = snap[best]
    # pass 3
    for i in range(nn):
        if agg[i] >= 0:
            continue
        agg[i] = n_agg
        for j in nbrs[i]:
            if agg[j] < 0:
                agg[j] = n_agg
        n_agg += 1
    return agg


def block_diag_inverse(A: sp.csr_matrix, P: int) -> sp.csr_matrix:
    nn = A.shape[0] // P
    Ad = A.toarray() if A.shape[0] <= 4096 else None
    blocks = []
    for s in range(nn):
        if Ad is not None:
            D = Ad[s * P:(s + 1) * P, s * P:(s + 1) * P]
        else:
            D = A[s * P:(s + 1) * P][:, s * P:(s + 1) * P].toarray()
        blocks.append(np.linalg.inv(D))
    return sp.block_diag(blocks, format="csr")


def tentative(agg: np.ndarray, P: int) -> sp.csr_matrix:
    nn = agg.size
    n_agg = int(agg.max()) + 1
    sizes = np.bincount(agg, minlength=n_agg).astype(np.float64)
    T = sp.csr_matrix((1.0 / np.sqrt(sizes[agg]), (np.arange(nn), agg)), shape=(nn, n_agg))
    return sp.kron(T, sp.identity(P), format="csr")


def spectral_radius(DinvA: sp.csr_matrix, its: int = POWER_ITS) -> float:
    v = np.ones(DinvA.shape[0])
    v /= np.linalg.norm(v)
    rho = 0.0
    for _ in range(its):
        w = DinvA @ v
        rho = np.linalg.norm(w)
        v = w / rho
    return float(rho)


@dataclass
class Hierarchy:
    P: int
    A: List[sp.csr_matrix] = field(default_factory=list)
    Dinv: List[sp.csr_matrix] = field(default_factory=list)
    Pr: List[sp.csr_matrix] = field(default_factory=list)
    aggs: List[np.ndarray] = field(default_factory=list)
    omegas: List[float] = field(default_factory=list)
    coarsest: tuple = None

    @property
    def n_levels(self) -> int:
        return len(self.A)


def setup(Ac: sp.csr_matrix, P: int, max_levels: int = MAX_LEVELS,
          min_nodes: int = MIN_NODES) -> Hierarchy:
    h = Hierarchy(P=P)
    A = Ac.tocsr()
    h.A.append(A)
    while len(h.A) < max_levels and A.shape[0] // P > min_nodes:
        agg = aggregate(strength_matrix(A, P))
        if agg.max() + 1 >= A.shape[0] // P:
            break
        Dinv = block_diag_inverse(A, P)
        T = tentative(agg, P)
        rho = spectral_radius((Dinv @ A).tocsr())
        omega = (4.0 / 3.0) / rho
        Pr = (T - omega * (Dinv @ (A @ T))).tocsr()
        h.Dinv.append(Dinv)
        h.Pr.append(Pr)
        h.aggs.append(agg)
        h.omegas.append(omega)
        A = (Pr.T @ A @ Pr).tocsr()
        h.A.append(A)
    h.coarsest = sla.cho_factor(h.A[-1].toarray(), lower=True)
    return h


def vcycle(h: Hierarchy, b: np.ndarray, level: int = 0) -> np.ndarray:
    """One V(1,1) cycle for A_level x = b, zero initial guess (flat vectors)."""
    if level == h.n_levels - 1:
        return sla.cho_solve(h.coarsest, b)
    A, Dinv, Pr = h.A[level], h.Dinv[level], h.Pr[level]
    x = OMEGA_S * (Dinv @ b)
    r = b - A @ x
    x = x + Pr @ vcycle(h, Pr.T @ r, level + 1)
    x = x + OMEGA_S * (Dinv @ (b - A @ x))
    return x


class AMGCoarse:
    """Coarse solve by one V-cycle on A_c ([n_sub, P] in and out)."""

    def __init__(self, Ac: sp.csr_matrix, P: int):
        self.h = setup(Ac, P)

    def __call__(self, rc: np.ndarray) -> np.ndarray:
        return vcycle(self.h, rc.ravel()).reshape(rc.shape)
