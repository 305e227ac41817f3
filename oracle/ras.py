"""One-level restricted additive Schwarz (paper Sec. 3, Eqs. RASstofixedpoint
and RASsto).  Test infrastructure only.

M_RAS^{-1} = sum_s R_s^T D_s (R_s A R_s^T)^{-1} R_s with Boolean D_s and
sum_s R_s^T D_s R_s = I.

Readings (the paper is silent on these):
* Overlap: subdomain s starts from the nodes it owns and grows by ``delta``
  layers of neighbours in the mesh graph (edges of the triangulation).
  D_s keeps the owned nodes, so every node is written by exactly one
  subdomain.
* Local solve, mean-based: the block R_s A R_s^T of the SG operator is
  replaced by (R_s K_0 R_s^T) (x) G_0, solved exactly (dense Cholesky).
  The paper's own local solves are inexact too (ILU, Sec. 3); FGMRES
  accepts an inexact preconditioner.  G_0 = diag(alpha!) so the local
  solve is (R_s K_0 R_s^T)^{-1} X diag(1/alpha!).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def mesh_adjacency(tri: np.ndarray, dof: np.ndarray, n: int) -> sp.csr_matrix:
    """Boolean adjacency between unknowns sharing a triangle edge."""
    d = dof[tri]
    rows, cols = [], []
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            m = (d[:, a] >= 0) & (d[:, b] >= 0)
            rows.append(d[m, a]); cols.append(d[m, b])
    r = np.concatenate(rows); c = np.concatenate(cols)
    A = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
    A.data[:] = 1.0
    return A


def grow_overlap(owned: np.ndarray, adj: sp.csr_matrix, delta: int) -> np.ndarray:
    """Owned nodes plus every node within ``delta`` graph steps, sorted."""
    n = adj.shape[0]
    inside = np.zeros(n, dtype=bool)
    inside[owned] = True
    for _ in range(delta):
        reach = adj @ inside.astype(np.float64)
        inside |= reach > 0
    return np.nonzero(inside)[0]


@dataclass
class Subdomain:
    nodes: np.ndarray        # global ids of R_s, sorted
    owned: np.ndarray        # bool mask over ``nodes`` (D_s)
    chol: tuple              # scipy cho_factor of R_s K0 R_s^T


def ras_setup(K0: sp.csr_matrix, owner: np.ndarray, n_sub: int,
              adj: sp.csr_matrix, delta: int) -> List[Subdomain]:
    subs = []
    for s in range(n_sub):
        own = np.nonzero(owner == s)[0]
        nodes = grow_overlap(own, adj, delta)
        Aloc = K0[nodes][:, nodes].toarray()
        subs.append(Subdomain(nodes=nodes, owned=owner[nodes] == s,
                              chol=sla.cho_factor(Aloc, lower=True)))
    return subs


def ras_apply(subs: List[Subdomain], R: np.ndarray, alpha_fact: np.ndarray) -> np.ndarray:
    """Z = sum_s R_s^T D_s [(R_s K0 R_s^T)^{-1} (R_s R) G_0^{-1}]."""
    Z = np.zeros_like(R)
    for sd in subs:
        loc = sla.cho_solve(sd.chol, R[sd.nodes]) / alpha_fact[None, :]
        Z[sd.nodes[sd.owned]] = loc[sd.owned]
    return Z


def kron_factor(K: List[sp.csr_matrix], G: np.ndarray) -> np.ndarray:
    """Ullmann's Kronecker factor for SG operators (the Kronecker-product
    preconditioners the paper cites, Sec. 1): the P x P matrix Gt that makes
    K_0 (x) Gt closest to sum_i K_i (x) G_i in the Frobenius norm,
    Gt = sum_i (<K_i, K_0>_F / <K_0, K_0>_F) G_i."""
    t0 = K[0].multiply(K[0]).sum()
    return sum((Ki.multiply(K[0]).sum() / t0) * G[i] for i, Ki in enumerate(K))


def ras_apply_kron(subs: List[Subdomain], R: np.ndarray, Gt: np.ndarray) -> np.ndarray:
    """RAS with Kronecker local solves:
    Z = sum_s R_s^T D_s [(R_s K0 R_s^T)^{-1} (R_s R) Gt^{-1}]."""
    Gi = np.linalg.inv(Gt)
    Z = np.zeros_like(R)
    for sd in subs:
        loc = sla.cho_solve(sd.chol, R[sd.nodes]) @ Gi
        Z[sd.nodes[sd.owned]] = loc[sd.owned]
    return Z
