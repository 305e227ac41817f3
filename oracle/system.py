"""Assembly of a whole linear SG problem from the generator's arrays, and the
solver built on it (paper Secs. 2-3).  Test infrastructure only."""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp

from . import amg, coarse, fem, krylov, pce, ras, sg
from .precond import TwoLevel, smoother_damping, smoother_radius


@dataclass
class SGSystem:
    alpha: np.ndarray
    ijk: np.ndarray
    val: np.ndarray
    L_in: int
    P: int
    G: np.ndarray
    alpha_fact: np.ndarray
    coef: np.ndarray            # [L_in, n_tri]
    K: List[sp.csr_matrix]
    F: np.ndarray
    B: np.ndarray
    adj: sp.csr_matrix

    def matvec(self, X: np.ndarray) -> np.ndarray:
        return sg.sg_matvec(self.K, self.G, X)


def build(xy, tri, dof, n, g0, g, M, p_in, p) -> SGSystem:
    alpha, ijk, val, L_in, P = pce.triple_products(M, p_in, p)
    G = pce.g_matrices(ijk, val, L_in, P)
    coef = pce.lognormal_coefficients(g0, g, alpha[:L_in])
    K = fem.assemble(xy, tri, dof, n, coef)
    F = fem.load_vector(xy, tri, dof, n)
    return SGSystem(alpha=alpha, ijk=ijk, val=val, L_in=L_in, P=P, G=G,
                    alpha_fact=pce.alpha_factorial(alpha), coef=coef, K=K, F=F,
                    B=sg.sg_rhs(F, P), adj=ras.mesh_adjacency(tri, dof, n))


def two_level(S: SGSystem, owner: np.ndarray, n_sub: int, delta: int,
              coarse_kind: str = "amg", omega=None):
    subs = ras.ras_setup(S.K[0], owner, n_sub, S.adj, delta)
    Z = coarse.nicolaides(owner, n_sub)
    C = coarse.coarse_blocks(S.K, Z)
    if coarse_kind == "mean":
        cs = coarse.MeanExactCoarse(C, S.alpha_fact)
    elif coarse_kind == "exact":
        cs = coarse.ExactCoarse(C, S.G)
    elif coarse_kind == "amg":
        cs = amg.AMGCoarse(coarse.coarse_operator(C, S.G), S.P)
    else:
        raise ValueError(coarse_kind)
    M = lambda R: ras.ras_apply(subs, R, S.alpha_fact)  # noqa: E731
    if omega is None:
        omega = smoother_damping(smoother_radius(S.matvec, M, S.B.shape))
    return TwoLevel(S.matvec, M, Z, cs, omega=omega), subs, C, cs


def solve(S: SGSystem, precond, m: int, rtol: float, max_it: int = 1000, x0=None):
    return krylov.fgmres(S.matvec, S.B, precond, x0=x0, m=m, rtol=rtol, max_it=max_it)
