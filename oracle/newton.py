"""Nonlinear stochastic Galerkin Poisson problem and Newton's method.
Test infrastructure only.

The paper's nonlinear model is -div(c(x,theta)(1 + alpha u) grad u) = f
(Eq. NLP_StrongPDE), linearised by Picard iterations (Eq. stonlp_system,
Eq. vectorvalPDENL).  Here kappa(u) = 1 + a1 u + a2 u^2: the paper's model is
a1 = alpha, a2 = 0; the Newton configuration uses a1 = 0, a2 = 0.5.  The
Galerkin system is solved by Newton's method or by the paper's Picard
iteration (``picard``: U <- K1(U)^{-1} F e_0 with the secant operator K1,
A(U) = K1(U) U, until ||U_{k+1} - U_k|| <= du_tol ||U_{k+1}||).

Exact-Galerkin residual, with u_b(xi) = sum_j U[b, j] Psi_j(xi):

  A(U)[a, m] = sum_T |T| E[ c_T(xi) kappa(u_T(xi)) (grad u_T(xi) . grad phi_a) Psi_m(xi) ]
  R(U)       = F e_0 - A(U)

c_T = sum_{i < L_in} c_bar_i(x_T) Psi_i (the truncated input PCE at the
centroid, as in the linear operator), u_T = (1/3) sum_{b in T} u_b (centroid
value), grad u_T = sum_{b in T} grad phi_b u_b.  The Jacobian dA/dU is

  J[(a,m),(b,n)] = sum_T |T| { E[c kappa(u_T) Psi_n Psi_m] grad phi_b . grad phi_a
                              + (1/3) E[c kappa'(u_T) (grad u_T . grad phi_a) Psi_n Psi_m] }.

The integrands are polynomials in xi of degree <= 2 + 2*2p + p + p = 14 for
p = 3, so a tensor Gauss-Hermite rule with 8 points per variable evaluates
the expectations exactly (up to rounding).

Newton: eta_k = max(1e-12, min(1e-2, ||R_k||/||F||)), raised to at least
0.5 tol ||F|| / ||R_k|| (capped at 1e-2) so that the last correction is not
solved beyond the final tolerance (||F|| replaced by the initial residual
when F = 0); backtracking tries lambda = 1, 1/2, ...,
1/512 until ||R(U + lambda d)|| <= (1 - 1e-4 lambda) ||R(U)|| and takes the
last trial if none passes; stop when ||R||/||F|| <= tol.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, pce


def gauss_hermite_tensor(M: int, q: int = 8):
    """Tensor probabilists' Gauss-Hermite rule: points [q^M, M], weights
    summing to one."""
    from numpy.polynomial.hermite_e import hermegauss
    if M == 0:
        return np.zeros((1, 0)), np.ones(1)
    x, w = hermegauss(q)
    w = w / w.sum()
    grids = np.meshgrid(*([x] * M), indexing="ij")
    wg = np.meshgrid(*([w] * M), indexing="ij")
    pts = np.stack([g.ravel() for g in grids], axis=1)
    wts = np.prod(np.stack([g.ravel() for g in wg], axis=1), axis=1)
    return pts, wts


@dataclass
class NLProblem:
    xy: np.ndarray
    tri: np.ndarray
    dof: np.ndarray
    n: int
    coef: np.ndarray          # [L, n_tri]
    alpha: np.ndarray         # [P, M]
    L: int
    P: int
    a2: float = 0.5
    a1: float = 0.0
    uD: Optional[np.ndarray] = None      # Dirichlet value per vertex (deterministic)
    fvals: Optional[np.ndarray] = None   # forcing per vertex (default 1)
    # derived
    area: np.ndarray = field(default=None)
    grad: np.ndarray = field(default=None)
    psi: np.ndarray = field(default=None)      # [Q, P]
    wq: np.ndarray = field(default=None)       # [Q]
    F: np.ndarray = field(default=None)        # [n]

    def __post_init__(self):
        self.area, self.grad = fem.element_geometry(self.xy, self.tri)
        M = self.alpha.shape[1]
        pts, self.wq = gauss_hermite_tensor(M, 8)
        self.psi = pce.psi_eval(self.alpha, pts) if M else np.ones((1, self.P))
        if self.fvals is None:
            self.F = fem.load_vector(self.xy, self.tri, self.dof, self.n)
        else:
            self.F = fem.load_vector_nodal(self.xy, self.tri, self.dof, self.n, self.fvals)

    def kappa(self, u):
        return 1.0 + self.a1 * u + self.a2 * u * u

    def dkappa(self, u):
        return self.a1 + 2.0 * self.a2 * u

    def _vertex_fields(self, U: np.ndarray, el: np.ndarray) -> np.ndarray:
        """u_b(xi_q) for the 3 vertices of elements el: [E, 3, Q]."""
        d = self.dof[self.tri[el]]                            # [E, 3]
        Ue = np.zeros((el.size, 3, self.P))
        m = d >= 0
        Ue[m] = U[d[m]]
        if self.uD is not None:
            v = self.tri[el]
            Ue[..., 0] += np.where(m, 0.0, self.uD[v])
        return Ue @ self.psi.T

    def residual(self, U: np.ndarray, chunk: int = 128) -> np.ndarray:
        R = np.zeros((self.n, self.P))
        R[:, 0] = self.F
        for e0 in range(0, self.tri.shape[0], chunk):
            el = np.arange(e0, min(e0 + chunk, self.tri.shape[0]))
            ub = self._vertex_fields(U, el)                            # [E,3,Q]
            c = self.coef[:, el].T @ self.psi[:, :self.L].T           # [E,Q]
            uT = ub.mean(axis=1)                                       # [E,Q]
            g = self.grad[el]                                          # [E,3,2]
            gu = np.einsum("ebd,ebq->eqd", g, ub)                      # [E,Q,2]
            flux = np.einsum("eqd,ead->eaq", gu, g)                    # [E,3,Q]
            wt = self.wq[None, :] * c * self.kappa(uT)                 # [E,Q]
            contrib = self.area[el, None, None] * ((flux * wt[:, None, :]) @ self.psi)  # [E,3,P]
            d = self.dof[self.tri[el]]
            for a in range(3):
                m = d[:, a] >= 0
                np.add.at(R, d[m, a], -contrib[m, a])
        return R

    def secant(self, U: np.ndarray) -> sp.csr_matrix:
        """K1(U) with A(U) = K1(U) U: the first term of the Jacobian,
        sum_T |T| E[c kappa(u_T) Psi_m Psi_n] grad phi_b . grad phi_a."""
        return self.jacobian(U, with_dkappa=False)

    def jacobian(self, U: np.ndarray, chunk: int = 16, with_dkappa: bool = True) -> sp.csr_matrix:
        """dA/dU in the row-major (a*P + m) numbering (without the kappa'
        term: the secant operator K1(U))."""
        P = self.P
        rows, cols, vals = [], [], []
        idx = np.arange(P)
        for e0 in range(0, self.tri.shape[0], chunk):
            el = np.arange(e0, min(e0 + chunk, self.tri.shape[0]))
            ub = self._vertex_fields(U, el)
            c = self.coef[:, el].T @ self.psi[:, :self.L].T
            uT = ub.mean(axis=1)
            g = self.grad[el]
            gu = np.einsum("ebd,ebq->eqd", g, ub)
            w1 = self.wq[None, :] * c * self.kappa(uT)                            # [E,Q]
            # E1[e,m,n] = sum_q w1[e,q] psi[q,m] psi[q,n]  (as a batched matmul)
            E1 = self.psi.T[None] @ (w1[:, :, None] * self.psi[None])           # [E,P,P]
            w2 = self.wq[None, None, :] * (c * self.dkappa(uT))[:, None, :] * \
                np.einsum("eqd,ead->eaq", gu, g)                                 # [E,3,Q]
            E2 = self.psi.T[None, None] @ (w2[..., None] * self.psi[None, None])  # [E,3,P,P]
            gg = np.einsum("ead,ebd->eab", g, g)                                   # [E,3,3]
            d = self.dof[self.tri[el]]
            for a in range(3):
                for b in range(3):
                    m = (d[:, a] >= 0) & (d[:, b] >= 0)
                    if not m.any():
                        continue
                    blk = self.area[el[m], None, None] * (
                        E1[m] * gg[m, a, b][:, None, None] +
                        (E2[m, a] / 3.0 if with_dkappa else 0.0))                   # [E,P(m),P(n)]
                    ra = d[m, a][:, None, None] * P + idx[None, :, None]
                    cb = d[m, b][:, None, None] * P + idx[None, None, :]
                    rows.append(np.broadcast_to(ra, blk.shape).ravel())
                    cols.append(np.broadcast_to(cb, blk.shape).ravel())
                    vals.append(blk.ravel())
        N = self.n * P
        J = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsr()
        J.sum_duplicates()
        return J

    def mean_stiffness(self, U: np.ndarray, chunk: int = 128) -> sp.csr_matrix:
        """Scalar stiffness with the element coefficient E[c kappa(u_T)]: the
        mean-coefficient part of the Jacobian, used by the preconditioner."""
        cm = np.zeros(self.tri.shape[0])
        for e0 in range(0, self.tri.shape[0], chunk):
            el = np.arange(e0, min(e0 + chunk, self.tri.shape[0]))
            ub = self._vertex_fields(U, el)
            c = self.coef[:, el].T @ self.psi[:, :self.L].T
            cm[el] = (self.wq[None, :] * c * self.kappa(ub.mean(axis=1))).sum(axis=1)
        return fem.assemble(self.xy, self.tri, self.dof, self.n, cm[None, :])[0]


@dataclass
class NewtonInfo:
    steps: int = 0
    krylov_its: List[int] = field(default_factory=list)
    residuals: List[float] = field(default_factory=list)
    lambdas: List[float] = field(default_factory=list)
    converged: bool = False


def newton(pr: NLProblem, U0: Optional[np.ndarray] = None, tol: float = 1e-8,
           max_steps: int = 30,
           linear_solve: Optional[Callable] = None) -> tuple:
    """Inexact Newton with backtracking.  ``linear_solve(J, R, eta, U)`` returns
    (d, its); by default a sparse direct solve (its = 0)."""
    U = np.zeros((pr.n, pr.P)) if U0 is None else U0.copy()
    info = NewtonInfo()
    R = pr.residual(U)
    rn = np.linalg.norm(R)
    # residuals are relative to ||F|| (to the initial residual when F = 0,
    # e.g. a problem driven only by its boundary data)
    Fn = np.linalg.norm(pr.F) if np.linalg.norm(pr.F) > 0 else rn
    info.residuals.append(rn / Fn)
    while info.steps < max_steps:
        if rn / Fn <= tol:
            info.converged = True
            break
        J = pr.jacobian(U)
        eta = max(1e-12, min(1e-2, rn / Fn))
        # no more accuracy than the final tolerance needs
        eta = min(1e-2, max(eta, 0.5 * tol * Fn / rn))
        if linear_solve is None:
            d = spla.spsolve(J.tocsc(), R.ravel()).reshape(R.shape)
            its = 0
        else:
            d, its = linear_solve(J, R, eta, U)
        lam = 1.0
        for trial in range(10):
            Rt = pr.residual(U + lam * d)
            if np.linalg.norm(Rt) <= (1.0 - 1e-4 * lam) * rn or trial == 9:
                break
            lam *= 0.5
        U = U + lam * d
        R = Rt
        rn = np.linalg.norm(R)
        info.steps += 1
        info.krylov_its.append(its)
        info.lambdas.append(lam)
        info.residuals.append(rn / Fn)
    if rn / Fn <= tol:
        info.converged = True
    return U, info


@dataclass
class PicardInfo:
    steps: int = 0
    du: List[float] = field(default_factory=list)          # ||U_{k+1} - U_k|| / ||U_{k+1}||
    residuals: List[float] = field(default_factory=list)   # ||R(U_k)|| / ||F||
    krylov_its: List[int] = field(default_factory=list)
    converged: bool = False


def picard(pr: NLProblem, U0: Optional[np.ndarray] = None, du_tol: float = 1e-6,
           max_steps: int = 100, linear_solve: Optional[Callable] = None) -> tuple:
    """The paper's Picard iteration on the Galerkin system: solve
    K1(U_k) U_{k+1} = F e_0, written as the correction K1(U_k) d = R(U_k),
    U_{k+1} = U_k + d (full step), until ||d|| <= du_tol ||U_{k+1}||.
    ``linear_solve(K1, R, U)`` returns (d, its); by default a direct solve."""
    U = np.zeros((pr.n, pr.P)) if U0 is None else U0.copy()
    info = PicardInfo()
    R = pr.residual(U)
    Fn = np.linalg.norm(pr.F) if np.linalg.norm(pr.F) > 0 else np.linalg.norm(R)
    info.residuals.append(np.linalg.norm(R) / Fn)
    while info.steps < max_steps:
        K1 = pr.secant(U)
        if linear_solve is None:
            d = spla.spsolve(K1.tocsc(), R.ravel()).reshape(R.shape)
            its = 0
        else:
            d, its = linear_solve(K1, R, U)
        U = U + d
        R = pr.residual(U)
        info.steps += 1
        info.krylov_its.append(its)
        info.residuals.append(np.linalg.norm(R) / Fn)
        un = np.linalg.norm(U)
        info.du.append(np.linalg.norm(d) / un if un > 0 else np.linalg.norm(d))
        if info.du[-1] <= du_tol:
            info.converged = True
            break
    return U, info


def build(xy, tri, dof, n, g0, g, M, p_in, p, a2=0.5, a1=0.0, **kw) -> NLProblem:
    alpha = pce.multi_indices(M, p)
    L = pce.n_terms(M, p_in)
    coef = pce.lognormal_coefficients(g0, g, alpha[:L])
    return NLProblem(xy=xy, tri=tri, dof=dof, n=n, coef=coef, alpha=alpha, L=L,
                     P=alpha.shape[0], a2=a2, a1=a1, **kw)
