"""Flexible GMRES(m) with right preconditioning (Saad 1993; the outer solver
of the paper, Sec. 3 and Sec. 4).  Test infrastructure only.

* Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
  matrix, all in FP64.
* Stopping test relative to the norm of the right-hand side (the PETSc
  convention the paper states in Sec. 3), so a good initial guess helps.
* When the Givens estimate passes, the true residual ||b - A x|| is
  computed; if it does not pass, the method restarts from x.
* h_{j+1,j} = 0 (lucky breakdown) ends the cycle: the Krylov space holds
  the solution.
Vectors are [n, P] arrays; inner products are Frobenius.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class KrylovInfo:
    iterations: int = 0
    converged: bool = False
    history: List[float] = field(default_factory=list)   # estimates / ||b||
    true_relres: float = float("nan")
    restarts: int = 0


def _dot(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.dot(a.ravel(), b.ravel()))


def fgmres(A: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
           precond: Optional[Callable[[np.ndarray], np.ndarray]] = None,
           x0: Optional[np.ndarray] = None, m: int = 30, rtol: float = 1e-8,
           max_it: int = 1000) -> tuple:
    B = precond if precond is not None else (lambda v: v.copy())
    x = np.zeros_like(b) if x0 is None else x0.copy()
    info = KrylovInfo()
    bnorm = np.sqrt(_dot(b, b))
    if bnorm == 0.0:
        info.converged = True
        info.true_relres = 0.0
        return np.zeros_like(b), info
    target = rtol * bnorm
    r = b - A(x)
    beta = np.sqrt(_dot(r, r))
    info.history.append(beta / bnorm)
    if beta <= target:
        info.converged = True
        info.true_relres = beta / bnorm
        return x, info
    while info.iterations < max_it:
        V = [r / beta]
        Zs = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m); sn = np.zeros(m)
        g = np.zeros(m + 1); g[0] = beta
        j_done = 0
        for j in range(m):
            z = B(V[j])
            Zs.append(z)
            w = A(z)
            for i in range(j + 1):
                H[i, j] = _dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.sqrt(_dot(w, w))
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V.append(w / H[j + 1, j])
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info.iterations += 1
            j_done = j + 1
            info.history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= target or breakdown or info.iterations >= max_it:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        for i in range(j_done):
            x = x + y[i] * Zs[i]
        r = b - A(x)
        beta = np.sqrt(_dot(r, r))
        info.true_relres = beta / bnorm
        if beta <= target:
            info.converged = True
            return x, info
        info.restarts += 1
    return x, info
