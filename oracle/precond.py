"""The two-grid multiplicative Schwarz preconditioner (paper Sec. 3,
Eq. RAS_2L).  Test infrastructure only.

Reading 1: as printed, Eq. RAS_2L contains Q P Q^{-1}, and
Q = R_0^T A_c^{-1} R_0 is singular.  Formally Q P Q^{-1} = Q (I - A Q) Q^{-1}
= I - Q A = P^T, and with that substitution the formula is exactly the
three-step cycle the text describes (RAS pre-smoothing, coarse correction of
the residual, RAS post-smoothing).  It is applied in that order and never
formed.

Reading 2: the paper's smoother solves the full local SG block by ILU.  With
the mean-based local solve used here, rho(M_RAS A) exceeds 2 once the input
variance is moderate, and the undamped multiplicative cycle amplifies error
(it stalls for sigma = 0.5).  The smoother is therefore damped:

    omega = min(1, 1.6 / rho~),  rho~ = power estimate of rho(M_RAS A)

(15 power iterations from the all-ones field, Rayleigh-free norm ratio, the
same recipe as the AMG prolongator damping).  For the deterministic problem
rho~ < 1.6 and the cycle is the paper's, undamped.

    z1 = omega M r
    z2 = z1 + Q (r - A z1)
    z  = z2 + omega M (r - A z2)
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from .coarse import prolong, restrict

POWER_ITS = 15
OMEGA_NUM = 1.6


def smoother_radius(matvec: Callable[[np.ndarray], np.ndarray],
                    ras: Callable[[np.ndarray], np.ndarray], shape,
                    its: int = POWER_ITS) -> float:
    v = np.ones(shape)
    v /= np.linalg.norm(v)
    rho = 0.0
    for _ in range(its):
        w = ras(matvec(v))
        rho = float(np.linalg.norm(w))
        v = w / rho
    return rho


def smoother_damping(rho: float) -> float:
    return min(1.0, OMEGA_NUM / rho)


class TwoLevel:
    def __init__(self, matvec: Callable[[np.ndarray], np.ndarray],
                 ras: Callable[[np.ndarray], np.ndarray],
                 Z, coarse_solve: Callable[[np.ndarray], np.ndarray],
                 omega: float = 1.0):
        self.A = matvec
        self.M = ras
        self.Z = Z
        self.coarse = coarse_solve
        self.omega = omega

    def coarse_correction(self, r: np.ndarray) -> np.ndarray:
        return prolong(self.Z, self.coarse(restrict(self.Z, r)))

    def __call__(self, r: np.ndarray) -> np.ndarray:
        z1 = self.omega * self.M(r)
        z2 = z1 + self.coarse_correction(r - self.A(z1))
        return z2 + self.omega * self.M(r - self.A(z2))
