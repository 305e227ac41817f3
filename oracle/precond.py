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

    omega = min(1, 1.8 / rho~),  rho~ = power estimate of rho(M_RAS A)

(15 power iterations, Rayleigh-free norm ratio, from a pseudo-random field:
entry i of the flattened node-major n x P array is output i + 1 of the
SplitMix64 generator from state 0 mapped to [-1/2, 1/2).  A smooth start
such as the all-ones field holds little of the oscillating modes at the top
of the spectrum, and 15 steps from it can underestimate rho by a factor 1.7
on fine partitions; omega rho > 2 then leaves the preconditioned operator
with eigenvalues near zero and FGMRES stalls.  From the pseudo-random start
the estimate is within a few per cent of rho, and the numerator 1.8 keeps
omega rho below 2 by that margin.)  For the deterministic problem
rho~ < 1.8 and the cycle is the paper's, undamped.

    z1 = omega M r
    z2 = z1 + Q (r - A z1)
    z  = z2 + omega M (r - A z2)
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from .coarse import prolong, restrict

POWER_ITS = 15
OMEGA_NUM = 1.8

_GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


def splitmix64(count: int, state: int = 0) -> np.ndarray:
    """Outputs 1..count of SplitMix64 (Steele, Lea and Flood, "Fast splittable
    pseudorandom number generators", OOPSLA 2014) from `state`: output i adds
    i times the golden-ratio increment to the state, then applies the
    generator's xor-shift-multiply finaliser (all modulo 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(state) + np.arange(1, count + 1, dtype=np.uint64) * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX2)
        return z ^ (z >> np.uint64(31))


def power_start(shape) -> np.ndarray:
    """The start of the power iteration: uniforms in [-1/2, 1/2) from the top
    53 bits of SplitMix64 outputs, in flattened row-major order."""
    n = int(np.prod(shape))
    return ((splitmix64(n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 - 0.5).reshape(shape)


def smoother_radius(matvec: Callable[[np.ndarray], np.ndarray],
                    ras: Callable[[np.ndarray], np.ndarray], shape,
                    its: int = POWER_ITS) -> float:
    v = power_start(shape)
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
