"""Polynomial chaos pieces (paper Sec. 2.1, Eqs. inputpc, inputlogn, outpc,
Galerkin_L_exp).  Test infrastructure only.

Basis: probabilists' Hermite polynomials He_n, un-normalised, so that
<Psi_a^2> = a! (the denominators of Eq. inputlogn).  Multi-indices with total
degree <= p are ordered by total degree, then descending lexicographically
(1, xi1, xi2, xi1^2-1, xi1 xi2, xi2^2-1 for M=2, p=2).  The input basis
(order p_in) is a prefix of the output basis, so an index names the same
polynomial in both.
"""
from __future__ import annotations

from math import comb, factorial
from typing import List, Tuple

import numpy as np


def multi_indices(M: int, p: int) -> np.ndarray:
    """All alpha in N^M with |alpha| <= p, in the order described above.
    The count is (M+p)!/(M!p!) (the term count below Eq. inputpc)."""
    out: List[Tuple[int, ...]] = []
    for d in range(p + 1):
        level: List[Tuple[int, ...]] = []

        def rec(prefix, left, slots):
            if slots == 1:
                level.append(prefix + (left,))
                return
            for v in range(left, -1, -1):
                rec(prefix + (v,), left - v, slots - 1)

        if M == 0:
            if d == 0:
                out.append(())
            continue
        rec((), d, M)
        out.extend(level)       # rec emits descending lexicographic order
    if M == 0:
        return np.zeros((1, 0), dtype=np.int64)
    return np.array(out, dtype=np.int64)


def n_terms(M: int, p: int) -> int:
    return comb(M + p, p)


def alpha_factorial(alpha: np.ndarray) -> np.ndarray:
    """<Psi_alpha^2> = prod_m alpha_m!."""
    return np.array([np.prod([factorial(int(v)) for v in a]) if len(a) else 1.0
                     for a in alpha], dtype=np.float64)


def hermite_triple_1d(a: int, b: int, c: int) -> int:
    """<He_a He_b He_c> for a standard Gaussian variable.  With a+b+c = 2s it
    equals a!b!c!/((s-a)!(s-b)!(s-c)!) when s >= max(a,b,c), else 0 (the
    classical linearisation formula of Hermite products)."""
    tot = a + b + c
    if tot % 2:
        return 0
    s = tot // 2
    if s < a or s < b or s < c:
        return 0
    return (factorial(a) * factorial(b) * factorial(c)
            // (factorial(s - a) * factorial(s - b) * factorial(s - c)))


def triple_products(M: int, p_in: int, p: int):
    """m_ijk = <Psi_i Psi_j Psi_k> (Eq. Galerkin_L_exp) for i over the input
    basis and j, k over the output basis; only non-zeros are kept (the paper
    stores "only the non-zero entries" of the multiplication tensor).

    Returns (alpha, ijk [T,3] int64, val [T] float64, L_in, P)."""
    alpha = multi_indices(M, p)
    P = alpha.shape[0]
    L_in = n_terms(M, p_in)
    rows, vals = [], []
    for i in range(L_in):
        for j in range(P):
            for k in range(P):
                m = 1
                for d in range(M):
                    m *= hermite_triple_1d(int(alpha[i, d]), int(alpha[j, d]), int(alpha[k, d]))
                    if m == 0:
                        break
                if m != 0:
                    rows.append((i, j, k))
                    vals.append(float(m))
    ijk = np.array(rows, dtype=np.int64).reshape(-1, 3)
    return alpha, ijk, np.array(vals, dtype=np.float64), L_in, P


def g_matrices(ijk: np.ndarray, val: np.ndarray, L_in: int, P: int) -> np.ndarray:
    """Dense G_i with (G_i)[k, j] = m_ijk, shape [L_in, P, P]."""
    G = np.zeros((L_in, P, P))
    for (i, j, k), v in zip(ijk, val):
        G[i, k, j] = v
    return G


def lognormal_coefficients(g0: np.ndarray, g: np.ndarray, alpha_in: np.ndarray) -> np.ndarray:
    """Input PCE coefficients of c = exp(g0 + sum_m g_m xi_m) (Eq. inputlogn).

    c_bar_alpha(x) = c0(x) prod_m g_m(x)^alpha_m / alpha_m!, with the mean
    c0 = exp(g0 + 1/2 sum_m g_m^2) (the equation following Eq. inputlogn).

    Reading: the paper writes <Psi_i(eta)> with eta = xi - g; taken
    literally that flips the sign of every odd-order coefficient.  The
    expansion of exp(g . xi) in Hermite polynomials (generating function
    exp(t x - t^2/2) = sum He_n(x) t^n / n!) fixes eta = xi + g, which is
    what is computed here.

    g0: [n_pts], g: [M, n_pts] -> [L_in, n_pts]."""
    M = g.shape[0]
    c0 = np.exp(g0 + 0.5 * (g ** 2).sum(axis=0))
    out = np.empty((alpha_in.shape[0], g0.shape[0]))
    for r, a in enumerate(alpha_in):
        term = c0.copy()
        for m in range(M):
            if a[m]:
                term = term * g[m] ** int(a[m]) / factorial(int(a[m]))
        out[r] = term
    return out


def psi_eval(alpha: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Psi_alpha(xi) for xi [S, M] -> [S, P] (probabilists' Hermite)."""
    from numpy.polynomial.hermite_e import hermeval
    S = xi.shape[0]
    out = np.ones((S, alpha.shape[0]))
    for r, a in enumerate(alpha):
        for m, deg in enumerate(a):
            if deg:
                cvec = np.zeros(int(deg) + 1); cvec[-1] = 1.0
                out[:, r] *= hermeval(xi[:, m], cvec)
    return out
