"""Pins of the oracle's polynomial-chaos pieces against facts fixed outside
the oracle: the printed term counts, Gauss-Hermite quadrature of the
Hermite products, and the Gaussian moment generating function."""
import os
from math import comb, factorial

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss, hermeval

from oracle import pce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _he(n, x):
    c = np.zeros(n + 1)
    c[-1] = 1.0
    return hermeval(x, c)


def _quad_expect(alpha_rows, M, q=12):
    """E[prod_r Psi_{alpha_r}(xi)] by a tensor Gauss-Hermite rule."""
    x, w = hermegauss(q)
    w = w / w.sum()
    total = 1.0
    for m in range(M):
        f = np.ones_like(x)
        for a in alpha_rows:
            f = f * _he(int(a[m]), x)
        total *= float(w @ f)
    return total


def test_term_counts_printed_in_paper():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "pce_term_counts.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert rows
    for r in rows:
        M, p, count = int(r[0]), int(r[1]), int(r[2])
        assert pce.multi_indices(M, p).shape[0] == count


@pytest.mark.parametrize("M,p", [(0, 0), (1, 4), (2, 2), (3, 3), (4, 3), (6, 3)])
def test_term_count_formula(M, p):
    a = pce.multi_indices(M, p)
    assert a.shape[0] == comb(M + p, p)
    # all distinct, all of degree <= p, degree non-decreasing
    assert len({tuple(r) for r in a}) == a.shape[0]
    deg = a.sum(axis=1) if M else np.zeros(1)
    assert (deg <= p).all() and (np.diff(deg) >= 0).all()


def test_ordering_m2_p2():
    a = pce.multi_indices(2, 2)
    assert [tuple(r) for r in a] == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def test_input_basis_is_prefix():
    assert (pce.multi_indices(4, 3)[:15] == pce.multi_indices(4, 2)).all()


def test_orthogonality_by_quadrature():
    a = pce.multi_indices(2, 3)
    fact = pce.alpha_factorial(a)
    for r in range(a.shape[0]):
        for s in range(a.shape[0]):
            e = _quad_expect([a[r], a[s]], 2)
            assert e == pytest.approx(fact[r] if r == s else 0.0, abs=1e-9)


@pytest.mark.parametrize("a,b,c", [(x, y, z) for x in range(6) for y in range(6) for z in range(6)])
def test_triple_1d_matches_quadrature(a, b, c):
    x, w = hermegauss(16)
    w = w / w.sum()
    q = float(w @ (_he(a, x) * _he(b, x) * _he(c, x)))
    assert pce.hermite_triple_1d(a, b, c) == pytest.approx(q, abs=1e-7 * max(1.0, abs(q)))


@pytest.mark.parametrize("M,p_in,p", [(2, 2, 3), (3, 2, 2)])
def test_triple_table_matches_quadrature(M, p_in, p):
    alpha, ijk, val, L_in, P = pce.triple_products(M, p_in, p)
    dense = np.zeros((L_in, P, P))
    dense[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = val
    for i in range(L_in):
        for j in range(P):
            for k in range(P):
                q = _quad_expect([alpha[i], alpha[j], alpha[k]], M)
                assert dense[i, j, k] == pytest.approx(q, abs=1e-8)


def test_triple_counts_and_structure():
    for (M, p_in, p), T in [((2, 2, 2), 36), ((4, 2, 3), 495), ((6, 2, 3), 1722)]:
        alpha, ijk, val, L_in, P = pce.triple_products(M, p_in, p)
        assert len(val) == T
        G = pce.g_matrices(ijk, val, L_in, P)
        assert np.array_equal(G, np.transpose(G, (0, 2, 1)))      # G_i symmetric
        assert np.array_equal(np.diag(G[0]), pce.alpha_factorial(alpha))
        assert np.count_nonzero(G[0] - np.diag(np.diag(G[0]))) == 0


def test_vector_pde_example_l1_n1():
    """The L = N = 1 illustration of the vector-PDE form (Sec. 2.1): for one
    variable, A_kj = sum_i m_ijk c_i gives [[c0, c1], [c1, c0]]."""
    alpha, ijk, val, L_in, P = pce.triple_products(1, 1, 1)
    G = pce.g_matrices(ijk, val, L_in, P)
    c = np.array([2.0, 0.5])
    A = np.einsum("i,ikj->kj", c, G)
    assert np.allclose(A, [[2.0, 0.5], [0.5, 2.0]])


def test_lognormal_coefficients_by_projection():
    """c_bar_alpha = <exp(g0 + g.xi) Psi_alpha> / <Psi_alpha^2>, computed by
    tensor Gauss-Hermite quadrature, including the sign of odd orders."""
    rng = np.random.default_rng(3)
    M = 2
    g = rng.uniform(-0.6, 0.6, size=(M, 5))
    g0 = rng.uniform(-0.3, 0.3, size=5)
    alpha = pce.multi_indices(M, 3)
    cbar = pce.lognormal_coefficients(g0, g, alpha)
    x, w = hermegauss(30)
    w = w / w.sum()
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    for pnt in range(5):
        field = np.exp(g0[pnt] + g[0, pnt] * X1 + g[1, pnt] * X2)
        for r, a in enumerate(alpha):
            psi = _he(int(a[0]), X1) * _he(int(a[1]), X2)
            proj = (W * field * psi).sum() / (factorial(int(a[0])) * factorial(int(a[1])))
            assert cbar[r, pnt] == pytest.approx(proj, rel=1e-10, abs=1e-13)
    # the mean is the log-normal mean exp(g0 + |g|^2/2)
    assert np.allclose(cbar[0], np.exp(g0 + 0.5 * (g ** 2).sum(0)))
