"""Pins of four oracle functions, written as checks that take the function
under test, so that the same check runs on the oracle itself
(test_oracle_pins.py) and on copies of it with a planted mistake
(test_oracle_mutants.py).  Each check returns True when the function passes.

None of these checks re-evaluates the oracle's own formula:

* aggregate(): a hand-worked strength graph whose three greedy passes
  (Vanek, Mandel and Brezina) were traced by hand, with a tie, a node whose
  strongest neighbour only joins an aggregate in the second pass, and two
  edges on either side of the strength threshold theta sqrt(|s_ss s_tt|).
* MeanExactCoarse: a dense LU solve of the explicit Kronecker product
  C_0 (x) diag(alpha!) (row index s*P + k), and the special case of a
  deterministic coefficient, where the mean-based coarse operator is the
  whole coarse operator.
* NLProblem.mean_stiffness(): the element coefficient E[c kappa(u_T)] in
  closed form through the Hermite triple products, E[c] = c_0,
  E[c u] = sum_i c_i u_i i!, E[c u^2] = sum m_ijk c_i u_j u_k, instead of the
  oracle's Gauss-Hermite quadrature.
* adam_step(): trajectories worked out by hand in exact rationals (Kingma
  and Ba's bias-corrected moments), including a gradient that changes sign,
  where the state carried between steps matters.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import scipy.linalg as sla

THETA = 0.08


# ------------------------------------------------------------- aggregation
def hand_graph():
    """Six block-nodes, strength entries S (symmetric).

    Node names a, d, b, c, m, n are numbered 0..5 in that order.  Strong
    couplings (|S_st| >= 0.08 sqrt(|S_ss S_tt|)):
      a-b: |S| = 1,   diag 8 and 2, threshold 0.32 (strong; 1 < 0.08*8*2 =
           1.28, so a test without the square root calls it weak);
      d-c: 1; b-m: 1; c-m: 1 (equal: the tie of m); m-n: 1.5; c-n: 0.5.
    One weak coupling: a-d, |S| = 0.15, diag 8 and 0.5, threshold 0.16 (a
    test against 0.08 min(diag) = 0.04 calls it strong).

    Pass 1 in node order: a seeds {a, b} (its only strong neighbour is b);
    d seeds {d, c}; b, c are taken; m has taken neighbours (b, c), skipped;
    n has a taken neighbour (c), skipped.
    Pass 2 against the pass-1 snapshot: m's candidates are b (aggregate 0)
    and c (aggregate 1) with equal strength; the lower node index, b, wins:
    m -> 0.  n's strongest neighbour m had no pass-1 aggregate, so its
    candidate is c: n -> 1 (joining m's new aggregate would give 0).
    Pass 3 has nothing left.  Expected aggregates: [0, 1, 0, 1, 0, 1].
    """
    a, d, b, c, m, n = range(6)
    S = np.zeros((6, 6))
    S[a, a], S[d, d], S[b, b], S[c, c], S[m, m], S[n, n] = 8.0, 0.5, 2.0, 2.0, 2.0, 2.0
    for s, t, v in [(a, b, -1.0), (d, c, -1.0), (b, m, -1.0), (c, m, -1.0),
                    (m, n, -1.5), (c, n, -0.5), (a, d, -0.15)]:
        S[s, t] = S[t, s] = v
    return S, np.array([0, 1, 0, 1, 0, 1])


def isolated_graph():
    """A chain 0-1-2-3 of strong couplings and node 4 coupled to 3 below the
    threshold (0.1 < 0.16).  Pass 1: 0 seeds {0, 1}; 2 has the taken
    neighbour 1 and is skipped; 3's neighbourhood {2} is free, so 3 seeds
    {3, 2}; 4 has no strong neighbour and seeds the singleton {4}.
    Expected [0, 0, 1, 1, 2]."""
    S = 2.0 * np.eye(5)
    for s, t in [(0, 1), (1, 2), (2, 3)]:
        S[s, t] = S[t, s] = -1.0
    S[3, 4] = S[4, 3] = -0.1      # 0.1 < 0.16: weak
    return S, np.array([0, 0, 1, 1, 2])


def pin_aggregate(aggregate) -> bool:
    try:
        for S, expect in (hand_graph(), isolated_graph()):
            got = np.asarray(aggregate(S, THETA))
            if got.shape != expect.shape or not np.array_equal(got, expect):
                return False
        return True
    except Exception:
        return False


# ------------------------------------------------------- mean-based coarse
def pin_mean_exact_coarse(cls, C, G, alpha_fact, C_det) -> bool:
    """C: coarse blocks of a stochastic problem; C_det: of a deterministic
    coefficient (only C_0 non-zero).  G: [L_in, P, P] triple matrices."""
    try:
        P = alpha_fact.size
        rng = np.random.default_rng(11)
        rc = rng.standard_normal((C[0].shape[0], P))
        got = cls(C, alpha_fact)(rc)
        A0 = np.kron(C[0].toarray(), np.diag(alpha_fact))
        ref = sla.lu_solve(sla.lu_factor(A0), rc.ravel()).reshape(rc.shape)
        if not np.allclose(got, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max()):
            return False
        # deterministic coefficient: A_c = sum_i C_i (x) G_i = C_0 (x) G_0
        Ad = sum(np.kron(Ci.toarray(), G[i]) for i, Ci in enumerate(C_det))
        got_d = cls(C_det, alpha_fact)(rc)
        return bool(np.allclose(Ad @ got_d.ravel(), rc.ravel(), rtol=1e-10,
                                atol=1e-12 * np.abs(rc).max()))
    except Exception:
        return False


# ------------------------------------------------------ Newton mean stiffness
def mean_coefficient_closed_form(pr, U, ijk, val):
    """E[c_T kappa(u_T)] per element by Hermite triple products."""
    from math import factorial
    tri = pr.tri
    d = pr.dof[tri]
    Ue = np.where((d >= 0)[..., None], U[np.maximum(d, 0)], 0.0)     # [E, 3, P]
    ub = Ue.mean(axis=1)                                              # centroid, [E, P]
    c = pr.coef.T                                                     # [E, L]
    L = c.shape[1]
    fact = np.array([np.prod([factorial(int(v)) for v in a]) for a in pr.alpha[:L]])
    e_c = c[:, 0]
    e_cu = (c * ub[:, :L] * fact[None, :]).sum(axis=1)
    e_cuu = np.zeros(tri.shape[0])
    for (i, j, k), v in zip(ijk, val):
        e_cuu += v * c[:, i] * ub[:, j] * ub[:, k]
    return e_c + pr.a1 * e_cu + pr.a2 * e_cuu


def pin_mean_stiffness(mean_stiffness, pr, ijk, val, assemble) -> bool:
    """mean_stiffness(pr, U) -> sparse [n, n]."""
    try:
        rng = np.random.default_rng(5)
        cases = [np.zeros((pr.n, pr.P)), 0.4 * rng.standard_normal((pr.n, pr.P))]
        U1 = np.zeros((pr.n, pr.P))
        U1[:, 0] = rng.standard_normal(pr.n)          # deterministic u: kappa(u_T) c_0
        cases.append(U1)
        for U in cases:
            got = mean_stiffness(pr, U).toarray()
            cm = mean_coefficient_closed_form(pr, U, ijk, val)
            ref = assemble(pr.xy, pr.tri, pr.dof, pr.n, cm[None, :])[0].toarray()
            if not np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max()):
                return False
        return True
    except Exception:
        return False


# ------------------------------------------------------------------- Adam
def adam_hand_trajectory():
    """beta1 = 1/2, beta2 = 3/4, lr = 1, eps = 0, scalar parameter p_0 = 0,
    gradients 2, -2, 2.
      t=1: m = 1, v = 1;       m^ = 1/(1/2) = 2,     v^ = 1/(1/4) = 4:   p = -1
      t=2: m = -1/2, v = 7/4;  m^ = -(1/2)/(3/4),    v^ = (7/4)/(7/16) = 4:
           step -1/3, p = -2/3
      t=3: m = 3/4, v = 37/16; m^ = (3/4)/(7/8) = 6/7, v^ = (37/16)/(37/64) = 4:
           step 3/7, p = -23/21
    """
    return [Fraction(-1), Fraction(-2, 3), Fraction(-23, 21)]


def pin_adam(adam_step) -> bool:
    try:
        # sign-changing gradients: the carried moments and t matter
        params = [(np.zeros((3, 3, 1, 1)), np.zeros(1))]
        state = {}
        for g, want in zip((2.0, -2.0, 2.0), adam_hand_trajectory()):
            grads = [(np.full((3, 3, 1, 1), g), np.array([-g]))]
            params = adam_step(params, grads, state, 1.0, 0.5, 0.75, 0.0)
            if not np.allclose(params[0][0], float(want), rtol=1e-14, atol=0):
                return False
            if not np.allclose(params[0][1], -float(want), rtol=1e-14, atol=0):
                return False
        # a constant gradient: with bias correction every step is lr * sign(g)
        params = [(np.full((3, 3, 1, 2), 0.25), np.array([1.0, -1.0]))]
        state = {}
        for t in range(1, 6):
            grads = [(np.full((3, 3, 1, 2), -0.3), np.array([5.0, -1e-3]))]
            params = adam_step(params, grads, state, 0.01, 0.9, 0.999, 0.0)
            if not (np.allclose(params[0][0], 0.25 + 0.01 * t, rtol=1e-13)
                    and np.allclose(params[0][1], [1.0 - 0.01 * t, -1.0 + 0.01 * t],
                                    rtol=1e-13)):
                return False
        return True
    except Exception:
        return False


def coarse_fixture():
    """Coarse blocks of a small stochastic problem and of the same mesh with
    a deterministic coefficient (g = 0), for pin_mean_exact_coarse."""
    from oracle import coarse, system
    from paper_2310_14649_amd.inputs import make_problem
    pr = make_problem("c0", nc=12, sub=(3, 3), overlap=1)
    m = pr.mesh
    S = system.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)
    Z = coarse.nicolaides(pr.owner, pr.n_sub)
    C = coarse.coarse_blocks(S.K, Z)
    Sd = system.build(m.xy, m.tri, m.dof, m.n, pr.g0, 0.0 * pr.g, pr.M, pr.p_in, pr.p)
    Cd = coarse.coarse_blocks(Sd.K, Z)
    return C, np.asarray(S.G), S.alpha_fact, Cd


def newton_fixture(a1=0.3, a2=0.5):
    from oracle import newton as onl
    from oracle import pce
    from paper_2310_14649_amd.inputs import make_problem
    pr = make_problem("c0", nc=6, M=2, p=2, sigma=0.4, sub=(1, 1))
    m = pr.mesh
    nl = onl.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p, a2=a2, a1=a1)
    _, ijk, val, _, _ = pce.triple_products(pr.M, pr.p_in, pr.p)
    return nl, ijk, val


# --------------------------------------------------------- geometric coarse
def pin_prolongation(prolongation) -> bool:
    """P e_J is the coarse hat of node J at the fine nodes: 1 - max(|X|,|Y|)
    where X Y >= 0 (the "/" diagonal is an edge there), else 1 - |X| - |Y|,
    clipped at 0, X, Y the offsets from the node in coarse cells."""
    from paper_2310_14649_amd.inputs import structured_mesh
    try:
        for N, r in ((8, 2), (12, 4), (9, 3)):
            P = prolongation(N, r)
            xf = structured_mesh(N).interior_xy()
            Nc = N // r
            nc = (Nc - 1) ** 2
            for J in range(nc):
                e = np.zeros(nc)
                e[J] = 1.0
                ci, cj = J % (Nc - 1) + 1, J // (Nc - 1) + 1
                X, Y = xf[:, 0] * Nc - ci, xf[:, 1] * Nc - cj
                hat = np.where(X * Y >= 0, 1 - np.maximum(np.abs(X), np.abs(Y)),
                               1 - np.abs(X) - np.abs(Y))
                if not np.allclose(P @ e, np.maximum(hat, 0.0), atol=1e-14):
                    return False
        return True
    except Exception:
        return False
