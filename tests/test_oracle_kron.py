"""Kronecker (Ullmann) local solves in the oracle: the factor Gt is the
Frobenius-nearest K_0 (x) G to the SG operator (checked by brute force on
the dense Kronecker matrices), it reproduces the operator exactly when every
K_i is a multiple of K_0, and the RAS built on it inverts such an operator
on a single subdomain."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ras
from oracle import system as osys
from paper_2310_14649_amd.inputs import make_problem


def _small(M=2, p=2, nc=6):
    pr = make_problem("c1", nc=nc, M=M, p=p, sub=(2, 2))
    m = pr.mesh
    return pr, osys.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)


def _dense_op(K, G):
    return sum(np.kron(Ki.toarray(), G[i]) for i, Ki in enumerate(K))


def test_factor_is_frobenius_nearest():
    pr, S = _small()
    A = _dense_op(S.K, S.G)
    K0 = S.K[0].toarray()
    Gt = ras.kron_factor(S.K, S.G)
    best = np.linalg.norm(A - np.kron(K0, Gt))
    rng = np.random.default_rng(3)
    for _ in range(6):
        E = rng.standard_normal(Gt.shape)
        for eps in (1e-3, 1e-1):
            assert np.linalg.norm(A - np.kron(K0, Gt + eps * E)) > best
    # and it is symmetric, with the mean block G_0 weighted by 1
    assert np.allclose(Gt, Gt.T, atol=1e-14)


def test_factor_exact_for_proportional_stiffness_and_single_subdomain_inverse():
    pr, S = _small(M=3, p=2)
    K0 = S.K[0]
    c = np.concatenate([[1.0], np.random.default_rng(4).uniform(-0.2, 0.2, len(S.K) - 1)])
    K = [sp.csr_matrix(ci * K0) for ci in c]
    Gt = ras.kron_factor(K, S.G)
    assert np.allclose(Gt, sum(ci * S.G[i] for i, ci in enumerate(c)), rtol=1e-13, atol=1e-13)
    n = K0.shape[0]
    subs = ras.ras_setup(K0, np.zeros(n, dtype=np.int32), 1, S.adj, 0)
    X = np.random.default_rng(5).standard_normal((n, S.P))
    AX = sum(K[i] @ (X @ S.G[i].T) for i in range(len(K)))
    Y = ras.ras_apply_kron(subs, AX, Gt)
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) < 1e-12
    # with G_t replaced by G_0 = diag(alpha!) it is the mean-based RAS
    Y0 = ras.ras_apply_kron(subs, AX, np.diag(S.alpha_fact.astype(np.float64)))
    assert np.allclose(Y0, ras.ras_apply(subs, AX, S.alpha_fact), rtol=1e-13, atol=1e-13)
