"""The conditioning study of the paper's appendix (Tab. ss_cond): the ratio
of the SG operator's condition number to the deterministic operator's grows
with the number of random variables M and with the order p.  The oracle's
figure is pinned by the zero-variance limit, the P = 1 reduction, Cauchy
interlacing with the mean block, and a generalized eigenproblem that does
the basis normalisation another way."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import cond
from oracle import system as osys
from paper_2310_14649_amd.inputs import make_problem


def _system(M, p, sigma=None, nc=6):
    pr = make_problem("c1", nc=nc, M=M, p=p, sigma=sigma, sub=(1, 1))
    m = pr.mesh
    return osys.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)


def test_deterministic_and_zero_variance_limits():
    S = _system(0, 2)
    assert S.P == 1
    assert cond.condition_ratio(S.K, S.G, S.alpha_fact)[2] == pytest.approx(1.0, abs=1e-12)
    S = _system(3, 2, sigma=1e-7)
    assert cond.condition_ratio(S.K, S.G, S.alpha_fact)[2] == pytest.approx(1.0, abs=1e-5)


@pytest.mark.parametrize("M,p", [(1, 2), (3, 2), (2, 3)])
def test_normalisation_and_interlacing(M, p):
    S = _system(M, p)
    A = cond.sg_dense(S.K, S.G, S.alpha_fact)
    P = S.P
    # the mean block of the orthonormal form is the mean-coefficient matrix
    mean_block = A[0::P, 0::P]
    assert np.allclose(mean_block, S.K[0].toarray() / S.alpha_fact[0], rtol=0, atol=1e-13)
    # the same spectrum from the unnormalised operator and the Gram matrix
    # of the basis: A_raw v = lambda (I (x) D) v
    raw = sum(np.kron(Ki.toarray(), S.G[i]) for i, Ki in enumerate(S.K))
    gram = np.kron(np.eye(S.K[0].shape[0]), np.diag(S.alpha_fact.astype(np.float64)))
    w = sla.eigh(raw, gram, eigvals_only=True)
    k_sg, k_det, ratio = cond.condition_ratio(S.K, S.G, S.alpha_fact)
    assert k_sg == pytest.approx(w[-1] / w[0], rel=1e-9)
    # Cauchy interlacing: the spectrum of A encloses that of its mean block
    assert ratio >= 1.0 - 1e-12


def test_ratio_grows_with_variables_and_order():
    rows = []
    for p in (2, 3):
        for M in range(1, 7 if p == 2 else 5):
            S = _system(M, p)
            k_sg, k_det, r = cond.condition_ratio(S.K, S.G, S.alpha_fact)
            rows.append((p, M, S.P, k_sg, k_det, r))
            print(f"p={p} M={M} P={S.P}: kappa_SG {k_sg:.3e} kappa_det {k_det:.3e} "
                  f"ratio {r:.3f}")
    for p in (2, 3):
        r = [row[5] for row in rows if row[0] == p]
        assert all(b > a for a, b in zip(r, r[1:]))
    by = {(row[0], row[1]): row[5] for row in rows}
    assert all(by[(3, M)] > by[(2, M)] for M in range(1, 5))
