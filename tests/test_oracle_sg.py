"""Pins of the oracle's SG operator: symmetry and definiteness, the explicit
Kronecker form, decoupling when the input is deterministic, reduction to the
deterministic FEM solve, and the SG moments against stochastic collocation
and Monte Carlo (the paper's own verification, Sec. 4.1)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import fem, pce, sg, stats, system
from paper_2310_14649_amd.inputs import make_problem, structured_mesh


def _build(pr):
    m = pr.mesh
    return system.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)


@pytest.fixture(scope="module")
def c0():
    pr = make_problem("c0")
    return pr, _build(pr)


def test_operator_symmetric(c0):
    pr, S = c0
    rng = np.random.default_rng(0)
    X = rng.standard_normal((pr.mesh.n, S.P))
    Y = rng.standard_normal((pr.mesh.n, S.P))
    a = np.sum(X * S.matvec(Y))
    b = np.sum(Y * S.matvec(X))
    assert abs(a - b) <= 1e-13 * abs(a)


def test_operator_positive_definite(c0):
    pr, S = c0
    A = sg.sg_kron(S.K, S.G).toarray()
    assert A.shape == (5766, 5766)
    sla.cholesky(A, lower=True)                       # raises if not SPD
    assert np.allclose(A, A.T, rtol=0, atol=1e-12)


def test_matvec_matches_kronecker_form(c0):
    pr, S = c0
    rng = np.random.default_rng(1)
    X = rng.standard_normal((pr.mesh.n, S.P))
    A = sg.sg_kron(S.K, S.G)
    assert np.allclose(S.matvec(X).ravel(), A @ X.ravel(), rtol=1e-13, atol=1e-12)


def test_rhs_only_mean_mode(c0):
    pr, S = c0
    assert np.count_nonzero(S.B[:, 1:]) == 0
    assert np.allclose(S.B[:, 0], S.F)


def test_deterministic_input_decouples():
    pr = make_problem("c0", nc=12)
    m = pr.mesh
    S = _build(pr)
    coef = np.zeros_like(S.coef)
    coef[0] = S.coef[0]
    K = fem.assemble(m.xy, m.tri, m.dof, m.n, coef)
    U = sg.sg_solve_direct(K, S.G, S.B)
    assert np.abs(U[:, 1:]).max() == 0.0
    u0 = spla.spsolve(K[0].tocsc(), S.F)
    assert np.allclose(U[:, 0], u0, rtol=1e-12, atol=1e-15)


def test_p1_reduces_to_deterministic_fem():
    """M = 0: one PCE term, the SG system is the deterministic FEM system
    with c = exp(g0)."""
    m = structured_mesh(10)
    g0 = 0.3 * np.sin(3 * m.centroids()[:, 0])
    S = system.build(m.xy, m.tri, m.dof, m.n, g0, np.zeros((0, m.n_tri)), 0, 0, 0)
    assert S.P == 1 and S.L_in == 1
    U = sg.sg_solve_direct(S.K, S.G, S.B)
    Kd = fem.assemble(m.xy, m.tri, m.dof, m.n, np.exp(g0)[None, :])[0]
    u = spla.spsolve(Kd.tocsc(), fem.load_vector(m.xy, m.tri, m.dof, m.n))
    assert np.allclose(U[:, 0], u, rtol=1e-13)


def test_moments_against_collocation():
    """SG mean/variance of the truncated-input problem converge to the
    stochastic-collocation moments as the output order grows."""
    pr2 = make_problem("c0", nc=8, p=2, sigma=0.3)
    S2 = _build(pr2)
    cm, cv = stats.collocation_moments(S2.K, S2.alpha[:S2.L_in], S2.F, 2, 12)
    errs = {}
    for p in (1, 2, 3):
        pr = make_problem("c0", nc=8, p=p, sigma=0.3)
        S = _build(pr)
        U = sg.sg_solve_direct(S.K, S.G, S.B)
        mean, var = stats.pce_mean_var(U, S.alpha_fact)
        errs[p] = (np.abs(mean - cm).max() / np.abs(cm).max(),
                   np.abs(var - cv).max() / np.abs(cv).max())
    assert errs[3][0] < 1e-4 and errs[3][1] < 2e-2
    assert errs[3][0] < errs[1][0] and errs[3][1] < errs[1][1]


def test_moments_against_monte_carlo():
    pr = make_problem("c0", nc=8, p=3, sigma=0.3)
    S = _build(pr)
    U = sg.sg_solve_direct(S.K, S.G, S.B)
    mean, var = stats.pce_mean_var(U, S.alpha_fact)
    rng = np.random.default_rng(7)
    xi = rng.standard_normal((20000, 2))
    u = stats.sample_solve(S.K[:S.L_in], S.alpha[:S.L_in], S.F, xi)
    mc_mean = u.mean(0)
    se = u.std(0) / np.sqrt(u.shape[0])
    assert (np.abs(mc_mean - mean) <= 4 * se + 1e-4 * np.abs(mean)).all()
    mc_var = u.var(0)
    # standard error of a variance estimate ~ var * sqrt(2/(N-1)) (near-Gaussian)
    assert (np.abs(mc_var - var) <= 4 * mc_var * np.sqrt(2.0 / 19999) + 2e-2 * var).all()
