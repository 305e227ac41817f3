"""Pins of the oracle's nonlinear SG residual, Jacobian and Newton loop:
finite-difference Jacobian, reduction to the linear SG operator at U = 0,
the Kirchhoff closed form of the deterministic strip problem (the paper's
analogous analytic benchmark is the (1+u)^m problem of its appendix), and
the SG mean against stochastic collocation of the nonlinear problem."""
import numpy as np
import pytest

from oracle import newton as onl
from oracle import sg as osg
from oracle import system as osys
from paper_2310_14649_amd.inputs import make_problem, structured_mesh


def _nl(nc=5, M=2, p=2, sigma=0.4, a2=0.5, a1=0.0):
    pr = make_problem("c0", nc=nc, M=M, p=p, sigma=sigma, sub=(1, 1))
    m = pr.mesh
    return pr, onl.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p, a2=a2,
                         a1=a1)


def test_quadrature_rule_exact_to_degree_15():
    pts, w = onl.gauss_hermite_tensor(2, 8)
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    # E[x^14] = 13!! = 135135, E[x^4 y^10] = 3 * 945
    assert (w * pts[:, 0] ** 14).sum() == pytest.approx(135135.0, rel=1e-10)
    assert (w * pts[:, 0] ** 4 * pts[:, 1] ** 10).sum() == pytest.approx(3 * 945.0, rel=1e-10)


# kappa(u) = 1 + a1 u + a2 u^2: the Newton configuration, the paper's 1 + u, a mix
KAPPAS = [(0.0, 0.5), (1.0, 0.0), (0.7, 0.3)]


@pytest.mark.parametrize("a1,a2", KAPPAS)
def test_jacobian_matches_finite_differences(a1, a2):
    pr, nl = _nl(a1=a1, a2=a2)
    rng = np.random.default_rng(0)
    U = 0.3 * rng.standard_normal((nl.n, nl.P))
    V = rng.standard_normal((nl.n, nl.P))
    J = nl.jacobian(U)
    eps = 1e-5
    fd = -(nl.residual(U + eps * V) - nl.residual(U - eps * V)) / (2 * eps)
    jv = (J @ V.ravel()).reshape(V.shape)
    assert np.abs(jv - fd).max() / np.abs(fd).max() < 1e-7


def test_jacobian_at_zero_is_linear_sg_operator():
    pr, nl = _nl(nc=6, M=2, p=3)
    m = pr.mesh
    S = osys.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)
    J0 = nl.jacobian(np.zeros((nl.n, nl.P))).toarray()
    A = osg.sg_kron(S.K, S.G).toarray()
    assert np.abs(J0 - A).max() / np.abs(A).max() < 1e-12
    # and with kappa = 1 the residual is the linear one
    _, lin = _nl(nc=6, M=2, p=3, a2=0.0)
    U = np.random.default_rng(1).standard_normal((nl.n, nl.P))
    assert np.allclose(lin.residual(U), S.B - S.matvec(U), rtol=1e-12, atol=1e-13)


def _kirchhoff_exact(x):
    """u + u^3/6 = 7x/6, the real root."""
    out = np.empty_like(x)
    for i, xv in enumerate(x):
        r = np.roots([1.0 / 6.0, 0.0, 1.0, -7.0 * xv / 6.0])
        out[i] = r[np.abs(r.imag) < 1e-12].real[0]
    return out


def test_deterministic_strip_kirchhoff_closed_form():
    """-(kappa(u) u')' = 0, u(0)=0, u(1)=1, no flux at y=0,1: with
    kappa = 1 + u^2/2 the Kirchhoff transform gives u + u^3/6 = 7x/6.
    Newton converges quadratically and the P1 error is O(h^2)."""
    errs = []
    for nc in (8, 16, 32):
        m = structured_mesh(nc)
        x = m.xy[:, 0]
        dof = np.full(m.n_vert, -1, dtype=np.int32)
        free = (x > 0) & (x < 1)
        dof[free] = np.arange(free.sum())
        uD = np.where(np.isclose(x, 1.0), 1.0, 0.0)
        nl = onl.NLProblem(xy=m.xy, tri=m.tri, dof=dof, n=int(free.sum()),
                           coef=np.ones((1, m.n_tri)), alpha=np.zeros((1, 0), dtype=np.int64),
                           L=1, P=1, a2=0.5, uD=uD, fvals=np.zeros(m.n_vert))
        U, info = onl.newton(nl, tol=1e-13)
        assert info.converged
        r = np.array(info.residuals)
        if len(r) >= 4:
            assert r[-1] < 1e-6 * r[-3]          # superlinear tail
        u = np.zeros(m.n_vert)
        u[free] = U[dof[free], 0]
        u += uD
        errs.append(np.abs(u - _kirchhoff_exact(x)).max())
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3, errs


def test_newton_quadratic_convergence_sg():
    pr, nl = _nl(nc=6, M=2, p=2, sigma=0.5)
    U, info = onl.newton(nl, tol=1e-13)
    assert info.converged and info.steps <= 8
    r = np.array(info.residuals)
    # the last steps square the residual (up to a constant)
    assert r[-2] < 1e-4 and r[-1] < 10 * r[-2] ** 2 + 1e-13


def test_sg_mean_against_collocation_of_nonlinear_problem():
    pr, nl = _nl(nc=5, M=2, p=3, sigma=0.3)
    U, info = onl.newton(nl, tol=1e-13)
    mean_sg = U[:, 0]
    # collocation: deterministic nonlinear solves at Gauss-Hermite nodes, with
    # the same truncated input c = sum_i c_bar_i Psi_i(xi)
    from numpy.polynomial.hermite_e import hermegauss
    from oracle import pce
    x, w = hermegauss(10)
    w = w / w.sum()
    mean_col = np.zeros(nl.n)
    alpha_in = nl.alpha[:nl.L]
    for i, xi1 in enumerate(x):
        for j, xi2 in enumerate(x):
            psi = pce.psi_eval(alpha_in, np.array([[xi1, xi2]]))[0]
            c = psi @ nl.coef
            det = onl.NLProblem(xy=nl.xy, tri=nl.tri, dof=nl.dof, n=nl.n, coef=c[None, :],
                                alpha=np.zeros((1, 0), dtype=np.int64), L=1, P=1, a2=nl.a2)
            Ud, _ = onl.newton(det, tol=1e-13)
            mean_col += w[i] * w[j] * Ud[:, 0]
    assert np.abs(mean_sg - mean_col).max() / np.abs(mean_col).max() < 2e-4


@pytest.mark.parametrize("a1,a2", KAPPAS)
def test_secant_operator_reproduces_residual(a1, a2):
    """A(U) = K1(U) U: the secant operator (assembled like the Jacobian's
    first term) and the residual (assembled from the flux) agree."""
    pr, nl = _nl(nc=6, M=2, p=2, a1=a1, a2=a2)
    U = 0.3 * np.random.default_rng(4).standard_normal((nl.n, nl.P))
    K1 = nl.secant(U)
    F = np.zeros((nl.n, nl.P))
    F[:, 0] = nl.F
    R = F - (K1 @ U.ravel()).reshape(U.shape)
    assert np.abs(R - nl.residual(U)).max() / np.abs(nl.residual(U)).max() < 1e-12


def _strip(nc, a1, a2):
    m = structured_mesh(nc)
    x = m.xy[:, 0]
    dof = np.full(m.n_vert, -1, dtype=np.int32)
    free = (x > 0) & (x < 1)
    dof[free] = np.arange(free.sum())
    uD = np.where(np.isclose(x, 1.0), 1.0, 0.0)
    nl = onl.NLProblem(xy=m.xy, tri=m.tri, dof=dof, n=int(free.sum()),
                       coef=np.ones((1, m.n_tri)), alpha=np.zeros((1, 0), dtype=np.int64),
                       L=1, P=1, a2=a2, a1=a1, uD=uD, fvals=np.zeros(m.n_vert))
    return m, x, dof, free, uD, nl


def test_paper_model_strip_kirchhoff_picard_and_newton():
    """The paper's kappa = 1 + u on the strip -(kappa(u) u')' = 0, u(0)=0,
    u(1)=1: the Kirchhoff transform gives u + u^2/2 = 3x/2, i.e.
    u = sqrt(1 + 3x) - 1.  Picard and Newton reach the same discrete solution,
    Picard with a contracting (linear) update sequence, and the P1 error is
    O(h^2)."""
    errs = []
    for nc in (8, 16, 32):
        m, x, dof, free, uD, nl = _strip(nc, 1.0, 0.0)
        Un, info_n = onl.newton(nl, tol=1e-13)
        Up, info_p = onl.picard(nl, du_tol=1e-12, max_steps=200)
        assert info_n.converged and info_p.converged
        assert np.abs(Up - Un).max() < 1e-10
        du = np.array(info_p.du)
        assert info_p.steps > info_n.steps
        assert np.all(du[2:] / du[1:-1] < 0.9)                # linear contraction
        u = np.zeros(m.n_vert)
        u[free] = Un[dof[free], 0]
        u += uD
        errs.append(np.abs(u - (np.sqrt(1.0 + 3.0 * x) - 1.0)).max())
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3, errs


def test_picard_and_newton_same_sg_solution():
    pr, nl = _nl(nc=6, M=2, p=2, sigma=0.4, a1=1.0, a2=0.0)
    Un, info_n = onl.newton(nl, tol=1e-13)
    Up, info_p = onl.picard(nl, du_tol=1e-12)
    assert info_n.converged and info_p.converged
    assert np.abs(Up - Un).max() / np.abs(Un).max() < 1e-10
    assert info_p.residuals[-1] < 1e-10
