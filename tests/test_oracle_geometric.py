"""Pins of the geometric coarse space: interpolation of linear functions,
the Galerkin coarse operator against the coarse P1 assembly with the fine
coefficient integrated over each coarse element (nested meshes), the coarse
correction as an A-orthogonal projection, and exactness at ratio 1."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import coarse, fem, geometric, system
from paper_2310_14649_amd.inputs import make_problem, structured_mesh


@pytest.mark.parametrize("N,r", [(8, 2), (12, 4), (16, 8), (9, 3)])
def test_prolongation_reproduces_linear_functions(N, r):
    """P1 interpolation is exact for functions linear on every coarse
    triangle, such as the hat of one coarse node: P e_J equals that hat,
    written from its definition, at every fine node."""
    P = geometric.prolongation(N, r)
    fine = structured_mesh(N)
    xf = fine.interior_xy()
    Nc = N // r
    nc = (Nc - 1) ** 2
    for J in (0, nc // 2, nc - 1):
        e = np.zeros(nc)
        e[J] = 1.0
        ci, cj = J % (Nc - 1) + 1, J // (Nc - 1) + 1
        # the coarse hat of node (ci, cj) at the fine nodes, from its
        # definition on the coarse "/" triangles
        X, Y = xf[:, 0] * Nc - ci, xf[:, 1] * Nc - cj
        hat = np.where(X * Y >= 0, 1 - np.maximum(np.abs(X), np.abs(Y)), 1 - np.abs(X) - np.abs(Y))
        hat = np.maximum(hat, 0.0)
        assert np.allclose(P @ e, hat, atol=1e-14)
    # partition of unity: rows sum to one where every coarse corner with a
    # non-zero weight is interior (fine lattice indices r <= i, j <= N - r),
    # and to at most one elsewhere
    s = np.asarray(P.sum(axis=1)).ravel().reshape(N - 1, N - 1)
    k = np.arange(1, N)
    inner = (k >= r) & (k <= N - r)
    assert np.allclose(s[np.ix_(inner, inner)], 1.0, atol=1e-15)
    assert s.max() <= 1.0 + 1e-15 and s.min() >= 0.0


def test_galerkin_equals_coarse_assembly_with_integrated_coefficient():
    """On nested lattices P^T K P is the coarse P1 stiffness with coefficient
    (1/|T|) sum_{t in T} |t| c(t) on each coarse triangle T."""
    N, r = 16, 4
    pr = make_problem("c1", nc=N, M=2, p=2, sub=(1, 1))
    m = pr.mesh
    S = system.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)
    P = geometric.prolongation(N, r)
    Cg = coarse.coarse_blocks(S.K, P)
    cm = structured_mesh(N // r)
    # fine element t = 2 (j N + i) + u lies in coarse element 2 (J Nc + I) + u'
    area, _ = fem.element_geometry(m.xy, m.tri)
    Nc = N // r
    t = np.arange(m.tri.shape[0])
    cell = t // 2
    i, j, u = cell % N, cell // N, t % 2
    I, J = i // r, j // r
    a, b = i % r, j % r
    # lower fine triangles of the diagonal cells (a == b) and of cells below
    # it (a > b) lie in the coarse lower triangle; upper ones likewise
    uc = np.where(a > b, 0, np.where(a < b, 1, u))
    T = 2 * (J * Nc + I) + uc
    carea, _ = fem.element_geometry(cm.xy, cm.tri)
    cc = np.zeros((S.coef.shape[0], cm.tri.shape[0]))
    for q in range(S.coef.shape[0]):
        np.add.at(cc[q], T, area * S.coef[q])
    cc /= carea[None, :]
    Kc = fem.assemble(cm.xy, cm.tri, cm.dof, cm.n, cc)
    for q in range(len(Kc)):
        d = (Cg[q] - Kc[q]).toarray()
        assert np.abs(d).max() <= 1e-13 * np.abs(Kc[q].toarray()).max(), q


def test_geometric_coarse_correction_is_a_projection():
    pr = make_problem("c1", nc=16, M=2, p=2, sub=(2, 2))
    m = pr.mesh
    S = system.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)
    P = geometric.prolongation(16, 4)
    cs = coarse.ExactCoarse(coarse.coarse_blocks(S.K, P), S.G)
    rng = np.random.default_rng(3)
    E = rng.standard_normal((P.shape[1], S.P))
    e = coarse.prolong(P, E)                       # a coarse-space field
    back = coarse.prolong(P, cs(coarse.restrict(P, S.matvec(e))))
    assert np.allclose(back, e, rtol=1e-11, atol=1e-12)


def test_ratio_one_is_the_exact_inverse():
    """r = 1: the coarse space is the whole fine space, the two-grid cycle
    is exact and FGMRES takes one step."""
    from oracle.precond import TwoLevel
    from oracle import ras
    pr = make_problem("c1", nc=8, M=2, p=2, sub=(2, 2))
    m = pr.mesh
    S = system.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)
    P = geometric.prolongation(8, 1)
    assert (P != __import__("scipy").sparse.identity(m.n)).nnz == 0
    subs = ras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    B2 = TwoLevel(S.matvec, lambda R: ras.ras_apply(subs, R, S.alpha_fact), P,
                  coarse.ExactCoarse(coarse.coarse_blocks(S.K, P), S.G), omega=1.0)
    x, info = system.solve(S, B2, 10, 1e-10)
    assert info.converged and info.iterations == 1
