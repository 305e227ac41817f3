"""Pins of the oracle's solver: restricted additive Schwarz, the Nicolaides
coarse space, smoothed-aggregation AMG, the two-grid cycle and FGMRES,
each against a property fixed outside the oracle (exact inverses, the
partition-of-unity identity of Eq. RASsto, library GMRES, brute-force
graph distances)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import amg, coarse, krylov, ras, sg, system
from oracle import precond
from oracle.precond import TwoLevel, smoother_damping, smoother_radius
from paper_2310_14649_amd.inputs import make_problem


def _build(pr):
    m = pr.mesh
    return system.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)


@pytest.fixture(scope="module")
def small():
    pr = make_problem("c0", nc=16, sub=(3, 3), overlap=2)
    return pr, _build(pr)


# ---------------------------------------------------------------- RAS
def test_single_subdomain_no_overlap_is_mean_based_inverse(small):
    pr, S = small
    n = pr.mesh.n
    owner = np.zeros(n, dtype=np.int32)
    subs = ras.ras_setup(S.K[0], owner, 1, S.adj, 0)
    R = np.random.default_rng(0).standard_normal((n, S.P))
    Z = ras.ras_apply(subs, R, S.alpha_fact)
    ref = spla.spsolve(S.K[0].tocsc(), R) / S.alpha_fact[None, :]
    assert np.allclose(Z, ref, rtol=1e-11, atol=1e-13)


def test_partition_of_unity(small):
    """sum_s R_s^T D_s R_s = I (Eq. RASsto)."""
    pr, S = small
    subs = ras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    n = pr.mesh.n
    acc = np.zeros(n)
    for sd in subs:
        acc[sd.nodes[sd.owned]] += 1.0
    assert np.array_equal(acc, np.ones(n))


def _graph_distance_7pt(dx, dy):
    """Distance in the graph of the "/" mesh (steps (+-1,0), (0,+-1),
    +-(1,1)): same-sign offsets use the diagonal."""
    if dx * dy > 0:
        return max(abs(dx), abs(dy))
    return abs(dx) + abs(dy)


def test_overlap_matches_brute_force_distance():
    pr = make_problem("c0", nc=20, sub=(4, 4), overlap=2)
    S = _build(pr)
    m1 = pr.mesh.nc - 1
    ij = np.stack([np.arange(pr.mesh.n) % m1, np.arange(pr.mesh.n) // m1], axis=1)
    for s in (0, 5, 10, 15):
        own = np.nonzero(pr.owner == s)[0]
        got = set(ras.grow_overlap(own, S.adj, 2).tolist())
        want = set()
        for a in range(pr.mesh.n):
            d = min(_graph_distance_7pt(ij[a, 0] - ij[b, 0], ij[a, 1] - ij[b, 1]) for b in own)
            if d <= 2:
                want.add(a)
        assert got == want


def test_ras_linear(small):
    pr, S = small
    subs = ras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal((2, pr.mesh.n, S.P))
    lhs = ras.ras_apply(subs, 2.0 * a - 3.0 * b, S.alpha_fact)
    rhs = 2.0 * ras.ras_apply(subs, a, S.alpha_fact) - 3.0 * ras.ras_apply(subs, b, S.alpha_fact)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- coarse
def test_coarse_operator_is_galerkin(small):
    pr, S = small
    Z = coarse.nicolaides(pr.owner, pr.n_sub)
    C = coarse.coarse_blocks(S.K, Z)
    Ac = coarse.coarse_operator(C, S.G).toarray()
    A = sg.sg_kron(S.K, S.G)
    Zb = sp.kron(Z, sp.identity(S.P))
    assert np.allclose(Ac, (Zb.T @ A @ Zb).toarray(), rtol=1e-13, atol=1e-12)


def test_coarse_correction_is_a_projection(small):
    pr, S = small
    Z = coarse.nicolaides(pr.owner, pr.n_sub)
    cs = coarse.ExactCoarse(coarse.coarse_blocks(S.K, Z), S.G)
    E = np.random.default_rng(2).standard_normal((pr.n_sub, S.P))
    e = coarse.prolong(Z, E)
    back = coarse.prolong(Z, cs(coarse.restrict(Z, S.matvec(e))))
    assert np.allclose(back, e, rtol=1e-11, atol=1e-12)


def test_full_coarse_space_gives_exact_inverse():
    """Every node its own subdomain: Z = I, the exact coarse solve is
    A^{-1}, so the two-grid cycle is exact and FGMRES needs one step."""
    pr = make_problem("c0", nc=8)
    S = _build(pr)
    n = pr.mesh.n
    owner = np.arange(n, dtype=np.int32)
    B2, subs, C, cs = system.two_level(S, owner, n, 0, "exact", omega=1.0)
    x, info = system.solve(S, B2, 10, 1e-10)
    assert info.iterations == 1 and info.converged


# ---------------------------------------------------------------- AMG
@pytest.fixture(scope="module")
def coarse_op():
    pr = make_problem("c1", nc=48, sub=(12, 12), M=2, p=2)
    S = _build(pr)
    Z = coarse.nicolaides(pr.owner, pr.n_sub)
    C = coarse.coarse_blocks(S.K, Z)
    return S, coarse.coarse_operator(C, S.G)


def test_aggregation_covers_every_node_once(coarse_op):
    S, Ac = coarse_op
    agg = amg.aggregate(amg.strength_matrix(Ac, S.P))
    assert agg.min() == 0 and (agg >= 0).all()
    assert set(agg.tolist()) == set(range(agg.max() + 1))
    assert agg.max() + 1 < agg.size


def test_tentative_prolongator_orthonormal(coarse_op):
    S, Ac = coarse_op
    agg = amg.aggregate(amg.strength_matrix(Ac, S.P))
    T = amg.tentative(agg, S.P).toarray()
    assert np.allclose(T.T @ T, np.eye(T.shape[1]), atol=1e-14)


def test_hierarchy_shape_and_single_level_exact(coarse_op):
    S, Ac = coarse_op
    h = amg.setup(Ac, S.P)
    assert 2 <= h.n_levels <= amg.MAX_LEVELS
    assert h.A[-1].shape[0] // S.P <= max(amg.MIN_NODES, h.A[-1].shape[0] // S.P)
    h1 = amg.setup(Ac, S.P, max_levels=1)
    b = np.random.default_rng(3).standard_normal(Ac.shape[0])
    assert np.allclose(amg.vcycle(h1, b), spla.spsolve(Ac.tocsc(), b), rtol=1e-10)


def test_vcycle_symmetric_and_contracting(coarse_op):
    S, Ac = coarse_op
    h = amg.setup(Ac, S.P)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((2, Ac.shape[0]))
    assert np.dot(u, amg.vcycle(h, v)) == pytest.approx(np.dot(amg.vcycle(h, u), v), rel=1e-10)
    # energy-norm contraction of the error operator I - V A
    for _ in range(5):
        e = rng.standard_normal(Ac.shape[0])
        e2 = e - amg.vcycle(h, Ac @ e)
        assert np.dot(e2, Ac @ e2) < np.dot(e, Ac @ e)


# ---------------------------------------------------------------- FGMRES
def test_unpreconditioned_matches_library_gmres(small):
    pr, S = small
    hist_lib = []
    spla.gmres(sg.sg_kron(S.K, S.G), S.B.ravel(), restart=20, rtol=1e-9, maxiter=3,
               callback=lambda r: hist_lib.append(r), callback_type="pr_norm")
    x, info = krylov.fgmres(S.matvec, S.B, None, m=20, rtol=1e-9, max_it=20)
    mine = np.array(info.history[1:21])
    lib = np.array(hist_lib[:20])
    assert np.allclose(mine, lib, rtol=1e-8, atol=1e-14)


def test_solution_matches_direct_solve(small):
    pr, S = small
    B2, *_ = system.two_level(S, pr.owner, pr.n_sub, pr.overlap, "amg")
    x, info = system.solve(S, B2, 30, 1e-12)
    ref = sg.sg_solve_direct(S.K, S.G, S.B)
    assert info.converged
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10


def test_lucky_breakdown():
    """b an eigenvector of A: the Krylov space is one-dimensional."""
    rng = np.random.default_rng(5)
    D = np.diag(rng.uniform(1, 2, 12))
    b = np.zeros((12, 1)); b[3, 0] = 1.0
    x, info = krylov.fgmres(lambda v: D @ v, b, None, m=5, rtol=1e-14)
    assert info.iterations == 1 and info.converged
    assert np.allclose(x[:, 0], b[:, 0] / D[3, 3])


def test_iteration_cap_reports_not_converged(small):
    pr, S = small
    x, info = krylov.fgmres(S.matvec, S.B, None, m=10, rtol=1e-12, max_it=1)
    assert info.iterations == 1 and not info.converged


def test_smoother_not_damped_for_deterministic_problem():
    pr = make_problem("c0", M=0, nc=24, sub=(3, 3))
    S = _build(pr)
    subs = ras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    rho = smoother_radius(S.matvec, lambda R: ras.ras_apply(subs, R, S.alpha_fact), S.B.shape)
    assert 1.0 < rho < 1.8 and smoother_damping(rho) == 1.0


def test_splitmix64_matches_published_sequence():
    """The generator of the power iteration's start: the first outputs of
    SplitMix64 from state 0 are the generator's published reference values;
    output i from state s is output 1 from state s + (i - 1) * gamma."""
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [int(v) for v in precond.splitmix64(4)] == ref
    gamma = 0x9E3779B97F4A7C15
    assert int(precond.splitmix64(1, state=(3 * gamma) % 2 ** 64)[0]) == ref[3]
    u = precond.power_start((5000, 7))
    assert u.min() >= -0.5 and u.max() < 0.5
    assert abs(u.mean()) < 0.01 and abs(u.std() - 12 ** -0.5) < 0.005


def test_power_start_reaches_top_of_spectrum():
    """15 power steps of M_RAS A from the pseudo-random start land within 5 %
    of rho (100 steps); from the smooth all-ones field they fall short by
    more than 10 % on this partition (8 x 8 subdomains of a 64^2 mesh)."""
    pr = make_problem("c1", nc=64, sub=(8, 8))
    S = _build(pr)
    subs = ras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    M = lambda R: ras.ras_apply(subs, R, S.alpha_fact)  # noqa: E731
    rho = smoother_radius(S.matvec, M, S.B.shape, 100)
    r15 = smoother_radius(S.matvec, M, S.B.shape, 15)
    v = np.ones(S.B.shape) / np.sqrt(S.B.size)
    for _ in range(15):
        w = M(S.matvec(v))
        o15 = float(np.linalg.norm(w))
        v = w / o15
    assert 0.95 * rho < r15 <= rho * (1 + 1e-6)
    assert o15 < 0.9 * rho


def test_ras_fixed_point_iteration_converges(small):
    """RAS as the stationary iteration of Eq. RASstofixedpoint on the
    mean-based system (K_0 (x) G_0) U = F converges to the exact solution;
    writing the overlap too (plain additive Schwarz) would not."""
    pr, S = small
    subs = ras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    Amean = lambda U: (S.K[0] @ U) * S.alpha_fact[None, :]  # noqa: E731
    rng = np.random.default_rng(6)
    F = rng.standard_normal((pr.mesh.n, S.P))
    U = np.zeros_like(F)
    for _ in range(80):
        U = U + ras.ras_apply(subs, F - Amean(U), S.alpha_fact)
    ref = spla.spsolve(S.K[0].tocsc(), F) / S.alpha_fact[None, :]
    assert np.linalg.norm(U - ref) / np.linalg.norm(ref) < 1e-8
