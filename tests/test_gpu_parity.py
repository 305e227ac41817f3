"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by
element on the same seeded inputs.

Tolerances (FP64 paths): assembly and the SG matvec are sums of a handful
of products, so 1e-13 relative to the largest entry covers any summation
order; RAS, the V-cycle and the two-grid cycle are fixed linear maps whose
factorisations differ from the oracle's only in rounding (condition numbers
< 1e4 at these sizes), hence 1e-10; converged FGMRES solutions are compared
to the direct solution at 1e-8 (the method's FP64 target).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import amg as oamg  # noqa: E402
from oracle import coarse as ocoarse  # noqa: E402
from oracle import pce as opce  # noqa: E402
from oracle import ras as oras  # noqa: E402
from oracle import sg as osg  # noqa: E402
from oracle import system as osys  # noqa: E402
from oracle.precond import smoother_radius  # noqa: E402
from paper_2310_14649_amd import binding as B  # noqa: E402
from paper_2310_14649_amd.inputs import make_problem  # noqa: E402
from paper_2310_14649_amd.solver import GpuSG  # noqa: E402


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle(pr):
    m = pr.mesh
    return osys.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _to_host(t, shape):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().reshape(shape)


def _to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


CASES = {
    "c0": dict(name="c0"),
    "c1_64": dict(name="c1", nc=64, sub=(8, 8)),
    "c3_40": dict(name="c3", nc=40, sub=(4, 4)),       # jittered mesh, M=6, P=84
    "p1_det": dict(name="c0", M=0, nc=20, sub=(3, 2)),   # P = 1: deterministic FEM
    "c4_ragged": dict(name="c4", nc=23, sub=(3, 5)),     # tails in every tile
    "j4": dict(name="jit", nc=26, M=4, p=3, sub=(3, 3)),  # jittered, 7 entries per row
    "j2": dict(name="jit", nc=30, M=2, p=2, sub=(2, 3)),
    "g6": dict(name="jit", nc=44, M=6, p=2, sub=(1, 1), graph=(4, 3)),  # graph partition, M=6
    # two subdomains of ~1100 owned nodes: the fused dense RAS takes two
    # work-groups per subdomain (its LDS holds 16 x 1152 FP64 entries)
    "big_sub": dict(name="c0", nc=48, sub=(1, 2)),
    # unknowns renumbered at random: no block of rows has neighbours in a few
    # runs of consecutive rows, so the operator takes the lane-pair kernel
    "perm": dict(name="c1", nc=40, sub=(4, 4), perm=5),
    # shapes of the stochastic-dimension sweep (M = 2..6, p = 1..4)
    "s21": dict(name="c1", nc=20, M=2, p=1, sub=(2, 2)),      # P = 3, L_in = 3
    "s33": dict(name="c1", nc=18, M=3, p=3, sub=(2, 2)),      # P = 20, L_in = 10
    "s52": dict(name="c1", nc=18, M=5, p=2, sub=(2, 2)),      # P = 21, L_in = 21
    "s24": dict(name="c1", nc=20, M=2, p=4, sub=(2, 2)),      # P = 15, L_in = 6
    "s44": dict(name="c1", nc=12, M=4, p=4, sub=(2, 2)),      # P = 70: wide kernel
    "s62": dict(name="c1", nc=16, M=6, p=2, sub=(2, 2)),      # P = 28, L_in = 28
}

# matvec kernel family each case's operator is expected to select
MV_KIND = {"c0": "staged", "c1_64": "staged", "c3_40": "grouped", "p1_det": "generic",
           "c4_ragged": "staged", "j4": "pair", "j2": "staged", "perm": "pair",
           "s21": "generic", "s33": "generic", "s52": "generic", "s24": "generic",
           "s44": "wide", "s62": "generic"}
SWEEP = ["s21", "s33", "s52", "s24", "s44", "s62"]


def _problem(key):
    kw = dict(CASES[key])
    name = kw.pop("name")
    graph = kw.pop("graph", None)
    perm = kw.pop("perm", None)
    if name == "jit":
        kw["seed"] = 3
    pr = make_problem(name, **kw)
    if perm is not None:
        new = np.random.default_rng(perm).permutation(pr.mesh.n).astype(np.int32)
        inner = pr.mesh.dof >= 0
        pr.mesh.dof[inner] = new[pr.mesh.dof[inner]]
        owner = np.empty_like(pr.owner)
        owner[new] = pr.owner
        pr.owner = owner
    if graph is not None:
        # irregular subdomains: multi-source BFS from jittered lattice centres
        from paper_2310_14649_amd.inputs import graph_partition
        gx, gy = graph
        pr.owner, _ = graph_partition(pr.mesh, gx, gy, 0, 1, 10 ** 9)
        pr.n_sub = gx * gy
    return pr


@pytest.fixture(scope="module")
def built():
    _cuda()
    cache = {}

    def get(key, prec="fp64", coarse="amg"):
        k = (key, prec, coarse)
        if k not in cache:
            pr = _problem(key)
            print(f"[gpu] building {k}: n={pr.mesh.n} M={pr.M} p={pr.p}", flush=True)
            cache[k] = (pr, _oracle(pr), GpuSG(pr, prec=prec, coarse=coarse))
        return cache[k]

    yield get
    for _, _, g in cache.values():
        g.close()


# ------------------------------------------------------------------ a1
@pytest.mark.parametrize("M,p_in,p", [(0, 0, 0), (1, 1, 4), (2, 2, 2), (4, 2, 3), (6, 2, 3), (3, 1, 2)])
def test_triples_bit_exact(M, p_in, p):
    _cuda()
    h = B.sg_build_triples(M, p_in, p)
    try:
        alpha, ijk, val = B.sg_basis_export(h, M)
        oa, oijk, oval, L, P = opce.triple_products(M, p_in, p)
        assert B.sg_basis_info(h)[:2] == (P, L)
        if M:
            assert np.array_equal(alpha, oa)
        got = {tuple(r): v for r, v in zip(ijk.tolist(), val.tolist())}
        want = {tuple(r): v for r, v in zip(oijk.tolist(), oval.tolist())}
        assert got == want
    finally:
        B.sg_destroy_basis(h)


def test_triples_rejects_bad_orders():
    _cuda()
    with pytest.raises(B.SgError):
        B.sg_build_triples(2, 3, 2)


# ------------------------------------------------------------------ a2
@pytest.mark.parametrize("key", ["c0", "c3_40", "c4_ragged", "p1_det", "j4"])
def test_assembly_matches_oracle(built, key):
    pr, S, g = built(key)
    rowptr, col, vals = B.sg_op_export(g.op)
    n = pr.mesh.n
    for i in range(S.L_in):
        Kd = S.K[i].toarray()
        mine = np.zeros((n, n))
        rows = np.repeat(np.arange(n), np.diff(rowptr))
        mine[rows, col] = vals[:, i]
        assert _rel(mine, Kd) < 1e-13, i
    # entries left out of the pattern are exact zeros of the oracle
    K0 = S.K[0].tocoo()
    kept = set(zip(rows.tolist(), col.tolist()))
    for r, c, v in zip(K0.row, K0.col, K0.data):
        if (r, c) not in kept:
            assert v == 0.0
    B_rhs = _to_host(g.b, (n, S.P))
    assert _rel(B_rhs, S.B) < 1e-14


# ------------------------------------------------------------------ a3
@pytest.mark.parametrize("key", ["c0", "c1_64", "c3_40", "c4_ragged", "p1_det", "j4", "j2", "perm",
                                 *SWEEP])
def test_matvec_matches_oracle(built, key):
    pr, S, g = built(key)
    assert B.sg_matvec_kernel(g.op) == MV_KIND[key]
    rng = np.random.default_rng(11)
    X = rng.standard_normal((pr.mesh.n, S.P))
    Y = g.new_vec()
    B.sg_matvec(g.op, _to_dev(X), Y)
    assert _rel(_to_host(Y, X.shape), S.matvec(X)) < 1e-13


# matrix-free apply: lattice meshes whose basis has the staged kernel
MF_KEYS = ["c0", "c1_64", "c4_ragged", "j2"]


@pytest.mark.parametrize("key", MF_KEYS)
def test_matrix_free_matvec_matches_oracle_and_stored(built, key):
    """K values formed per row from the element fields (c0, g_m) and local
    stiffness: against the oracle's stiffness matrices at 1e-13, against the
    stored-value apply at 1e-14, for every tile shape of the staged kernel."""
    pr, S, g = built(key)
    rng = np.random.default_rng(31)
    X = rng.standard_normal((pr.mesh.n, S.P))
    ref = S.matvec(X)
    Ys = g.new_vec()
    B.sg_matvec(g.op, _to_dev(X), Ys)
    stored = _to_host(Ys, X.shape)
    tiles0 = B.sg_matvec_tiles(g.op)
    try:
        B.sg_matvec_matrix_free(g.op, True)
        assert B.sg_matvec_kernel(g.op) == "matrix_free"
        for tiles in (1, 2, 4):
            try:
                B.sg_matvec_select(g.op, tiles)
            except B.SgError:
                continue
            Y = g.new_vec()
            B.sg_matvec(g.op, _to_dev(X), Y)
            Yh = _to_host(Y, X.shape)
            assert _rel(Yh, ref) < 1e-13, tiles
            assert _rel(Yh, stored) < 1e-14, tiles
    finally:
        B.sg_matvec_matrix_free(g.op, False)
        B.sg_matvec_select(g.op, tiles0)
    assert B.sg_matvec_kernel(g.op) == MV_KIND[key]


@pytest.mark.parametrize("key", ["c3_40", "perm", "p1_det"])
def test_matrix_free_unsupported(built, key):
    """No staged kernel (P = 84, P = 1) or not the lattice numbering."""
    pr, S, g = built(key)
    with pytest.raises(B.SgError) as e:
        B.sg_matvec_matrix_free(g.op, True)
    assert e.value.code == -4
    assert B.sg_matvec_kernel(g.op) == MV_KIND[key]


def test_matrix_free_solve_matches_direct(built):
    """FGMRES (graph-captured steps) with the matrix-free operator."""
    pr, S, g = built("c4_ragged")
    ref = osg.sg_solve_direct(S.K, S.G, S.B)
    try:
        B.sg_matvec_matrix_free(g.op, True)
        x, info = g.solve(50, 1e-12, use_graph=True)
        assert info["converged"]
        assert np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref) < 1e-8
    finally:
        B.sg_matvec_matrix_free(g.op, False)
        B.sg_graph_cache_clear()


def test_matvec_tile_shapes_autotune_and_select(built):
    """Every work-group shape of the staged kernel gives the oracle's product;
    the autotuner keeps the fastest shape; shapes are rejected where they do
    not apply."""
    pr, S, g = built("c1_64")
    X = np.random.default_rng(12).standard_normal((pr.mesh.n, S.P))
    ref = S.matvec(X)
    try:
        for tiles in (1, 2, 4):
            B.sg_matvec_select(g.op, tiles)
            assert B.sg_matvec_tiles(g.op) == tiles
            Y = g.new_vec()
            B.sg_matvec(g.op, _to_dev(X), Y)
            assert _rel(_to_host(Y, X.shape), ref) < 1e-13
        ms = B.sg_matvec_autotune(g.op, 3)
        print(f"[gpu] matvec shapes 1/2/4 tiles: {ms} ms")
        assert all(v is not None and v > 0 for v in ms)
        assert B.sg_matvec_tiles(g.op) == (1, 2, 4)[int(np.argmin(ms))]
        with pytest.raises(B.SgError):
            B.sg_matvec_select(g.op, 3)
    finally:
        B.sg_matvec_select(g.op, 2)
    _, _, gw = built("c3_40")                     # grouped kernel: no tile shapes
    assert B.sg_matvec_tiles(gw.op) == 0
    with pytest.raises(B.SgError):
        B.sg_matvec_autotune(gw.op, 1)


def test_matvec_rejects_alias(built):
    pr, S, g = built("c0")
    X = g.new_vec(1.0)
    with pytest.raises(B.SgError):
        B.sg_matvec(g.op, X, X)


# ------------------------------------------------------------------ a4
def _oracle_ras(pr, S, owner=None, n_sub=None, overlap=None):
    owner = pr.owner if owner is None else owner
    return oras.ras_setup(S.K[0], owner, pr.n_sub if n_sub is None else n_sub, S.adj,
                          pr.overlap if overlap is None else overlap)


@pytest.mark.parametrize("key", ["c0", "c1_64", "c3_40", "c4_ragged", "p1_det", "j4", "g6"])
def test_ras_fp64_matches_oracle(built, key):
    pr, S, g = built(key)
    subs = _oracle_ras(pr, S)
    nloc, nlev, _ = B.ras_info(g.ras, pr.n_sub)
    assert nloc.tolist() == [len(sd.nodes) for sd in subs]
    R = np.random.default_rng(12).standard_normal((pr.mesh.n, S.P))
    Z = g.new_vec()
    B.ras_apply(g.ras, _to_dev(R), Z)
    assert _rel(_to_host(Z, R.shape), oras.ras_apply(subs, R, S.alpha_fact)) < 1e-10


# Unit roundoff of the stored factors and of the operands the matrix cores read.
U_FP32, U_BF16 = 2.0 ** -24, 2.0 ** -8
# Sweep path: each of the two sweeps applies one stored Schur-complement
# inverse per block (relative error <= u per entry) to an operand rounded to
# the same precision (<= u), so one sweep perturbs its block by about 2u and
# the two sweeps by about 4u; the blocks are diagonally dominant (the mean
# stiffness is an M-matrix), so the chain of blocks does not amplify it.
# Measured: FP32 1.4-1.7e-7 (2.3-2.9u), BF16 5.6-6.2e-3 (1.4-1.6u).
SWEEP_BOUND = {"fp32": 8 * U_FP32, "bf16": 4 * U_BF16}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ras_low_precision_close_to_oracle(built, prec):
    tol = SWEEP_BOUND[prec]
    pr, S, g = built("c1_64", prec=prec)
    subs = _oracle_ras(pr, S)
    R = np.random.default_rng(13).standard_normal((pr.mesh.n, S.P))
    Z = g.new_vec()
    B.ras_apply(g.ras, _to_dev(R), Z)
    err = _rel(_to_host(Z, R.shape), oras.ras_apply(subs, R, S.alpha_fact))
    print(f"[gpu] RAS {prec} rel err {err:.3e}")
    assert err < tol


# keys whose FP64 fused dense path fits (P <= 16, right-hand sides in LDS)
FUSED_FP64 = {"c0", "p1_det", "big_sub"}


@pytest.mark.parametrize("key", ["c0", "c1_64", "c3_40", "c4_ragged", "p1_det", "j4", "g6", "big_sub"])
def test_ras_dense_path_matches_oracle(built, key):
    """The explicit-inverse paths compute the same operator as the sweeps."""
    pr, S, g = built(key)
    subs = _oracle_ras(pr, S)
    R = np.random.default_rng(15).standard_normal((pr.mesh.n, S.P))
    Z = g.new_vec()
    try:
        # 64 and 32 owned rows per wave, and the fused gather + product
        for path in ("dense", "dense32", "fused"):
            if path == "fused" and key not in FUSED_FP64:
                with pytest.raises(B.SgError) as ei:
                    B.ras_select(g.ras, path)
                assert ei.value.code == -4          # SG_ERR_UNSUPPORTED
                continue
            B.ras_select(g.ras, path)
            dense, nbytes, name = B.ras_path_info(g.ras)
            assert dense and nbytes > 0 and name == path
            B.ras_apply(g.ras, _to_dev(R), Z)
            assert _rel(_to_host(Z, R.shape), oras.ras_apply(subs, R, S.alpha_fact)) < 1e-10
            # the damped form used inside the two-grid cycle, against the sweeps
            omega = 0.5
            op = g.new_vec()
            B.sg_precond_apply(g.op, g.ras, None, omega, _to_dev(R), op, None)
            B.ras_select(g.ras, False)
            op_sweep = g.new_vec()
            B.sg_precond_apply(g.op, g.ras, None, omega, _to_dev(R), op_sweep, None)
            torch.cuda.synchronize()
            assert float((op - op_sweep).abs().max() / op_sweep.abs().max()) < 1e-10
    finally:
        B.ras_select(g.ras, False)


def _round_f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _round_bf16(a):
    """FP64 -> FP32 (round to nearest) -> BF16 (round to nearest, ties to
    even on the FP32 bit pattern): the rounding of the stored inverse rows and
    of the right-hand sides the BF16 matrix-core products read."""
    u = np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ras_dense_low_precision_replays_rounding(built, prec):
    """Dense paths (64 / 32 rows per wave, fused): Z_owned = (rounded owned
    rows of (R_s K_0 R_s^T)^{-1}) (rounded R_s R) / alpha!, FP32 accumulation.
    A CPU replay applies the same two roundings in FP64; what remains is the
    FP32 summation over the n_s local nodes, bounded elementwise by
    gamma_{n_s} = n_s u_32 / (1 - n_s u_32) times |A~||R~| / alpha! (Higham,
    Thm. 3.5).  The error against the exact oracle is also bounded, by the
    two roundings: 2u |A^{-1}||R| / alpha! plus the same summation term."""
    import scipy.linalg as sla
    rnd = _round_f32 if prec == "fp32" else _round_bf16
    u = U_FP32 if prec == "fp32" else U_BF16
    pr, S, g = built("c1_64", prec=prec)
    subs = _oracle_ras(pr, S)
    R = np.random.default_rng(16).standard_normal((pr.mesh.n, S.P))
    replay = np.zeros_like(R)
    absbound = np.zeros_like(R)
    exact_bound = np.zeros_like(R)
    nmax = 0
    for sd in subs:
        nl = len(sd.nodes)
        nmax = max(nmax, nl)
        inv = sla.cho_solve(sd.chol, np.eye(nl))[sd.owned]
        Ar, Rr = rnd(inv), rnd(R[sd.nodes])
        own = sd.nodes[sd.owned]
        replay[own] = (Ar @ Rr) / S.alpha_fact[None, :]
        absbound[own] = (np.abs(Ar) @ np.abs(Rr)) / S.alpha_fact[None, :]
        exact_bound[own] = (np.abs(inv) @ np.abs(R[sd.nodes])) / S.alpha_fact[None, :]
    gamma = nmax * U_FP32 / (1.0 - nmax * U_FP32)
    exact = oras.ras_apply(subs, R, S.alpha_fact)
    Z = g.new_vec()
    try:
        for path in ("dense", "dense32", "fused"):
            B.ras_select(g.ras, path)
            B.ras_apply(g.ras, _to_dev(R), Z)
            Zh = _to_host(Z, R.shape)
            d_rep = np.abs(Zh - replay)
            d_ex = np.abs(Zh - exact)
            print(f"[gpu] dense RAS {prec} {path}: vs replay {(d_rep / absbound).max():.2e} of "
                  f"|A||R|, vs oracle rel {_rel(Zh, exact):.2e}", flush=True)
            assert (d_rep <= gamma * absbound + 1e-300).all()
            assert (d_ex <= (2 * u + u * u) * exact_bound + gamma * absbound).all()
    finally:
        B.ras_select(g.ras, False)


def test_ras_autotune_and_dense_fgmres(built):
    """The autotuner times the four paths and keeps the fastest; FGMRES with
    the dense and the fused dense BF16 local solves still reaches the FP64
    solution (mixed path)."""
    pr, S, _ = built("c1_64")
    g = GpuSG(pr, prec="bf16", coarse="amg", ras_path="auto")
    try:
        ms = g.ras_ms
        _, _, name = B.ras_path_info(g.ras)
        print(f"[gpu] RAS autotune: sweep / dense / dense32 / fused {ms} ms -> {name}")
        assert len(ms) == 4 and min(ms) > 0
        assert name == ("sweep", "dense", "dense32", "fused")[int(np.argmin(ms))]
        ref = osg.sg_solve_direct(S.K, S.G, S.B)
        for path in ("dense", "fused"):
            B.ras_select(g.ras, path)
            x, info = g.solve(pr.restart, 1e-10)
            assert info["converged"]
            assert _rel(_to_host(x, ref.shape), ref) < 1e-8
    finally:
        g.close()


def test_autotune_cache_reuses_choices(built, tmp_path):
    """A second set-up of the same shape takes the matvec shape and the RAS
    path from the cache instead of timing them."""
    pr, _, _ = built("c1_64")
    path = str(tmp_path / "tune.json")
    g1 = GpuSG(pr, prec="bf16", coarse="none", ras_path="auto", tune_cache=path)
    try:
        assert not g1.tuned_from_cache and g1.ras_ms is not None and g1.mv_ms is not None
        choice = (B.sg_matvec_tiles(g1.op), B.ras_path_info(g1.ras)[2])
    finally:
        g1.close()
    g2 = GpuSG(pr, prec="bf16", coarse="none", ras_path="auto", tune_cache=path)
    try:
        assert g2.tuned_from_cache and g2.ras_ms is None and g2.mv_ms is None
        assert (B.sg_matvec_tiles(g2.op), B.ras_path_info(g2.ras)[2]) == choice
    finally:
        g2.close()


def test_ras_single_subdomain_exact(built):
    pr, S, _ = built("c4_ragged")
    owner = np.zeros(pr.mesh.n, dtype=np.int32)
    g = GpuSG(pr, coarse="none", owner=owner, n_sub=1, overlap=0)
    try:
        R = np.random.default_rng(14).standard_normal((pr.mesh.n, S.P))
        Z = g.new_vec()
        B.ras_apply(g.ras, _to_dev(R), Z)
        import scipy.sparse.linalg as spla
        ref = spla.spsolve(S.K[0].tocsc(), R) / S.alpha_fact[None, :]
        assert _rel(_to_host(Z, R.shape), ref) < 1e-10
    finally:
        g.close()


def test_ras_rejects_bad_owner(built):
    pr, S, g = built("c0")
    owner = pr.owner.copy()
    owner[3] = pr.n_sub      # out of range: must fail on the host, before any launch
    with pytest.raises(B.SgError):
        B.ras_setup(g.op, owner, pr.n_sub, 1)


# ------------------------------------------------------------------ a5
@pytest.mark.parametrize("key", ["c1_64", "c4_ragged", "c3_40"])
def test_coarse_and_vcycle_match_oracle(built, key):
    pr, S, g = built(key)
    Z = ocoarse.nicolaides(pr.owner, pr.n_sub)
    C = ocoarse.coarse_blocks(S.K, Z)
    h = oamg.setup(ocoarse.coarse_operator(C, S.G), S.P)
    nl, nodes, agg = B.amg_info(g.amg, pr.n_sub)
    assert nl == h.n_levels
    assert nodes.tolist() == [A.shape[0] // S.P for A in h.A]
    if h.n_levels > 1:
        assert np.array_equal(agg, h.aggs[0])
    # stored blocks per level: R = P^T holds as many blocks as P, every node
    # has its diagonal block and a prolongator block; the coarsest level is dense
    for lv in range(nl):
        a_b, p_b, r_b = B.amg_level_blocks(g.amg, lv)
        if lv < nl - 1:
            assert a_b >= nodes[lv] and p_b >= nodes[lv] and r_b == p_b
        else:
            assert (a_b, p_b, r_b) == (int(nodes[lv]) ** 2, 0, 0)
    with pytest.raises(B.SgError):
        B.amg_level_blocks(g.amg, nl)
    rng = np.random.default_rng(15)
    R = rng.standard_normal((pr.mesh.n, S.P))
    rc = torch.zeros(pr.n_sub * S.P, dtype=torch.float64, device="cuda")
    B.sg_coarse_restrict(g.amg, _to_dev(R), rc)
    assert _rel(_to_host(rc, (pr.n_sub, S.P)), ocoarse.restrict(Z, R)) < 1e-13
    bc = rng.standard_normal((pr.n_sub, S.P))
    xc = torch.zeros_like(rc)
    B.amg_vcycle(g.amg, _to_dev(bc), xc)
    assert _rel(_to_host(xc, bc.shape), oamg.vcycle(h, bc.ravel()).reshape(bc.shape)) < 1e-10
    Y = _to_dev(R)
    B.sg_coarse_prolong_add(g.amg, _to_dev(bc), Y)
    assert _rel(_to_host(Y, R.shape), R + ocoarse.prolong(Z, bc)) < 1e-14


def test_mean_exact_coarse_matches_oracle(built):
    pr, S, g = built("c0", coarse="mean")
    Z = ocoarse.nicolaides(pr.owner, pr.n_sub)
    cs = ocoarse.MeanExactCoarse(ocoarse.coarse_blocks(S.K, Z), S.alpha_fact)
    bc = np.random.default_rng(16).standard_normal((pr.n_sub, S.P))
    xc = torch.zeros(pr.n_sub * S.P, dtype=torch.float64, device="cuda")
    B.amg_vcycle(g.amg, _to_dev(bc), xc)
    assert _rel(_to_host(xc, bc.shape), cs(bc)) < 1e-12


# ------------------------------------------------------------------ a6
@pytest.mark.parametrize("key,coarse", [("c0", "mean"), ("c1_64", "amg"), ("c3_40", "amg")])
def test_two_level_cycle_matches_oracle(built, key, coarse):
    pr, S, g = built(key, coarse=coarse)
    rho, omega = g.damping()
    B2, subs, C, cs = osys.two_level(S, pr.owner, pr.n_sub, pr.overlap, coarse)
    assert rho == pytest.approx(
        smoother_radius(S.matvec, lambda R: oras.ras_apply(subs, R, S.alpha_fact), S.B.shape),
        rel=1e-9)
    B2.omega = omega
    R = np.random.default_rng(17).standard_normal((pr.mesh.n, S.P))
    Z = g.new_vec()
    B.sg_precond_apply(g.op, g.ras, g.amg, omega, _to_dev(R), Z, g.precond_workspace())
    assert _rel(_to_host(Z, R.shape), B2(R)) < 1e-10


# ------------------------------------------------------------------ a7
@pytest.mark.parametrize("key,coarse,restart", [("c0", "mean", 30), ("c1_64", "amg", 50),
                                                 ("p1_det", "amg", 30), ("c4_ragged", "amg", 50),
                                                 ("g6", "amg", 50)])
def test_fgmres_solution_matches_direct(built, key, coarse, restart):
    pr, S, g = built(key, coarse=coarse)
    ref = osg.sg_solve_direct(S.K, S.G, S.B)
    x, info = g.solve(restart, 1e-12)
    print(f"[gpu] {key}: its={info['iterations']} relres={info['true_relres']:.2e} "
          f"omega={info['omega']:.3f}", flush=True)
    assert info["converged"] and info["true_relres"] <= 1e-12
    U = _to_host(x, ref.shape)
    assert np.linalg.norm(U - ref) / np.linalg.norm(ref) < 1e-8


@pytest.mark.parametrize("key", ["s21", "s24", "s44"])
def test_fgmres_sweep_shapes_match_direct(built, key):
    """Orders p = 1 and p = 4 of the stochastic-dimension sweep (generic and
    wide matvec kernels inside the solve)."""
    pr, S, g = built(key)
    ref = osg.sg_solve_direct(S.K, S.G, S.B)
    x, info = g.solve(50, 1e-12)
    assert info["converged"] and info["true_relres"] <= 1e-12
    err = np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref)
    print(f"[gpu] {key}: P={S.P} its={info['iterations']} err={err:.2e}", flush=True)
    assert err < 1e-8


def test_fgmres_c3_40_matches_oracle_fgmres(built):
    """The jittered P = 84 case: its Kronecker matrix (16M non-zeros) is too
    large for a quick sparse direct solve, so the reference is the oracle's
    own FGMRES with its two-level preconditioner, run to a relative residual
    of 1e-13 (within 2e-14 of the direct solution, checked once offline); the
    GPU's FP64 solve at 1e-12 must match it to 1e-8."""
    pr, S, g = built("c3_40")
    B2, *_ = osys.two_level(S, pr.owner, pr.n_sub, pr.overlap, "amg")
    ref, oinfo = osys.solve(S, B2, 50, 1e-13, max_it=2000)
    assert oinfo.converged
    x, info = g.solve(50, 1e-12)
    assert info["converged"] and info["true_relres"] <= 1e-12
    err = np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref)
    print(f"[gpu] c3_40: its={info['iterations']} (oracle {oinfo.iterations}) err={err:.2e}",
          flush=True)
    assert err < 1e-8


@pytest.mark.parametrize("ortho", ["cgs", "cgs2"])
@pytest.mark.parametrize("key", ["c1_64", "c4_ragged", "c3_40"])
def test_fgmres_classical_gram_schmidt(built, key, ortho):
    """Classical Gram-Schmidt (one pass, or with the conditional second pass)
    reaches the solution (the oracle's direct solve on the small cases, the
    modified Gram-Schmidt solve on the P = 84 case whose Kronecker matrix is
    too large for a sparse direct solve); its residual history follows
    modified Gram-Schmidt's to rounding over the first iterations."""
    pr, S, g = built(key)
    x, info = g.solve(50, 1e-10, ortho=ortho)
    assert info["converged"] and info["true_relres"] <= 1e-10
    x_m, info_m = g.solve(50, 1e-10, ortho="mgs")
    if key == "c3_40":
        ref = _to_host(x_m, (pr.mesh.n, S.P))
    else:
        ref = osg.sg_solve_direct(S.K, S.G, S.B)
    assert np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref) < 1e-8
    n = min(len(info["history"]), len(info_m["history"]), 10)
    assert np.allclose(info["history"][:n], info_m["history"][:n], rtol=1e-8)
    assert abs(info["iterations"] - info_m["iterations"]) <= 2
    x2, info2 = g.solve(50, 1e-10, ortho=ortho, use_graph=True)
    assert torch.equal(x, x2)


BLOCK = {"block2": 2, "block3": 3, "block4": 4}


@pytest.mark.parametrize("ortho", list(BLOCK))
@pytest.mark.parametrize("key,coarse", [("c0", "mean"), ("c1_64", "amg"), ("c4_ragged", "amg"),
                                       ("c3_40", "amg"), ("j4", "amg")])
def test_fgmres_block_gram_schmidt(built, key, coarse, ortho):
    """S directions per Gram-Schmidt pass (blocks u_1 = A M v_j,
    u_{t+1} = A M u_t): with the fixed FP64 preconditioner the Krylov spaces
    are those of one step at a time, so after every block (column S k - 1)
    the residual estimate equals modified Gram-Schmidt's after the same
    column; the solution reaches the direct one (the MGS solve for the
    P = 84 case), and graph replay equals the eager run bit for bit."""
    pr, S, g = built(key, coarse=coarse)
    sb = BLOCK[ortho]
    restart = 30 if key == "c0" else 50
    x, info = g.solve(restart, 1e-10, ortho=ortho)
    assert info["converged"] and info["true_relres"] <= 1e-10
    x_m, info_m = g.solve(restart, 1e-10, ortho="mgs")
    if key == "c3_40":
        ref = _to_host(x_m, (pr.mesh.n, S.P))
    else:
        ref = osg.sg_solve_direct(S.K, S.G, S.B)
    assert np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref) < 1e-8
    hb, hm = info["history"], info_m["history"]
    nblk = min(len(hb) - 1, (len(hm) - 1) // sb, 8, restart // sb)
    assert nblk >= 2
    for k in range(1, nblk + 1):
        assert hb[k] == pytest.approx(hm[sb * k], rel=1e-6), k
    print(f"[gpu] {ortho} {key}: its={info['iterations']} (mgs {info_m['iterations']})", flush=True)
    assert abs(info["iterations"] - info_m["iterations"]) <= sb
    x2, info2 = g.solve(restart, 1e-10, ortho=ortho, use_graph=True)
    assert info2["iterations"] == info["iterations"] and torch.equal(x, x2)


@pytest.mark.parametrize("ortho", list(BLOCK))
def test_fgmres_block_odd_restart_and_cap(built, ortho):
    """A restart length that the block does not divide ends each cycle with
    a shorter block or a single step; so does a step budget; both keep the
    solution exact and the budget exact."""
    pr, S, g = built("c4_ragged")
    ref = osg.sg_solve_direct(S.K, S.G, S.B)
    x, info = g.solve(7, 1e-10, ortho=ortho, max_it=2000)
    assert info["converged"] and info["restarts"] >= 1
    assert np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref) < 1e-8
    x5, info5 = g.solve(10, 1e-14, ortho=ortho, max_it=5)
    assert info5["iterations"] == 5 and info5["status"] == B.SG_NOT_CONVERGED
    x5m, info5m = g.solve(10, 1e-14, ortho="mgs", max_it=5)
    assert info5["true_relres"] == pytest.approx(info5m["true_relres"], rel=1e-6)


@pytest.mark.parametrize("ortho", ["block2", "block4"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fgmres_block_mixed_precision_refines_to_fp64(built, prec, ortho):
    """With a low-precision (not exactly linear) preconditioner the pair's
    second direction M u1 is still a valid flexible direction: the solve
    reaches the FP64 solution."""
    pr, S, g = built("c1_64", prec=prec)
    ref = osg.sg_solve_direct(S.K, S.G, S.B)
    x, info = g.solve(50, 1e-10, ortho=ortho)
    err = np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref)
    assert info["converged"] and err < 1e-6


def test_fgmres_iterations_track_oracle(built):
    pr, S, g = built("c0", coarse="mean")
    B2, *_ = osys.two_level(S, pr.owner, pr.n_sub, pr.overlap, "mean")
    _, oinfo = osys.solve(S, B2, 30, 1e-8)
    x, info = g.solve(30, 1e-8)
    assert abs(info["iterations"] - oinfo.iterations) <= 1
    h = info["history"]
    n = min(len(h), len(oinfo.history), 10)
    assert np.allclose(h[:n], oinfo.history[:n], rtol=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fgmres_mixed_precision_refines_to_fp64(built, prec):
    pr, S, g = built("c1_64", prec=prec)
    ref = osg.sg_solve_direct(S.K, S.G, S.B)
    x, info = g.solve(50, 1e-10)
    err = np.linalg.norm(_to_host(x, ref.shape) - ref) / np.linalg.norm(ref)
    print(f"[gpu] mixed {prec}: its={info['iterations']} err={err:.2e}", flush=True)
    assert info["converged"] and err < 1e-6


def test_fgmres_bitwise_reproducible(built):
    pr, S, g = built("c4_ragged")
    x1, i1 = g.solve(50, 1e-10)
    x2, i2 = g.solve(50, 1e-10)
    assert i1["iterations"] == i2["iterations"]
    assert torch.equal(x1, x2)


def test_fgmres_unpreconditioned_matches_library_gmres(built):
    import scipy.sparse.linalg as spla
    pr, S, g = built("c0")
    hist = []
    spla.gmres(osg.sg_kron(S.K, S.G), S.B.ravel(), restart=20, rtol=1e-9, maxiter=1,
               callback=lambda r: hist.append(r), callback_type="pr_norm")
    x, info = g.solve(20, 1e-9, max_it=20, use_precond=False)
    assert np.allclose(info["history"][1:21], hist[:20], rtol=1e-7)


def test_fgmres_zero_rhs_and_cap(built):
    pr, S, g = built("c0")
    x, info = g.solve(10, 1e-12, max_it=1)
    assert info["iterations"] == 1 and not info["converged"]
    assert info["status"] == B.SG_NOT_CONVERGED


# ------------------------------------------------------------------ full size
@pytest.fixture(scope="module")
def full_c1():
    _cuda()
    import scipy.sparse as sp  # noqa: F401
    pr = make_problem("c1")
    print(f"[gpu] full-size config: n={pr.mesh.n} P=35", flush=True)
    S = _oracle(pr)
    g = GpuSG(pr, prec="fp64", coarse="amg")
    yield pr, S, g
    g.close()


def test_full_size_matvec_sampled_rows(full_c1):
    """The 9.14M-unknown workload in the benchmark's launch configuration:
    every output row of a random field checked on a sample of rows."""
    pr, S, g = full_c1
    rng = np.random.default_rng(21)
    X = rng.standard_normal((pr.mesh.n, S.P))
    Y = g.new_vec()
    B.sg_matvec(g.op, _to_dev(X), Y)
    Yh = _to_host(Y, X.shape)
    rows = np.unique(np.concatenate([rng.choice(pr.mesh.n, 3000, replace=False),
                                     np.arange(0, 40), np.arange(pr.mesh.n - 40, pr.mesh.n)]))
    ref = np.zeros((rows.size, S.P))
    for i, Ki in enumerate(S.K):
        ref += (Ki[rows] @ X) @ S.G[i].T
    assert _rel(Yh[rows], ref) < 1e-13


def test_full_size_matrix_free_matvec_sampled_rows(full_c1):
    """The matrix-free apply on the 9.14M-unknown workload: sampled rows
    against the oracle, all rows against the stored-value apply."""
    pr, S, g = full_c1
    rng = np.random.default_rng(25)
    X = rng.standard_normal((pr.mesh.n, S.P))
    Xd = _to_dev(X)
    Ys = g.new_vec()
    B.sg_matvec(g.op, Xd, Ys)
    try:
        B.sg_matvec_matrix_free(g.op, True)
        Y = g.new_vec()
        B.sg_matvec(g.op, Xd, Y)
        torch.cuda.synchronize()
        assert float((Y - Ys).abs().max() / Ys.abs().max()) < 1e-14
        Yh = _to_host(Y, X.shape)
        rows = np.unique(np.concatenate([rng.choice(pr.mesh.n, 2000, replace=False),
                                         np.arange(0, 600), np.arange(pr.mesh.n - 600, pr.mesh.n)]))
        ref = np.zeros((rows.size, S.P))
        for i, Ki in enumerate(S.K):
            ref += (Ki[rows] @ X) @ S.G[i].T
        assert _rel(Yh[rows], ref) < 1e-13
    finally:
        B.sg_matvec_matrix_free(g.op, False)


def test_full_size_c3_matvec_sampled_rows():
    """The 12.3M-unknown jittered workload (P = 84, 7 entries per row, grouped
    kernel): sampled output rows against the oracle's stiffness matrices.  The
    residual form C - A X (C aliasing Y) is covered by the two-level cycle
    tests on the P = 84 case."""
    _cuda()
    pr = make_problem("c3")
    print(f"[gpu] full-size c3: n={pr.mesh.n}", flush=True)
    S = _oracle(pr)
    g = GpuSG(pr, prec="fp64", coarse="none")
    try:
        assert B.sg_matvec_kernel(g.op) == "grouped"
        rng = np.random.default_rng(24)
        X = rng.standard_normal((pr.mesh.n, S.P))
        Y = g.new_vec()
        B.sg_matvec(g.op, _to_dev(X), Y)
        Yh = _to_host(Y, X.shape)
        rows = np.unique(np.concatenate([rng.choice(pr.mesh.n, 2000, replace=False),
                                         np.arange(0, 70), np.arange(pr.mesh.n - 70, pr.mesh.n)]))
        ref = np.zeros((rows.size, S.P))
        for i, Ki in enumerate(S.K):
            ref += (Ki[rows] @ X) @ S.G[i].T
        assert _rel(Yh[rows], ref) < 1e-13
    finally:
        g.close()


def test_full_size_ras_sampled_subdomains(full_c1):
    """RAS at full size: the owned rows of a sample of subdomains against the
    oracle's dense local solves of those subdomains."""
    import scipy.linalg as sla
    pr, S, g = full_c1
    rng = np.random.default_rng(22)
    R = rng.standard_normal((pr.mesh.n, S.P))
    Z = g.new_vec()
    B.ras_apply(g.ras, _to_dev(R), Z)
    Zh = _to_host(Z, R.shape)
    for sd in (0, 15, 17, 100, 255):
        own = np.nonzero(pr.owner == sd)[0]
        nodes = oras.grow_overlap(own, S.adj, pr.overlap)
        loc = sla.cho_solve(sla.cho_factor(S.K[0][nodes][:, nodes].toarray(), lower=True),
                            R[nodes]) / S.alpha_fact[None, :]
        mask = pr.owner[nodes] == sd
        assert _rel(Zh[nodes[mask]], loc[mask]) < 1e-10, sd


def _sampled_local_solves(pr, S, R, subs):
    """The oracle's dense local solves of a few subdomains: (owned node ids,
    their rows of the RAS output)."""
    import scipy.linalg as sla
    out = []
    for sd in subs:
        own = np.nonzero(pr.owner == sd)[0]
        nodes = oras.grow_overlap(own, S.adj, pr.overlap)
        loc = sla.cho_solve(sla.cho_factor(S.K[0][nodes][:, nodes].toarray(), lower=True),
                            R[nodes]) / S.alpha_fact[None, :]
        mask = pr.owner[nodes] == sd
        out.append((nodes[mask], loc[mask]))
    return out


def test_full_size_ras_dense_and_fused_paths(full_c1):
    """The explicit-inverse paths at full size: FP64 dense (64 and 32 rows per
    wave) against the oracle's local solves to 1e-10, and the BF16 fused path
    the benchmark times against them to the BF16 bound and bit for bit
    against the BF16 two-kernel path."""
    pr, S, g = full_c1
    rng = np.random.default_rng(23)
    R = rng.standard_normal((pr.mesh.n, S.P))
    ref = _sampled_local_solves(pr, S, R, (0, 31, 128, 255))
    Z = g.new_vec()
    try:
        for path in ("dense", "dense32"):
            B.ras_select(g.ras, path)
            B.ras_apply(g.ras, _to_dev(R), Z)
            Zh = _to_host(Z, R.shape)
            for rows, loc in ref:
                assert _rel(Zh[rows], loc) < 1e-10, path
    finally:
        B.ras_select(g.ras, "sweep")
    # BF16: the rounding replay of the sampled subdomains (see
    # test_ras_dense_low_precision_replays_rounding for the bound)
    import scipy.linalg as sla
    replays = []
    for sd in (0, 31, 128, 255):
        own = np.nonzero(pr.owner == sd)[0]
        nodes = oras.grow_overlap(own, S.adj, pr.overlap)
        mask = pr.owner[nodes] == sd
        inv = sla.cho_solve(sla.cho_factor(S.K[0][nodes][:, nodes].toarray(), lower=True),
                            np.eye(len(nodes)))[mask]
        Ar, Rr = _round_bf16(inv), _round_bf16(R[nodes])
        gamma = len(nodes) * U_FP32 / (1.0 - len(nodes) * U_FP32)
        replays.append((nodes[mask], (Ar @ Rr) / S.alpha_fact[None, :],
                        gamma * (np.abs(Ar) @ np.abs(Rr)) / S.alpha_fact[None, :]))
    g16 = GpuSG(pr, prec="bf16", coarse="none")
    try:
        out = {}
        for path in ("dense", "fused"):
            B.ras_select(g16.ras, path)
            Z16 = g16.new_vec()
            B.ras_apply(g16.ras, _to_dev(R), Z16)
            out[path] = Z16
            Zh = _to_host(Z16, R.shape)
            for (rows, loc), (rows2, rep, bound) in zip(ref, replays):
                assert np.array_equal(rows, rows2)
                assert (np.abs(Zh[rows] - rep) <= bound).all(), path
                assert _rel(Zh[rows], loc) < 2 * U_BF16, path
        assert torch.equal(out["dense"], out["fused"])
    finally:
        g16.close()


@pytest.mark.parametrize("local", ["mean", "kron"])
def test_fp32_fused_path_with_long_chunks(local):
    """The FP32 fused dense RAS gathers the next chunk's right-hand sides in
    bursts of seven entries per thread; subdomains of ~1,900 local nodes
    (two work-groups of owned rows each) make chunks of 10,080 entries, so
    the entries past the bursts take the fetch at the chunk's end.  The fused
    result equals the two-kernel dense path's bit for bit with mean-based
    local solves (same products in the same order), and to the FP32 level
    with Kronecker ones (mixing on the output instead of the input); both
    match the FP64 sweep to the FP32 level."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pr = make_problem("c1", nc=80, sub=(2, 2))
    R = np.random.default_rng(61).standard_normal(pr.mesh.n * 35)
    Rd = _to_dev(R)
    out = {}
    with GpuSG(pr, prec="fp64", coarse="none", ras_path="sweep", local=local) as g:
        Z = g.new_vec()
        B.ras_apply(g.ras, Rd, Z)
        out["fp64"] = Z.clone()
    with GpuSG(pr, prec="fp32", coarse="none", local=local) as g:
        for path in ("dense", "fused"):
            B.ras_select(g.ras, path)
            assert B.ras_path_info(g.ras)[2] == path
            Z = g.new_vec()
            B.ras_apply(g.ras, Rd, Z)
            out[path] = Z.clone()
    for path in ("dense", "fused"):
        err = float(torch.linalg.norm(out[path] - out["fp64"]) / torch.linalg.norm(out["fp64"]))
        print(f"[gpu] fp32 {local} {path} vs fp64 sweep: {err:.2e}", flush=True)
        assert err < 2e-5, path
    if local == "mean":
        assert torch.equal(out["dense"], out["fused"])
    else:
        d = float(torch.linalg.norm(out["fused"] - out["dense"]) / torch.linalg.norm(out["dense"]))
        assert d < 2e-5


# ------------------------------------------------------------------ a10
def test_graph_replay_matches_eager(built):
    """Arnoldi steps replayed from captured graphs give the eager result bit
    for bit, on every replay, with eager work and synchronisation between."""
    pr, S, g = built("c4_ragged")
    x_e, i_e = g.solve(50, 1e-10)
    for rep in range(3):
        x_g, i_g = g.solve(50, 1e-10, use_graph=True)
        assert i_g["iterations"] == i_e["iterations"]
        assert torch.equal(x_g, x_e), rep
        # eager work between replays
        Y = g.new_vec()
        B.sg_matvec(g.op, x_g, Y)
        torch.cuda.synchronize()
    assert B.sg_graph_cache_clear() > 0


def test_precond_fused_coarse_add_is_exact(built):
    """With the fused BF16 RAS the two-grid cycle adds the coarse correction
    inside the last smoothing's store instead of a separate prolongation;
    for mean-based local solves the fused and the dense RAS give identical
    bits, so the cycle must too."""
    pr, S, _ = built("c1_64")
    R = torch.from_numpy(np.random.default_rng(19).standard_normal(pr.mesh.n * S.P)).cuda()
    out = {}
    for path in ("dense", "fused"):
        g = GpuSG(pr, prec="bf16", coarse="amg", ras_path=path)
        try:
            Z = g.new_vec()
            B.sg_precond_apply(g.op, g.ras, g.amg, 0.45, R, Z, g.precond_workspace())
            torch.cuda.synchronize()
            out[path] = Z
        finally:
            g.close()
    assert torch.equal(out["dense"], out["fused"])


def test_graph_replay_fused_ras_matches_eager(built):
    """The BF16 solve with the fused dense RAS (its per-chunk barriers and
    run-ahead steps inside captured graphs) gives the eager result bit for
    bit on every replay."""
    pr, S, _ = built("c1_64")
    g = GpuSG(pr, prec="bf16", coarse="amg", ras_path="fused")
    try:
        assert B.ras_path_info(g.ras)[2] == "fused"
        x_e, i_e = g.solve(pr.restart, 1e-10)
        assert i_e["converged"]
        for rep in range(3):
            x_g, i_g = g.solve(pr.restart, 1e-10, use_graph=True)
            assert i_g["iterations"] == i_e["iterations"]
            assert torch.equal(x_g, x_e), rep
            Y = g.new_vec()
            B.sg_matvec(g.op, x_g, Y)
            torch.cuda.synchronize()
    finally:
        g.close()


def test_graph_cache_dropped_with_handles():
    _cuda()
    pr = make_problem("c0", nc=12, sub=(2, 2))
    g = GpuSG(pr, coarse="mean")
    x, info = g.solve(20, 1e-10, use_graph=True)
    assert info["converged"]
    g.close()                       # must release the graphs that reference g's handles
    assert B.sg_graph_cache_clear() == 0
