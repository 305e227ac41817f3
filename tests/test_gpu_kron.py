"""Kronecker (Ullmann) local solves on the GPU against the oracle: the
factor Gt, the RAS apply on every path, and the whole two-level solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ras as oras
from oracle import system as osys
from paper_2310_14649_amd import binding as B
from paper_2310_14649_amd.inputs import make_problem
from paper_2310_14649_amd.solver import GpuSG

pytestmark = pytest.mark.gpu

CASES = {
    "c1_64": dict(name="c1", nc=64, sub=(8, 8)),
    "c4_ragged": dict(name="c4", nc=23, sub=(3, 5)),
    "c3_40": dict(name="c3", nc=40, sub=(4, 4)),          # P = 84
    "m5p3": dict(name="c1", nc=24, M=5, p=3, sub=(3, 3)),  # P = 56
    "m2p3": dict(name="c1", nc=24, M=2, p=3, sub=(3, 3)),  # P = 10: the FP64 fused path
}


def _setup(key):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kw = dict(CASES[key])
    pr = make_problem(kw.pop("name"), **kw)
    m = pr.mesh
    S = osys.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)
    print(f"[gpu] kron case {key}: n={m.n} P={S.P}", flush=True)
    return pr, S


def _host(t, shape):
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(shape)


@pytest.mark.parametrize("key", ["c1_64", "c4_ragged", "c3_40", "m5p3", "m2p3"])
def test_kron_factor_and_ras_match_oracle(key):
    pr, S = _setup(key)
    subs = oras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    Gt = oras.kron_factor(S.K, S.G)
    R = np.random.default_rng(41).standard_normal((pr.mesh.n, S.P))
    ref = oras.ras_apply_kron(subs, R, Gt)
    with GpuSG(pr, prec="fp64", coarse="none", local="kron") as g:
        gt = B.ras_local_factor(g.ras, S.P)
        assert np.abs(gt - Gt).max() <= 1e-12 * np.abs(Gt).max()
        Rd = torch.from_numpy(R.ravel()).cuda()
        Zd = torch.zeros_like(Rd)
        for path in ("sweep", "dense", "dense32", "fused"):
            try:
                B.ras_select(g.ras, path)
            except B.SgError:
                assert path == "fused"          # where it does not fit LDS
                continue
            B.ras_apply(g.ras, Rd, Zd)
            Z = _host(Zd, R.shape)
            err = np.linalg.norm(Z - ref) / np.linalg.norm(ref)
            print(f"[gpu] {key} kron {path}: {err:.2e}", flush=True)
            assert err < 1e-10
        # back to the mean-based solves: the mean-based oracle again
        B.ras_select(g.ras, "sweep")
        B.ras_set_local(g.ras, g.op, "mean")
        B.ras_apply(g.ras, Rd, Zd)
        ref0 = oras.ras_apply(subs, R, S.alpha_fact)
        assert np.linalg.norm(_host(Zd, R.shape) - ref0) / np.linalg.norm(ref0) < 1e-10
        with pytest.raises(B.SgError):
            B.ras_local_factor(g.ras, S.P)
        with pytest.raises(B.SgError):
            B.ras_set_local(g.ras, g.op, 5)


# relative bounds from the operands' rounding: BF16 keeps 8 significant
# bits (2^-8 = 3.9e-3 per operand, a few of them per product), FP32 24 bits
# (6e-8 per operand, sums over ~1,300 local nodes)
LOW_BOUND = {"bf16": 2e-2, "fp32": 2e-5}


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
@pytest.mark.parametrize("key", ["c1_64", "c4_ragged"])
def test_kron_fused_output_mixing(key, prec):
    """The fused path applies the Kronecker mixing to its output
    (Z = N(R) Gt^{-1}) instead of its input; the other dense paths mix the
    input.  Both equal the oracle up to the rounding of the operands in the
    RAS precision, and each other to the same level."""
    pr, S = _setup(key)
    subs = oras.ras_setup(S.K[0], pr.owner, pr.n_sub, S.adj, pr.overlap)
    Gt = oras.kron_factor(S.K, S.G)
    R = np.random.default_rng(43).standard_normal((pr.mesh.n, S.P))
    ref = oras.ras_apply_kron(subs, R, Gt)
    out = {}
    with GpuSG(pr, prec=prec, coarse="none", local="kron") as g:
        Rd = torch.from_numpy(R.ravel()).cuda()
        for path in ("dense", "fused"):
            B.ras_select(g.ras, path)
            Zd = torch.zeros_like(Rd)
            B.ras_apply(g.ras, Rd, Zd)
            out[path] = _host(Zd, R.shape)
            err = np.linalg.norm(out[path] - ref) / np.linalg.norm(ref)
            print(f"[gpu] {key} kron {prec} {path}: {err:.2e}", flush=True)
            assert err < LOW_BOUND[prec]
    d = np.linalg.norm(out["fused"] - out["dense"]) / np.linalg.norm(out["dense"])
    assert d < LOW_BOUND[prec]


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
@pytest.mark.parametrize("key", ["c1_64", "c3_40"])
def test_kron_two_level_solve(key, prec):
    """The two-level FGMRES with Kronecker local solves meets the tolerance in
    the oracle's operator, agrees with the mean-based solve's solution and
    takes no more iterations (graphs on, so the captured steps see the mode)."""
    pr, S = _setup(key)
    res, its, sol = {}, {}, {}
    for local in ("mean", "kron"):
        with GpuSG(pr, prec=prec, coarse="amg", local=local) as g:
            x, info = g.solve(50, 1e-10, use_graph=True, ortho="cgs")
            U = _host(x, S.B.shape)
        res[local] = np.linalg.norm(S.B - S.matvec(U)) / np.linalg.norm(S.B)
        its[local], sol[local] = info["iterations"], U
        print(f"[gpu] {key} {prec} {local}: {its[local]} its, oracle relres {res[local]:.2e}",
              flush=True)
        assert info["converged"] and res[local] < 1e-9
    assert its["kron"] <= its["mean"]
    d = np.linalg.norm(sol["kron"] - sol["mean"]) / np.linalg.norm(sol["mean"])
    assert d < 1e-8
