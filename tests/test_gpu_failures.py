"""Error paths of the C ABI on the GPU, forced from the host with inputs that
every kernel processes normally (no fault, trap or hang): a non-finite
right-hand side or initial guess, an indefinite local block, and FGMRES's
lucky breakdown (the Krylov space holds the solution exactly)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2310_14649_amd import binding as B  # noqa: E402
from paper_2310_14649_amd.inputs import make_problem  # noqa: E402
from paper_2310_14649_amd.solver import GpuNewton, GpuSG  # noqa: E402

SG_ERR_NUMERIC = -3


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_rhs_is_a_numeric_error(bad):
    _cuda()
    pr = make_problem("c0", nc=12, sub=(2, 2))
    with GpuSG(pr, coarse="amg") as g:
        b = g.b.clone()
        b[17] = bad
        ws = g.workspace(30)
        x = g.new_vec()
        with pytest.raises(B.SgError) as e:
            B.fgmres_solve(g.op, g.ras, g.amg, b, x, 30, 100, 1e-8, 0.0, ws)
        assert e.value.code == SG_ERR_NUMERIC and "right-hand side" in str(e.value)
        # a finite b with a non-finite initial guess: the initial residual
        x0 = g.new_vec()
        x0[5] = bad
        with pytest.raises(B.SgError) as e:
            B.fgmres_solve(g.op, g.ras, g.amg, g.b, x0, 30, 100, 1e-8, 0.0, ws)
        assert e.value.code == SG_ERR_NUMERIC and "initial residual" in str(e.value)
        # the handles still work afterwards
        x, info = g.solve(30, 1e-10)
        assert info["converged"]


def test_indefinite_local_block_is_a_numeric_error():
    """kappa(u) = 1 + u at u = -5 (mean mode only) makes the mean-coefficient
    stiffness E[c kappa(u_T)] = -4 c_0 negative definite: the local
    factorisation meets a negative pivot at once."""
    _cuda()
    pr = make_problem("c4", nc=12, sub=(2, 2))
    with GpuNewton(pr, a2=0.0, a1=1.0) as g:
        U = torch.zeros(g.n * g.P, dtype=torch.float64, device="cuda")
        U.view(g.n, g.P)[:, 0] = -5.0
        g.residual(U)                                  # K1 assembled at U
        kop = B.sg_nl_mean_op(g.nl)
        with pytest.raises(B.SgError) as e:
            B.ras_setup(kop, g.owner, g.n_sub, g.overlap, B.SG_FP64)
        assert e.value.code == SG_ERR_NUMERIC and "pivot" in str(e.value)
        # a factorisation at a positive coefficient, then a refactorisation at
        # the indefinite one: the same error from ras_refactor
        g.residual(torch.zeros_like(U))
        ras = B.ras_setup(kop, g.owner, g.n_sub, g.overlap, B.SG_FP64)
        try:
            g.residual(U)
            with pytest.raises(B.SgError) as e:
                B.ras_refactor(ras, kop)
            assert e.value.code == SG_ERR_NUMERIC
        finally:
            B.sg_destroy_ras(ras)


@pytest.mark.parametrize("ortho", ["mgs", "block2", "block3", "block4"])
def test_lucky_breakdown_returns_exact_solution(ortho):
    """One unknown, deterministic (P = 1), no preconditioner: A v = k v
    exactly, so the first Arnoldi step leaves w - h v = 0, the breakdown
    flag ends the cycle, and x = b / k.  With step pairs the pair's first
    direction breaks down and the cycle keeps one column."""
    _cuda()
    pr = make_problem("c0", nc=2, M=0, p=0, sub=(1, 1))
    m = pr.mesh
    assert m.n == 1
    basis = B.sg_build_triples(0, 0, 0)
    op = B.sg_assemble(basis, m.xy, m.tri, m.dof, m.n, pr.g0, pr.g)
    try:
        rowptr, col, vals = B.sg_op_export(op)
        k = float(vals[0, 0])
        b = torch.tensor([3.0], dtype=torch.float64, device="cuda")
        x = torch.zeros(1, dtype=torch.float64, device="cuda")
        ws = torch.empty((B.fgmres_workspace_bytes(op, None, 10) + 7) // 8, dtype=torch.float64,
                         device="cuda")
        info = B.fgmres_solve(op, None, None, b, x, 10, 10, 1e-14, 1.0, ws, ortho=ortho)
        assert info["converged"] and info["iterations"] == 1
        assert float(x[0]) == pytest.approx(3.0 / k, rel=1e-15)
    finally:
        B.sg_destroy_op(op)
        B.sg_destroy_basis(basis)
