"""ras_refactor on a RAS that applies the dense inverse rows, followed by a
graph-replayed FGMRES solve: the refactorisation rebuilds the rows in the
buffer the captured Arnoldi-step graphs read, so the replayed solve equals
the eager solve bit for bit (before, the rebuild reallocated the buffer and
the graphs kept the old address)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2310_14649_amd import binding as B  # noqa: E402
from paper_2310_14649_amd.inputs import make_problem  # noqa: E402
from paper_2310_14649_amd.solver import GpuNewton  # noqa: E402


@pytest.mark.parametrize("path,prec", [("dense", "fp64"), ("fused", "bf16")])
def test_refactor_then_graph_replay_equals_eager(path, prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pr = make_problem("c4", nc=24, sub=(3, 3))
    with GpuNewton(pr) as g:
        # two smooth states (mean mode only): kappa(u) = 1 + u^2/2 changes the
        # values of K1 and of the Jacobian, not their conditioning
        U1 = torch.zeros(g.n * g.P, dtype=torch.float64, device="cuda")
        U2 = torch.zeros_like(U1)
        U2.view(g.n, g.P)[:, 0] = 0.5
        kop, jop = B.sg_nl_mean_op(g.nl), B.sg_nl_jac_op(g.nl)
        b = g.residual(U1)
        ras = B.ras_setup(kop, g.owner, g.n_sub, g.overlap, B.PREC[prec])
        amg = None
        try:
            B.ras_select(ras, path)
            amg = B.amg_setup(jop, ras, B.SG_COARSE_AMG, B.PREC[prec])
            ws = torch.empty((B.fgmres_workspace_bytes(jop, amg, 20) + 7) // 8,
                             dtype=torch.float64, device="cuda")
            x = torch.zeros_like(b)
            B.fgmres_solve(jop, ras, amg, b, x, 20, 400, 1e-8, 0.5, ws, use_graph=True)
            # new values at U2: K1 and the Jacobian change in place, the RAS is refactored
            b2 = g.residual(U2)
            B.ras_refactor(ras, kop)
            xg = torch.zeros_like(b2)
            ig = B.fgmres_solve(jop, ras, amg, b2, xg, 20, 400, 1e-8, 0.5, ws, use_graph=True)
            xe = torch.zeros_like(b2)
            ie = B.fgmres_solve(jop, ras, amg, b2, xe, 20, 400, 1e-8, 0.5, ws, use_graph=False)
            print(f"[gpu] refactor + graph ({path}, {prec}): {ie['iterations']} its, "
                  f"relres {ie['true_relres']:.2e}", flush=True)
            torch.cuda.synchronize()
            assert ig["iterations"] == ie["iterations"]
            assert torch.equal(xg, xe)
            assert ie["converged"]
        finally:
            B.sg_graph_cache_clear()
            if amg is not None:
                B.sg_destroy_amg(amg)
            B.sg_destroy_ras(ras)
