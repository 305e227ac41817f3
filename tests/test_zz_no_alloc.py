"""sg_precond_apply_noalloc (the two-grid cycle with its workspace in a
static device array) against sg_precond_apply with a caller workspace: the
same kernels on the same inputs, so the outputs agree bit for bit.  Two
calls in a row, the second on a smaller problem, so the second runs on
scratch that still holds the first call's contents; and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2310_14649_amd import binding as B  # noqa: E402
from paper_2310_14649_amd.inputs import make_problem  # noqa: E402
from paper_2310_14649_amd.solver import GpuSG  # noqa: E402


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(g, omega, seed, amg=True):
    N = g.n * g.P
    R = torch.from_numpy(np.random.default_rng(seed).standard_normal(N)).cuda()
    Z_ws = g.new_vec(7.0)
    Z_na = g.new_vec(-3.0)
    a = g.amg if amg else None
    B.sg_precond_apply(g.op, g.ras, a, omega, R, Z_ws, g.precond_workspace())
    B.sg_precond_apply_noalloc(g.op, g.ras, a, omega, R, Z_na)
    torch.cuda.synchronize()
    return Z_ws.cpu().numpy(), Z_na.cpu().numpy()


def test_noalloc_matches_workspace_apply_two_calls_second_smaller():
    _cuda()
    big = make_problem("c1", nc=64, sub=(4, 4))                     # P = 35, 139,195 unknowns
    small = make_problem("c0", nc=20, sub=(2, 2))                   # P = 6, 2,166 unknowns
    with GpuSG(big, prec="fp64", coarse="amg", local="kron") as g:
        print(f"noalloc: big n={g.n} P={g.P} ws={B.sg_precond_workspace_bytes(g.op, g.amg)}",
              flush=True)
        a, b = _both(g, 0.47, 1)
        assert np.array_equal(a, b)
        assert np.abs(a).max() > 0
        # the scratch now holds this call's T, r_c, e_c
    with GpuSG(small, prec="bf16", coarse="amg", ras_path="dense") as g:
        print(f"noalloc: small n={g.n} P={g.P}", flush=True)
        a, b = _both(g, 0.8, 2)
        assert np.array_equal(a, b)
        a, b = _both(g, 0.8, 3, amg=False)                          # one-level: no scratch
        assert np.array_equal(a, b)
    with GpuSG(small, prec="fp64", coarse="mean") as g:             # exact mean coarse solve
        a, b = _both(g, 1.0, 4)
        assert np.array_equal(a, b)


def test_noalloc_rejects_problems_beyond_the_scratch():
    _cuda()
    pr = make_problem("c1", nc=700, sub=(24, 24))                   # 488,601 x 35 unknowns
    with GpuSG(pr, prec="fp64", coarse="mean") as g:
        need = B.sg_precond_workspace_bytes(g.op, g.amg)
        print(f"noalloc: n={g.n} P={g.P} needs {need} bytes", flush=True)
        assert need > B.SG_NOALLOC_SCRATCH_BYTES
        R, Z = g.new_vec(1.0), g.new_vec()
        with pytest.raises(B.SgError) as e:
            B.sg_precond_apply_noalloc(g.op, g.ras, g.amg, 1.0, R, Z)
        assert e.value.code == -5 and "scratch" in str(e.value)
        # without the coarse solve the cycle needs no scratch
        B.sg_precond_apply_noalloc(g.op, g.ras, None, 1.0, R, Z)
        torch.cuda.synchronize()
        assert torch.isfinite(Z).all()
