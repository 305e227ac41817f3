"""Caller-owned device memory (sg_set_allocator / sg_set_arena): every
device buffer of the setup calls (sg_assemble, ras_setup, amg_setup,
sg_nl_setup, nn_create) and of the handles comes from the caller's source,
the results are bitwise those of the hipMalloc default, an arena sized by a
dry run fits exactly, and an arena one allocation too small fails with
SG_ERR_WORKSPACE and leaves nothing held."""
import gc

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2310_14649_amd import binding as B  # noqa: E402
from paper_2310_14649_amd.inputs import make_problem  # noqa: E402
from paper_2310_14649_amd.learned import init_params  # noqa: E402
from paper_2310_14649_amd.solver import GpuNewton, GpuSG  # noqa: E402

SG_ERR_WORKSPACE = -5


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(pr):
    with GpuSG(pr, coarse="amg", ras_path="sweep") as g:
        x, info = g.solve(pr.restart, 1e-10)
        assert info["converged"]
        torch.cuda.synchronize()
        return x.clone()


def test_torch_allocator_holds_every_setup_buffer():
    _cuda()
    pr = make_problem("c1", nc=40, sub=(4, 4))
    x_ref = _solve(pr)
    live0 = B.memory_stats()[0]
    torch.cuda.synchronize()
    t0 = torch.cuda.memory_allocated()
    B.use_torch_allocator(True)
    try:
        g = GpuSG(pr, coarse="amg", ras_path="sweep")
        held = B.memory_stats()[0] - live0
        grew = torch.cuda.memory_allocated() - t0
        assert held > 0 and grew >= held
        x, info = g.solve(pr.restart, 1e-10)
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref)
        # the nonlinear problem's handles and the network come from torch too
        prn = make_problem("c4", nc=24, sub=(2, 2))
        before = B.memory_stats()[0]
        nl = GpuNewton(prn)
        assert B.memory_stats()[0] > before
        nn = B.nn_create([5, 8, 8, 35], 23, 23, 2)
        B.nn_set_params(nn, init_params([5, 8, 8, 35], 0))
        B.nn_destroy(nn)
        nl.close()
        g.close()
        torch.cuda.synchronize()
    finally:
        B.use_torch_allocator(False)
    gc.collect()
    assert B.memory_stats()[0] == live0


def test_arena_sized_by_a_dry_run_fits_and_a_smaller_one_fails_cleanly():
    _cuda()
    pr = make_problem("c0", nc=24, sub=(2, 2))
    x_ref = _solve(pr)
    live0 = B.memory_stats()[0]
    big = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    with B.Arena(big) as ar:
        with GpuSG(pr, coarse="amg", ras_path="sweep") as g:
            x, _ = g.solve(pr.restart, 1e-10)
            torch.cuda.synchronize()
        need = ar.used()
        ar.reset()
    assert need > 0 and torch.equal(x, x_ref)
    exact = torch.empty(need, dtype=torch.uint8, device="cuda")
    with B.Arena(exact) as ar:
        with GpuSG(pr, coarse="amg", ras_path="sweep") as g:
            x, _ = g.solve(pr.restart, 1e-10)
            torch.cuda.synchronize()
            assert ar.used() == need
        assert torch.equal(x, x_ref)
    small = torch.empty(need - 4096, dtype=torch.uint8, device="cuda")
    with B.Arena(small):
        with pytest.raises(B.SgError) as e:
            g = GpuSG(pr, coarse="amg", ras_path="sweep")
            g.solve(pr.restart, 1e-10)
        code, msg = e.value.code, str(e.value)
        del e
    assert code == SG_ERR_WORKSPACE and "arena exhausted" in msg
    gc.collect()
    assert B.memory_stats()[0] == live0


def test_arena_reset_refuses_while_handles_live():
    _cuda()
    pr = make_problem("c0", nc=12, sub=(2, 2))
    buf = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
    with B.Arena(buf) as ar:
        g = GpuSG(pr, coarse="mean", ras_path="sweep")
        with pytest.raises(B.SgError, match="live buffers"):
            ar.reset()
        g.close()
        ar.reset()
        assert ar.used() == 0


def test_allocator_needs_both_functions():
    _cuda()
    fn = B._ALLOC_FN(lambda n, d, c: None)
    assert B.lib().sg_set_allocator(B.C.cast(fn, B._vp), None, None) == -1
    assert B.lib().sg_set_allocator(None, None, None) == 0
    np.testing.assert_equal(B.memory_stats()[2], 0)
