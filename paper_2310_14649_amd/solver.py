"""Handle lifetimes for one SG problem on the GPU.

``GpuSG`` only sequences C-ABI calls (basis -> operator -> RAS -> coarse
solver -> FGMRES) and owns the torch buffers they write into; all
arithmetic happens in ``libsgsolve.so``.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import binding as B
from .inputs import Problem, structured_partition

COARSE = {"none": B.SG_COARSE_NONE, "mean": B.SG_COARSE_MEAN_EXACT, "amg": B.SG_COARSE_AMG}


class Geometric:
    """Parameters of the geometric coarse space (amg_setup_geometric): the
    fine:coarse cell ratio, the coarse lattice's subdomains (sx, sy) and
    overlap, the coarse level's own coarse correction ("none", "mean" or
    "amg"), and the inner FGMRES tolerance and step limit."""

    def __init__(self, ratio: int, sub=None, overlap: int = 1, level_coarse: str = "mean",
                 rtol: float = 1e-5, max_its: int = 100, nodes_per_side: int = 16):
        self.ratio, self.overlap = ratio, overlap
        self.sub = None if sub is None else tuple(sub)
        self.nodes_per_side = nodes_per_side
        self.level_coarse, self.rtol, self.max_its = level_coarse, rtol, max_its

    def owner(self, nc: int):
        """Lattice partition of the coarse unknowns: `sub`, or (default)
        subdomains of about nodes_per_side x nodes_per_side coarse nodes."""
        Nc = nc // self.ratio
        if self.sub is None:
            k = max(1, round((Nc - 1) / self.nodes_per_side))
            sx = sy = k
        else:
            sx, sy = self.sub
        sx, sy = min(sx, Nc - 1), min(sy, Nc - 1)
        return structured_partition(Nc, sx, sy), sx * sy


class GpuSG:
    """local: the subdomain solves, "mean" (K_0 (x) G_0) or "kron" (K_0 (x) Gt).
    matrix_free: apply the operator with sg_matvec_matrix_free (lattice meshes).
    ras_path: "sweep", "dense", "dense32", "fused", or "auto" (timed by the library,
    also choosing the staged matvec's work-group shape).  tune_cache: with
    "auto", a ``TuneCache`` (or its file path) that supplies choices already
    made for this shape and records new ones.  coarse: "none", "mean", "amg"
    (Nicolaides coarse space) or a ``Geometric`` (coarser lattice)."""

    def __init__(self, pr: Problem, prec: str = "fp64", coarse: str = "amg",
                 overlap: Optional[int] = None, owner: Optional[np.ndarray] = None,
                 n_sub: Optional[int] = None, stream=None, ras_path: str = "sweep",
                 tune_cache=None, local: str = "mean", matrix_free: bool = False):
        import torch
        self.torch = torch
        self.pr = pr
        self.stream = stream
        self.basis = self.op = self.ras = self.amg = None
        m = pr.mesh
        self.basis = B.sg_build_triples(pr.M, pr.p_in, pr.p)
        self.op = B.sg_assemble(self.basis, m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, stream=stream)
        self.n, self.P, self.L, self.nnz = B.sg_op_info(self.op)
        if matrix_free:
            B.sg_matvec_matrix_free(self.op, True, stream=stream)
        dev = torch.device("cuda")
        self.b = torch.empty(self.n * self.P, dtype=torch.float64, device=dev)
        B.sg_op_rhs(self.op, self.b, stream=stream)
        self.owner = pr.owner if owner is None else owner
        self.n_sub = pr.n_sub if n_sub is None else n_sub
        self.overlap = pr.overlap if overlap is None else overlap
        self.prec = prec
        self.coarse = coarse
        self.ras = B.ras_setup(self.op, self.owner, self.n_sub, self.overlap, B.PREC[prec],
                               stream=stream)
        if local != "mean":
            B.ras_set_local(self.ras, self.op, local, stream=stream)
        self.ras_ms = None
        self.mv_ms = None
        self.tuned_from_cache = False
        if ras_path in ("dense", "dense32", "fused"):
            B.ras_select(self.ras, ras_path, stream=stream)
        elif ras_path == "auto":
            self._autotune(tune_cache, stream)
        elif ras_path != "sweep":
            raise ValueError(f"unknown RAS path {ras_path!r}")
        if isinstance(coarse, Geometric):
            owner_c, nsub_c = coarse.owner(m.nc)
            self.amg = B.amg_setup_geometric(self.op, coarse.ratio, owner_c, nsub_c,
                                             coarse.overlap, COARSE[coarse.level_coarse],
                                             B.PREC[prec], coarse.rtol, coarse.max_its,
                                             stream=stream)
        elif coarse != "none":
            self.amg = B.amg_setup(self.op, self.ras, COARSE[coarse], B.PREC[prec], stream=stream)
        self._ws = None
        self._ws_restart = None

    def new_vec(self, fill: float = 0.0):
        return self.torch.full((self.n * self.P,), fill, dtype=self.torch.float64, device="cuda")

    def workspace(self, restart: int):
        if self._ws is None or self._ws_restart != restart:
            nbytes = B.fgmres_workspace_bytes(self.op, self.amg, restart)
            self._ws = self.torch.empty((nbytes + 7) // 8, dtype=self.torch.float64, device="cuda")
            self._ws_restart = restart
        return self._ws

    def precond_workspace(self):
        nbytes = max(B.sg_precond_workspace_bytes(self.op, self.amg), 8)
        return self.torch.empty((nbytes + 7) // 8, dtype=self.torch.float64, device="cuda")

    def damping(self, its: int = 15):
        N = self.n * self.P
        ws = self.torch.empty(2 * N + 4096, dtype=self.torch.float64, device="cuda")
        return B.sg_smoother_damping(self.op, self.ras, its, ws, stream=self.stream)

    def _autotune(self, tune_cache, stream):
        from .autotune import TuneCache, make_key
        cache = TuneCache(tune_cache) if isinstance(tune_cache, str) else tune_cache
        arch = self.torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        pr = self.pr
        shape = dict(n=self.n, P=self.P, L=self.L, nnz=self.nnz, M=pr.M, p=pr.p)
        staged = B.sg_matvec_kernel(self.op) == "staged"
        kmv = make_key("sg_matvec", arch, **shape)
        kras = make_key("ras_apply", arch, prec=self.prec, n_sub=self.n_sub,
                        overlap=self.overlap, **shape)
        hit_mv = cache.get(kmv) if cache is not None else None
        hit_ras = cache.get(kras) if cache is not None else None
        if staged:
            if hit_mv is not None:
                B.sg_matvec_select(self.op, int(hit_mv["tiles"]))
            else:
                self.mv_ms = B.sg_matvec_autotune(self.op, 10, stream=stream)
                if cache is not None:
                    cache.put(kmv, dict(tiles=B.sg_matvec_tiles(self.op), ms=self.mv_ms))
        if hit_ras is not None:
            B.ras_select(self.ras, hit_ras["path"], stream=stream)
        else:
            self.ras_ms = B.ras_autotune(self.ras, 5, stream=stream)
            if cache is not None:
                cache.put(kras, dict(path=B.ras_path_info(self.ras)[2], ms=list(self.ras_ms)))
        self.tuned_from_cache = hit_ras is not None and (hit_mv is not None or not staged)

    def set_inner(self, inner: str = "none", rtol: float = 1e-5, max_its: int = 100):
        """The coarse solve of the two-grid cycle: one V-cycle ("none"), or an
        inner GMRES preconditioned by a V-cycle ("gmres_amg", the paper's 2GV3)
        or by block Jacobi ("gmres_bj", 2GV2)."""
        B.amg_set_inner(self.amg, inner, rtol, max_its)

    def solve(self, restart: int, rtol: float, max_it: int = 2000, omega: float = 0.0,
              x0=None, use_precond: bool = True, use_graph: bool = False, ortho: str = "mgs"):
        x = self.new_vec() if x0 is None else x0.clone()
        ras = self.ras if use_precond else None
        amg = self.amg if use_precond else None
        ws = self.workspace(restart) if use_precond else self.torch.empty(
            (B.fgmres_workspace_bytes(self.op, None, restart) + 7) // 8, dtype=self.torch.float64,
            device="cuda")
        info = B.fgmres_solve(self.op, ras, amg, self.b, x, restart, max_it, rtol, omega, ws,
                              use_graph=use_graph, ortho=ortho, stream=self.stream)
        return x, info

    def close(self):
        if self.amg is not None:
            B.sg_destroy_amg(self.amg)
            self.amg = None
        if self.ras is not None:
            B.sg_destroy_ras(self.ras)
            self.ras = None
        if self.op is not None:
            B.sg_destroy_op(self.op)
            self.op = None
        if self.basis is not None:
            B.sg_destroy_basis(self.basis)
            self.basis = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GpuNewton:
    """Nonlinear SG problem (kappa(u) = 1 + a1 u + a2 u^2) on the GPU: sequences
    ``sg_nl_setup`` / ``sg_nl_eval`` / ``newton_solve`` and owns the buffers."""

    def __init__(self, pr: Problem, a2: float = 0.5, prec: str = "fp64", coarse: str = "amg",
                 overlap: Optional[int] = None, owner: Optional[np.ndarray] = None,
                 n_sub: Optional[int] = None, stream=None, a1: float = 0.0,
                 ortho: str = "mgs", ras_path: str = "sweep"):
        import torch
        self.torch = torch
        self.pr = pr
        self.stream = stream
        self.ortho = ortho
        self.ras_path = ras_path         # default of solve(): see binding.newton_solve
        self.basis = self.nl = None
        m = pr.mesh
        self.basis = B.sg_build_triples(pr.M, pr.p_in, pr.p)
        self.nl = B.sg_nl_setup(self.basis, m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, a2, a1=a1,
                                stream=stream)
        self.n, self.P, self.L2, self.nnz = B.sg_nl_info(self.nl)
        self.owner = pr.owner if owner is None else owner
        self.n_sub = pr.n_sub if n_sub is None else n_sub
        self.overlap = pr.overlap if overlap is None else overlap
        self.prec = prec
        self.coarse = coarse
        self._ws = None
        self._ws_restart = None

    def new_vec(self, fill: float = 0.0):
        return self.torch.full((self.n * self.P,), fill, dtype=self.torch.float64, device="cuda")

    def residual(self, U):
        """R(U) = F e_0 - A(U); also leaves K1 and the Jacobian assembled at U."""
        R = self.new_vec()
        B.sg_nl_eval(self.nl, U, R, stream=self.stream)
        return R

    def jac_apply(self, X):
        Y = self.new_vec()
        B.sg_nl_jac_apply(self.nl, X, Y, stream=self.stream)
        return Y

    def workspace(self, restart: int):
        if self._ws is None or self._ws_restart != restart:
            nbytes = B.newton_workspace_bytes(self.nl, self.n_sub, COARSE[self.coarse], restart)
            self._ws = self.torch.empty((nbytes + 7) // 8, dtype=self.torch.float64, device="cuda")
            self._ws_restart = restart
        return self._ws

    def solve(self, U0=None, tol: float = 1e-8, max_steps: int = 30, restart: Optional[int] = None,
              max_it: int = 1000, eta_max: float = 1e-2, omega: float = 0.0,
              use_graph: bool = False, amg_rebuild: int = 0, method: str = "newton",
              du_tol: float = 0.0, ras_path: Optional[str] = None):
        restart = self.pr.restart if restart is None else restart
        ras_path = self.ras_path if ras_path is None else ras_path
        U = self.new_vec() if U0 is None else U0.clone()
        info = B.newton_solve(self.nl, self.owner, self.n_sub, self.overlap, B.PREC[self.prec],
                              COARSE[self.coarse], U, self.workspace(restart), max_steps=max_steps,
                              tol=tol, eta_max=eta_max, restart=restart, max_it=max_it,
                              omega=omega, use_graph=use_graph, amg_rebuild=amg_rebuild,
                              method=method, du_tol=du_tol, ortho=self.ortho,
                              ras_path=ras_path, stream=self.stream)
        return U, info

    def close(self):
        if self.nl is not None:
            B.sg_destroy_nl(self.nl)
            self.nl = None
        if self.basis is not None:
            B.sg_destroy_basis(self.basis)
            self.basis = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
