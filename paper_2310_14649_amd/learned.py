"""Learned initial guess for the nonlinear SG problem: a small convolutional
network maps the input fields of a draw (the mean-coefficient factor and the
KL mode fields at the interior vertices) to the chaos coefficient fields of
the solution, and ``newton_guess`` turns its prediction into a Newton
starting point (never worse than the zero guess).

The training data are solutions the method itself computes (``newton_solve``
on draws of the correlation length and standard deviation); training and
inference run in the library's kernels (``nn_*``).  This module only
draws the inputs, moves buffers and sequences the calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import binding as B
from .inputs import kl_fields, make_problem
from .solver import GpuNewton, GpuSG

CHANNELS = [5, 64, 64, 64, 35]


def draw_params(n: int, seed: int, ell=(0.1, 0.5), sigma=(0.2, 0.6)):
    """n draws of (sigma, ell), uniform on the given ranges."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        e = rng.uniform(*ell)
        s = rng.uniform(*sigma)
        out.append((s, e))
    return out


def vertex_modes(mesh, M: int, sigma: float, ell: float) -> np.ndarray:
    """[M, npts]: the KL mode fields g_1..g_M of a draw at the interior
    vertices (dof order = y-major, x fastest); the generator's part of the
    network input (the library forms the input channels from them)."""
    g, _, _ = kl_fields(mesh.interior_xy(), M, sigma, ell)
    return np.ascontiguousarray(g)


def init_params(channels: List[int], seed: int) -> np.ndarray:
    """He-normal weights, zero biases, flattened W_1, b_1, W_2, ... (the
    layout nn_set_params expects)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in zip(channels[:-1], channels[1:]):
        parts.append(rng.standard_normal(9 * ci * co) * np.sqrt(2.0 / (9 * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


@dataclass
class Dataset:
    X: object                 # torch FP64 [N, H, W, 5] on the device
    T: object                 # torch FP64 [N, H, W, P] on the device
    draws: list
    newton_steps: List[int] = field(default_factory=list)
    krylov_its: List[int] = field(default_factory=list)
    seconds: float = 0.0


class LearnedGuess:
    """Owns the solver for one mesh/basis, the network and its output map."""

    def __init__(self, name: str = "c4", nc: Optional[int] = None, max_batch: int = 16,
                 channels: Optional[List[int]] = None, seed: int = 0, prec: str = "fp64",
                 ortho: str = "mgs", ras_path: str = "sweep"):
        import torch
        self.torch = torch
        self.name = name
        self.nc = nc
        self.base = make_problem(name, nc=nc)
        self.mesh = self.base.mesh
        self.M, self.P = self.base.M, None
        self.H = self.W = self.mesh.nc - 1
        self.solver = GpuNewton(self.base, prec=prec, ortho=ortho, ras_path=ras_path)
        self.P = self.solver.P
        self.channels = list(channels or [1 + self.M, 64, 64, 64, self.P])
        assert self.channels[0] == 1 + self.M and self.channels[-1] == self.P
        self.max_batch = max_batch
        self.nn = B.nn_create(self.channels, self.H, self.W, max_batch)
        B.nn_set_params(self.nn, init_params(self.channels, seed))
        self.shape = self._envelope()
        self.have_map = False
        self.g0v = torch.zeros(self.H * self.W, dtype=torch.float64, device="cuda")
        self.gv = torch.empty((self.M, self.H * self.W), dtype=torch.float64, device="cuda")
        self.guess_ws = torch.empty((B.newton_guess_workspace_bytes(self.solver.nl) + 7) // 8,
                                    dtype=torch.float64, device="cuda")

    def _envelope(self):
        """Solution of the deterministic problem with unit coefficient (P = 1)
        on the device: the shape every chaos mode vanishes with at the
        Dirichlet boundary (nn_fit_output_map normalises it)."""
        det = make_problem(self.name, nc=self.nc, M=0)
        with GpuSG(det, coarse="mean") as g:
            x, info = g.solve(det.restart, 1e-10)
            assert info["converged"]
        return x

    def set_draw(self, sigma: float, ell: float):
        """The draw's coefficient fields into the nonlinear problem and its KL
        modes at the vertices onto the device (generator work, outside any
        timed region)."""
        pr = make_problem(self.name, nc=self.nc, sigma=sigma, ell=ell)
        B.sg_nl_set_coefficients(self.solver.nl, pr.g0, pr.g)
        self.gv.copy_(self.torch.from_numpy(vertex_modes(self.mesh, self.M, sigma, ell)))
        return pr

    def features(self, X):
        """The network input of the current draw into X (device [H, W, 1+M])."""
        B.nn_input_fields(self.H * self.W, self.M, self.g0v, self.gv, X)

    def generate(self, draws, tol: float = 1e-10) -> Dataset:
        torch = self.torch
        N = len(draws)
        X = torch.empty((N, self.H, self.W, 1 + self.M), dtype=torch.float64, device="cuda")
        T = torch.empty((N, self.H, self.W, self.P), dtype=torch.float64, device="cuda")
        ds = Dataset(X=X, T=T, draws=list(draws))
        t0 = time.perf_counter()
        for i, (s, e) in enumerate(draws):
            self.set_draw(s, e)
            self.features(X[i])
            U, info = self.solver.solve(tol=tol)
            if not info["converged"]:
                raise RuntimeError(f"training solve {i} did not converge: {info}")
            T[i].copy_(U.view(self.H, self.W, self.P))
            ds.newton_steps.append(info["steps"])
            ds.krylov_its.append(info["krylov_its"])
        torch.cuda.synchronize()
        ds.seconds = time.perf_counter() - t0
        return ds

    def fit_output_scale(self, ds: Dataset, n_samples: int = 32):
        """The output map from the first n_samples training targets
        (nn_fit_output_map: envelope normalised to one, per-mode RMS scale)."""
        nb = min(n_samples, ds.T.shape[0])
        B.nn_fit_output_map(self.nn, self.shape, ds.T[:nb], nb)
        self.have_map = True

    def train(self, ds: Dataset, steps: int, batch: int = 16, lr: float = 1e-3,
              lr_final: float = 1e-5, log_every: int = 0):
        """Adam on consecutive mini-batches of the (i.i.d.) draws, learning
        rate decayed geometrically from lr to lr_final."""
        if not self.have_map:
            self.fit_output_scale(ds)
        N = ds.X.shape[0]
        batch = min(batch, self.max_batch, N)
        losses = []
        t0 = time.perf_counter()
        for it in range(steps):
            b0 = (it * batch) % max(N - batch + 1, 1)
            rate = lr * (lr_final / lr) ** (it / max(steps - 1, 1))
            loss = B.nn_loss_grad(self.nn, ds.X[b0:b0 + batch], ds.T[b0:b0 + batch], batch)
            B.nn_adam_step(self.nn, rate)
            losses.append(loss)
            if log_every and (it % log_every == 0 or it == steps - 1):
                print(f"[learned] step {it} loss {loss:.4e} lr {rate:.2e}", flush=True)
        self.torch.cuda.synchronize()
        return losses, time.perf_counter() - t0

    def predict(self, X):
        """X [B,H,W,5] device -> U [B, H*W*P] device FP64."""
        Bn = X.shape[0]
        U = self.torch.empty((Bn, self.H * self.W * self.P), dtype=self.torch.float64,
                             device="cuda")
        B.nn_forward(self.nn, X, Bn, U)
        return U

    def solve(self, sigma: float, ell: float, use_nn: bool, tol: float = 1e-8):
        """Newton for one draw from the zero guess or from the guess
        newton_guess makes of the network's prediction (never a larger
        residual than the zero guess).  The draw's fields are generated
        before the clock starts, for both arms; the time of the learned arm
        includes the network's input channels, inference and the guess."""
        torch = self.torch
        self.set_draw(sigma, ell)
        X = torch.empty((1, self.H, self.W, 1 + self.M), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U0 = None
        choice, rel = 0, None
        if use_nn:
            self.features(X[0])
            Up = self.predict(X)[0]
            U0 = torch.empty_like(Up)
            choice, rel = B.newton_guess(self.solver.nl, Up, U0, self.guess_ws)
        U, info = self.solver.solve(U0=U0, tol=tol)
        torch.cuda.synchronize()
        info["seconds"] = time.perf_counter() - t0
        info["guess_choice"] = choice
        info["guess_relres"] = None if rel is None else rel.tolist()
        return U, info

    def close(self):
        if self.nn is not None:
            B.nn_destroy(self.nn)
            self.nn = None
        self.solver.close()
