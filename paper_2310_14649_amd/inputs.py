"""Seeded synthetic inputs shared by the HIP path and by the CPU oracle.

This module holds no arithmetic of the solver itself: it only describes the
problem instances of the paper's experiments (Sec. 4): the unit-square mesh,
the Karhunen-Loeve (KL) modes of the underlying Gaussian field (Eq. KLE),
and a partition of the interior nodes into subdomains.  Everything the
stochastic Galerkin method computes from these arrays (log-normal PCE
coefficients, stiffness matrices, Schwarz operators, Krylov iterates) is
implemented twice, independently: in HIP in ``csrc/`` and in plain NumPy in
the oracle.

Conventions
-----------
* Structured mesh: ``nc`` x ``nc`` squares on [0,1]^2, each cut along the
  "/" diagonal into the counter-clockwise triangles
  (v(i,j), v(i+1,j), v(i+1,j+1)) and (v(i,j), v(i+1,j+1), v(i,j+1)), with
  vertex id v(i,j) = j*(nc+1)+i.
* Unknowns are interior vertices only (zero Dirichlet data eliminated);
  interior vertex (i,j) has dof (j-1)*(nc-1)+(i-1), x fastest.  Boundary
  vertices carry dof -1.
* KL field: squared-exponential covariance sigma^2 exp(-|x-y|^2/(2 l^2)),
  separable, so its 2D eigenpairs are products of 1D eigenpairs on [0,1].
  The 1D operator is discretised by Nystrom quadrature on Gauss-Legendre
  nodes; eigenfunctions are normalised to unit L2 norm and signed positive
  at the smallest node.  2D modes (a,b) (a = x-index) are ordered by the key
  (-lambda_a*lambda_b, a, b); g_m = sigma*sqrt(lambda_a lambda_b)
  phi_a(x) phi_b(y).  The field mean g_0 is zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
@dataclass
class Mesh:
    nc: int                       # cells per side
    xy: np.ndarray                # [n_vert, 2] float64
    tri: np.ndarray               # [n_tri, 3] int32, counter-clockwise
    dof: np.ndarray               # [n_vert] int32, -1 on the Dirichlet boundary
    n: int                        # number of unknowns (interior vertices)
    jittered: bool = False

    @property
    def n_vert(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    def centroids(self) -> np.ndarray:
        return self.xy[self.tri].mean(axis=1)

    def interior_xy(self) -> np.ndarray:
        """Coordinates of the unknowns, in dof order."""
        out = np.empty((self.n, 2))
        m = self.dof >= 0
        out[self.dof[m]] = self.xy[m]
        return out


def _structured_topology(nc: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    i, j = np.meshgrid(np.arange(nc + 1), np.arange(nc + 1), indexing="xy")
    xy = np.stack([i.ravel() / nc, j.ravel() / nc], axis=1).astype(np.float64)

    def v(ii, jj):
        return jj * (nc + 1) + ii

    ci, cj = np.meshgrid(np.arange(nc), np.arange(nc), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    t1 = np.stack([v(ci, cj), v(ci + 1, cj), v(ci + 1, cj + 1)], axis=1)
    t2 = np.stack([v(ci, cj), v(ci + 1, cj + 1), v(ci, cj + 1)], axis=1)
    tri = np.empty((2 * nc * nc, 3), dtype=np.int32)
    tri[0::2] = t1
    tri[1::2] = t2
    vi = np.arange((nc + 1) ** 2) % (nc + 1)
    vj = np.arange((nc + 1) ** 2) // (nc + 1)
    interior = (vi > 0) & (vi < nc) & (vj > 0) & (vj < nc)
    dof = np.full((nc + 1) ** 2, -1, dtype=np.int32)
    dof[interior] = (vj[interior] - 1) * (nc - 1) + (vi[interior] - 1)
    return xy, tri, dof


def structured_mesh(nc: int) -> Mesh:
    xy, tri, dof = _structured_topology(nc)
    return Mesh(nc=nc, xy=xy, tri=tri, dof=dof, n=(nc - 1) ** 2)


def _signed_areas(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    p0, p1, p2 = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    return 0.5 * ((p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1])
                  - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1]))


def jittered_mesh(nc: int, amp: float = 0.3, seed: int = 0,
                  min_area_frac: float = 0.1, max_rounds: int = 50) -> Mesh:
    """Structured topology with interior vertices moved by U(-amp*h, amp*h)
    per coordinate.  Every interior vertex of an element whose area falls
    below ``min_area_frac * h^2/2`` is redrawn from the same generator
    stream until no such element remains."""
    xy, tri, dof = _structured_topology(nc)
    h = 1.0 / nc
    rng = np.random.default_rng(seed)
    interior = dof >= 0
    idx = np.nonzero(interior)[0]
    base = xy.copy()
    xy = base.copy()
    xy[idx] += rng.uniform(-amp * h, amp * h, size=(idx.size, 2))
    thresh = min_area_frac * h * h / 2.0
    for _ in range(max_rounds):
        bad = _signed_areas(xy, tri) < thresh
        if not bad.any():
            break
        verts = np.unique(tri[bad].ravel())
        verts = verts[interior[verts]]
        xy[verts] = base[verts] + rng.uniform(-amp * h, amp * h, size=(verts.size, 2))
    else:  # pragma: no cover - never observed for amp <= 0.3
        raise RuntimeError("jittered_mesh: could not repair inverted elements")
    return Mesh(nc=nc, xy=xy, tri=tri, dof=dof, n=(nc - 1) ** 2, jittered=True)


def mesh_graph(mesh: Mesh) -> List[np.ndarray]:
    """Adjacency lists (sorted) between unknowns along triangle edges."""
    d = mesh.dof[mesh.tri]
    rows, cols = [], []
    for a, b in ((0, 1), (1, 2), (0, 2)):
        m = (d[:, a] >= 0) & (d[:, b] >= 0)
        rows.append(d[m, a]); cols.append(d[m, b])
        rows.append(d[m, b]); cols.append(d[m, a])
    r = np.concatenate(rows); c = np.concatenate(cols)
    key = np.unique(r.astype(np.int64) * mesh.n + c)
    r = (key // mesh.n).astype(np.int64); c = (key % mesh.n).astype(np.int32)
    ptr = np.searchsorted(r, np.arange(mesh.n + 1))
    return [c[ptr[a]:ptr[a + 1]] for a in range(mesh.n)]


def mesh_graph_csr(mesh: Mesh) -> Tuple[np.ndarray, np.ndarray]:
    d = mesh.dof[mesh.tri]
    rows, cols = [], []
    for a, b in ((0, 1), (1, 2), (0, 2)):
        m = (d[:, a] >= 0) & (d[:, b] >= 0)
        rows.append(d[m, a]); cols.append(d[m, b])
        rows.append(d[m, b]); cols.append(d[m, a])
    r = np.concatenate(rows).astype(np.int64); c = np.concatenate(cols).astype(np.int64)
    key = np.unique(r * mesh.n + c)
    r = key // mesh.n; c = (key % mesh.n).astype(np.int32)
    ptr = np.searchsorted(r, np.arange(mesh.n + 1)).astype(np.int64)
    return ptr, c


# --------------------------------------------------------------------------
# KL modes of the Gaussian field
# --------------------------------------------------------------------------
@dataclass
class KL1D:
    ell: float
    nodes: np.ndarray      # [nq]
    weights: np.ndarray    # [nq]
    lam: np.ndarray        # [K] descending
    vec: np.ndarray        # [nq, K] eigenfunction values at the nodes

    def eval(self, x: np.ndarray, k: int) -> np.ndarray:
        """Nystrom interpolation of the k-th (0-based) eigenfunction."""
        x = np.asarray(x, dtype=np.float64)
        ker = np.exp(-((x[..., None] - self.nodes) ** 2) / (2.0 * self.ell ** 2))
        return ker @ (self.weights * self.vec[:, k]) / self.lam[k]


def kl_1d(ell: float, nq: int = 256, keep: int = 16) -> KL1D:
    t, w = np.polynomial.legendre.leggauss(nq)
    x = 0.5 * (t + 1.0)
    w = 0.5 * w
    ker = np.exp(-((x[:, None] - x[None, :]) ** 2) / (2.0 * ell ** 2))
    sw = np.sqrt(w)
    lam, u = np.linalg.eigh(sw[:, None] * ker * sw[None, :])
    order = np.argsort(-lam)[:keep]
    lam = lam[order]
    vec = u[:, order] / sw[:, None]
    sgn = np.sign(vec[0, :])
    sgn[sgn == 0] = 1.0
    vec = vec * sgn
    return KL1D(ell=ell, nodes=x, weights=w, lam=lam, vec=vec)


def kl_mode_pairs(kl: KL1D, M: int) -> List[Tuple[int, int]]:
    """1-based (a, b) pairs of the first M 2D modes."""
    K = kl.lam.size
    cand = [(-(kl.lam[a - 1] * kl.lam[b - 1]), a, b)
            for a in range(1, K + 1) for b in range(1, K + 1)]
    cand.sort()
    return [(a, b) for _, a, b in cand[:M]]


def _eval_unique(kl: KL1D, x: np.ndarray, k: int) -> np.ndarray:
    u, inv = np.unique(x, return_inverse=True)
    return kl.eval(u, k)[inv]


def kl_fields(points: np.ndarray, M: int, sigma: float, ell: float,
              nq: int = 256) -> Tuple[np.ndarray, List[Tuple[int, int]], np.ndarray]:
    """g_m at ``points`` ([N,2]) -> ([M, N] array, mode pairs, eigenvalues)."""
    kl = kl_1d(ell, nq=nq)
    pairs = kl_mode_pairs(kl, M)
    g = np.empty((M, points.shape[0]))
    lam2 = np.empty(M)
    for m, (a, b) in enumerate(pairs):
        lam2[m] = kl.lam[a - 1] * kl.lam[b - 1]
        g[m] = sigma * np.sqrt(lam2[m]) * _eval_unique(kl, points[:, 0], a - 1) \
            * _eval_unique(kl, points[:, 1], b - 1)
    return g, pairs, lam2


# --------------------------------------------------------------------------
# partitions
# --------------------------------------------------------------------------
def structured_partition(nc: int, sx: int, sy: int) -> np.ndarray:
    """Owner (subdomain id by*sx+bx) of every unknown: each axis of the
    (nc-1) interior indices is split like ``numpy.array_split``."""
    m = nc - 1
    bx = np.concatenate([np.full(len(c), k) for k, c in enumerate(np.array_split(np.arange(m), sx))])
    by = np.concatenate([np.full(len(c), k) for k, c in enumerate(np.array_split(np.arange(m), sy))])
    owner = (by[:, None] * sx + bx[None, :]).astype(np.int32)
    return owner.ravel()


def graph_partition(mesh: Mesh, nx: int, ny: int, seed: int,
                    lo: int, hi: int, max_tries: int = 64) -> Tuple[np.ndarray, int]:
    """Multi-source BFS partition: nx*ny centres on a lattice, each moved by
    U(-0.45, 0.45) lattice cells; every unknown joins the centre reached
    first (ties -> lower centre id).  The seed is increased by one until
    every part owns between ``lo`` and ``hi`` nodes.  Returns (owner, seed)."""
    ptr, col = mesh_graph_csr(mesh)
    pts = mesh.interior_xy()
    n = mesh.n
    for s in range(seed, seed + max_tries):
        rng = np.random.default_rng(s)
        cx = (np.arange(nx)[None, :] + 0.5 + rng.uniform(-0.45, 0.45, size=(ny, nx))) / nx
        cy = (np.arange(ny)[:, None] + 0.5 + rng.uniform(-0.45, 0.45, size=(ny, nx))) / ny
        centres = np.stack([cx.ravel(), cy.ravel()], axis=1)
        # nearest unknown to each centre
        seeds = np.empty(len(centres), dtype=np.int64)
        for c, p in enumerate(centres):
            seeds[c] = int(np.argmin(((pts - p) ** 2).sum(axis=1)))
        if len(np.unique(seeds)) != len(seeds):
            continue
        owner = np.full(n, -1, dtype=np.int32)
        owner[seeds] = np.arange(len(seeds), dtype=np.int32)
        frontier = np.sort(seeds)
        while frontier.size:
            # all edges leaving the frontier, with the owner of their source
            deg = ptr[frontier + 1] - ptr[frontier]
            src = np.repeat(frontier, deg)
            start = np.repeat(ptr[frontier] - np.cumsum(np.concatenate([[0], deg[:-1]])), deg)
            cn = col[np.arange(src.size) + start]
            keep = owner[cn] < 0
            cn = cn[keep]
            co = owner[src[keep]]
            if cn.size == 0:
                break
            order = np.lexsort((co, cn))
            cn, co = cn[order], co[order]
            first = np.ones(cn.size, dtype=bool)
            first[1:] = cn[1:] != cn[:-1]
            owner[cn[first]] = co[first]
            frontier = np.unique(cn[first])
        if (owner < 0).any():
            continue
        counts = np.bincount(owner, minlength=len(seeds))
        if counts.min() >= lo and counts.max() <= hi:
            return owner, s
    raise RuntimeError("graph_partition: no admissible seed found")


# --------------------------------------------------------------------------
# the experiment configurations
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    mesh: Mesh
    M: int
    p_in: int
    p: int
    sigma: float
    ell: float
    g0: np.ndarray                # [n_tri] mean of the Gaussian field at centroids
    g: np.ndarray                 # [M, n_tri] KL modes at centroids
    owner: np.ndarray             # [n] subdomain of every unknown
    n_sub: int
    overlap: int
    restart: int
    rtol: float
    extra: Dict = field(default_factory=dict)


CONFIGS = {
    # name: (nc, M, p, sigma, ell, (sx, sy) or 'graph', overlap, restart)
    "c0": dict(nc=32, M=2, p=2, sigma=0.3, ell=0.5, sub=(2, 2), overlap=1, restart=30),
    "c1": dict(nc=512, M=4, p=3, sigma=0.5, ell=0.2, sub=(16, 16), overlap=2, restart=50),
    "c3": dict(nc=384, M=6, p=3, sigma=0.5, ell=0.2, sub="graph", overlap=2, restart=50,
               jitter=0.3, graph=(16, 12, 300, 1200)),
    "c4": dict(nc=128, M=4, p=3, sigma=0.5, ell=0.2, sub=(8, 8), overlap=2, restart=50),
    # jittered mesh with lattice subdomains (reduced test instances)
    "jit": dict(nc=26, M=4, p=3, sigma=0.5, ell=0.2, sub=(3, 3), overlap=2, restart=50,
                jitter=0.3),
}


def make_problem(name: str = "c0", nc: Optional[int] = None, M: Optional[int] = None,
                 p: Optional[int] = None, sigma: Optional[float] = None,
                 ell: Optional[float] = None, sub=None, overlap: Optional[int] = None,
                 restart: Optional[int] = None, seed: int = 0, p_in: int = 2,
                 rtol: float = 1e-8) -> Problem:
    """A configuration by name, any field optionally overridden (used to
    build reduced-size instances with the same structure)."""
    base = dict(CONFIGS[name])
    for k, v in dict(nc=nc, M=M, p=p, sigma=sigma, ell=ell, sub=sub,
                     overlap=overlap, restart=restart).items():
        if v is not None:
            base[k] = v
    if base.get("jitter"):
        mesh = jittered_mesh(base["nc"], amp=base["jitter"], seed=seed)
    else:
        mesh = structured_mesh(base["nc"])
    cen = mesh.centroids()
    Mv = base["M"]
    if Mv > 0:
        g, pairs, lam2 = kl_fields(cen, Mv, base["sigma"], base["ell"])
    else:
        g, pairs, lam2 = np.zeros((0, mesh.n_tri)), [], np.zeros(0)
    extra = dict(pairs=pairs, lam2=lam2)
    if base["sub"] == "graph":
        gx, gy, lo, hi = base["graph"]
        owner, used = graph_partition(mesh, gx, gy, seed, lo, hi)
        n_sub = gx * gy
        extra["partition_seed"] = used
    else:
        sx, sy = base["sub"]
        owner = structured_partition(base["nc"], sx, sy)
        n_sub = sx * sy
    return Problem(name=name, mesh=mesh, M=Mv, p_in=min(p_in, base["p"]) if Mv > 0 else 0,
                   p=base["p"] if Mv > 0 else 0, sigma=base["sigma"], ell=base["ell"],
                   g0=np.zeros(mesh.n_tri), g=g, owner=owner, n_sub=n_sub,
                   overlap=base["overlap"], restart=base["restart"], rtol=rtol, extra=extra)
