#!/usr/bin/env python3
"""Benchmark of the stochastic Galerkin hot path on one MI355X.

Workload: the linear SG Poisson problem on a 512 x 512 P1 grid (261,121
interior nodes), log-normal coefficient with M = 4 KL variables, output
order 3 (P = 35, 9,139,235 unknowns), restricted additive Schwarz on 16 x 16
subdomains with overlap 2 and a smoothed-aggregation AMG coarse solve on
the Nicolaides space, flexible GMRES(50) to a true relative residual of
1e-8 from a zero initial guess.

One timed step = one complete FGMRES solve (preconditioner application,
SG matvecs, Gram-Schmidt, Givens, true residual) with the preconditioner's
local solves and smoothing in the mixed precision (BF16 by default, FP32
also timed); the same solve with an all-FP64 preconditioner is timed beside
it.  Each precision's RAS apply path (factored sweeps or dense inverse rows)
is picked by the autotuner at setup.  Setup (assembly,
factorisations, AMG hierarchy) is outside the timed region, as in the
paper's split between PC setup and KSP solve.

Also measured: the SG matvec (the kernel the metric names) with HIP events
around each launch, the Infinity Cache flushed between launches, against
its algorithmic bytes; and the CPU oracle on the host's cores over a
bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the matvec kernel measured with the FETCH_SIZE and
# WRITE_SIZE counters, scaled by the counters' reading of a copy of known
# size (profiles/sg_matvec_512x512_P35_hbm_traffic.txt), keyed by kernel and
# workload; a workload or kernel without a measurement reports null.
MEASURED_TRAFFIC = {("kron_matvec_split_kernel<4, 2, 3, 5, 1>", 261121, 35): 331.9e6,
                    ("kron_matvec_split_kernel<4, 2, 3, 5, 2>", 261121, 35): 335.9e6,
                    ("kron_matvec_split_kernel<4, 2, 3, 5, 4>", 261121, 35): 351.7e6}
# The same for the fused dense RAS apply with Kronecker local solves and BF16
# inverse rows (profiles/ras_512x512_P35_counters.txt), keyed by precision and
# workload.
MEASURED_RAS_TRAFFIC = {("bf16", 261121, 35): 872.1e6}
MV_KERNEL_NAMES = {"staged": "kron_matvec_split_kernel", "pair": "kron_matvec_spec_kernel",
                   "wide": "kron_matvec_wide_kernel", "generic": "kron_matvec_kernel",
                   "grouped": "kron_matvec_group_kernel", "row_tiled": "kron_matvec_rowtile_kernel"}


def ras_roofline(ras, prec: str, n: int, P: int):
    """The RAS apply beside the matvec's roofline: it takes the larger share
    of the mixed-precision solve (two applies per iteration against two
    matvecs), so its HBM figures are reported the same way (algorithmic
    bytes of one flushed apply over its HIP-event time); None without the
    RAS part."""
    if not ras or ras.get("path") not in ("fused", "dense", "dense32"):
        return None
    return {"bound": "hbm", "kernel": f"dense RAS ({ras['path']}, {prec})",
            "achieved": ras["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ras["GBps"] / HBM_PEAK_GBS, 4),
            "traffic": MEASURED_RAS_TRAFFIC.get((prec, n, P)) if ras["path"] == "fused" else None,
            "traffic_unit": "bytes per launch"}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def matvec_bytes(n: int, nnz: int, L: int, P: int) -> int:
    """Algorithmic bytes of one Y = sum_i K_i X G_i: the L values, column
    index and row pointer of every stored non-zero, X read once, Y written
    once."""
    return L * nnz * 8 + nnz * 4 + (n + 1) * 4 + 2 * n * P * 8


def matvec_mf_bytes(n: int, P: int, M: int, n_tri: int, uniform: bool, S: int) -> int:
    """Algorithmic bytes of the matrix-free apply: X read and Y written once,
    each element's fields (c0, g_1..g_M) read once, its six local stiffness
    entries unless the lattice is uniform, and a 16-bit staging index per
    stencil direction of every row."""
    return 2 * n * P * 8 + n_tri * (M + 1) * 8 + (0 if uniform else n_tri * 6 * 8) + n * S * 2


def matvec_flops(n: int, nnz: int, L: int, P: int, T: int) -> int:
    return 2 * nnz * L * P + 2 * n * T


def time_launches(fn, launches: int, torch):
    """Mean and median duration (ms) of fn() on the current stream (where
    the library launches when given no stream), HIP events around each call,
    512 MB written between calls to flush the 256 MB Infinity Cache."""
    flush = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(5):
        fn()
    times = []
    for _ in range(launches):
        flush.add_(1.0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.mean(times)), float(np.median(times))


def time_matvec(g, launches: int, torch):
    """Average duration of the matvec kernel (see time_launches)."""
    from paper_2310_14649_amd import binding as B
    X = g.new_vec()
    X.normal_()
    Y = g.new_vec()
    return time_launches(lambda: B.sg_matvec(g.op, X, Y), launches, torch)


ENTRY_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2}
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense, MI355X


def ras_only(pr, prec: str, path: str, launches: int, torch, g=None, local: str = "mean") -> dict:
    """One RAS apply (Z = sum_s R_s^T D_s A_s^{-1} R_s R) timed alone.
    Algorithmic bytes: the stored inverse data read once (dense rows, or the
    sweep's Schur-complement inverses), R read once, Z written once; flops
    of the dense paths: 2 n_own n_local P per subdomain.  g: an existing
    GpuSG of that precision to reuse (kept open), else one is set up."""
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.solver import GpuSG
    own = g is None
    if own:
        g = GpuSG(pr, prec=prec, coarse="none", ras_path=path, local=local)
    try:
        name = B.ras_path_info(g.ras)[2]
        nloc, _, factor_bytes = B.ras_info(g.ras, pr.n_sub)
        nown = np.bincount(np.asarray(pr.owner), minlength=pr.n_sub).astype(np.int64)
        vec = g.n * g.P * 8
        dense_entries = int((nown * nloc.astype(np.int64)).sum())
        if name == "sweep":
            stored = int(factor_bytes)
            flops = None
        else:
            stored = dense_entries * ENTRY_BYTES[prec]
            flops = 2 * dense_entries * g.P
        R = g.new_vec()
        R.normal_()
        Z = g.new_vec()
        mean_ms, med_ms = time_launches(lambda: B.ras_apply(g.ras, R, Z), launches, torch)
        nbytes = stored + 2 * vec
        out = {"ras_only": True, "prec": prec, "path": name, "us": round(mean_ms * 1e3, 2),
               "median_us": round(med_ms * 1e3, 2), "bytes": nbytes, "stored_bytes": stored,
               "GBps": round(nbytes / (mean_ms * 1e-3) / 1e9, 1),
               "frac_hbm_peak": round(nbytes / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "ras_ms_sweep_dense_dense32_fused": g.ras_ms}
        if flops is not None:
            tf = flops / (mean_ms * 1e-3) / 1e12
            out.update(flops=flops, TFLOPs=round(tf, 2),
                       frac_mfma_peak=round(tf / MFMA_PEAK_TFLOPS[prec], 4))
        return out
    finally:
        if own:
            g.close()


def amg_only(pr, prec: str, launches: int, torch, g=None) -> dict:
    """One SA-AMG V(1,1)-cycle on the coarse problem timed alone.
    Algorithmic bytes per cycle: on every level but the coarsest, the
    operator's blocks twice (the residuals after pre- and post-smoothing),
    the prolongator and restriction once each and the block-Jacobi inverses
    twice; the coarsest dense FP64 inverse once (vectors are negligible).
    g: an existing GpuSG with an AMG coarse solver to reuse (kept open)."""
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.solver import GpuSG
    own = g is None
    if own:
        g = GpuSG(pr, prec=prec, coarse="amg", ras_path="sweep")
    try:
        P = g.P
        nl, nodes, _ = B.amg_info(g.amg, pr.n_sub)
        blk = P * P * 8
        levels = []
        nbytes = 0
        for lv in range(nl):
            a_b, p_b, r_b = B.amg_level_blocks(g.amg, lv)
            if lv < nl - 1:
                lb = (2 * a_b + p_b + r_b) * blk + 2 * int(nodes[lv]) * P * P * ENTRY_BYTES[prec]
            else:
                lb = a_b * blk
            levels.append(dict(nodes=int(nodes[lv]), a_blocks=a_b, p_blocks=p_b, r_blocks=r_b,
                               bytes=lb))
            nbytes += lb
        b_c = torch.randn(pr.n_sub * P, dtype=torch.float64, device="cuda")
        x_c = torch.empty_like(b_c)
        mean_ms, med_ms = time_launches(lambda: B.amg_vcycle(g.amg, b_c, x_c), launches, torch)
        return {"amg_only": True, "prec": prec, "levels": levels, "us": round(mean_ms * 1e3, 2),
                "median_us": round(med_ms * 1e3, 2), "bytes": nbytes,
                "GBps": round(nbytes / (mean_ms * 1e-3) / 1e9, 1),
                "frac_hbm_peak": round(nbytes / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    finally:
        if own:
            g.close()


def stochastic_sweep(args, torch, shapes=None, nc=None) -> dict:
    """Iterations and time against the number of random variables M and the
    output order p on one mesh (the paper's weak scaling in the stochastic
    dimensions): config 1's field (sigma 0.5, l 0.2), input order
    min(2, p), N_c = nc (default args.sweep_nc), 8 x 8 subdomains with
    overlap 2, the two-level preconditioner in FP64 and BF16, FGMRES(50) to
    1e-8, for every (M, p) of `shapes` (default: M in 2..6, p in 1..4 with
    P <= 128)."""
    from math import comb
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.inputs import make_problem
    from paper_2310_14649_amd.solver import GpuSG
    nc = args.sweep_nc if nc is None else nc
    if shapes is None:
        shapes = [(M, p) for M in range(2, 7) for p in range(1, 5) if comb(M + p, p) <= 128]
    rows = []
    for M, p in shapes:
        P = comb(M + p, p)
        pr = make_problem("c1", nc=nc, M=M, p=p, sub=(8, 8))
        row = dict(M=M, p=p, P=P, L_in=comb(M + min(2, p), min(2, p)),
                   unknowns=pr.mesh.n * P)
        for prec in ("fp64", "bf16"):
            try:
                g = GpuSG(pr, prec=prec, coarse="amg", ras_path="auto", local=args.local)
            except B.SgError as e:          # a shape outside a compiled limit
                row[prec] = dict(error=str(e))
                continue
            with g:
                rho, omega = g.damping()
                g.solve(pr.restart, pr.rtol, omega=omega, use_graph=True, ortho=args.ortho)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=True,
                                  ortho=args.ortho)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                row[prec] = dict(its=info["iterations"], ms=round(ms, 3),
                                 us_per_it=round(ms * 1e3 / max(info["iterations"], 1), 1),
                                 relres=info["true_relres"],
                                 ras_path=B.ras_path_info(g.ras)[2])
                row["matvec_kernel"] = B.sg_matvec_kernel(g.op)
        log(f"[bench] sweep M={M} p={p} P={P}: " + ", ".join(
            f"{k} " + (f"{row[k]['its']} its {row[k]['ms']:.1f} ms" if "its" in row[k]
                       else row[k]["error"]) for k in ("fp64", "bf16"))
            + f" ({row.get('matvec_kernel', '?')} matvec)")
        rows.append(row)
    return {"sweep": True, "nc": nc, "local_solves": args.local, "rows": rows}


def _timed_solve(g, pr, omega, torch, graph=True, ortho="block3"):
    """One warm solve, then one timed: (milliseconds, info)."""
    g.solve(pr.restart, pr.rtol, omega=omega, use_graph=graph, ortho=ortho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=graph, ortho=ortho)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, info


def coarse_study(args, torch) -> dict:
    """The paper's coarse-solve variants and coarse-grid ratio (Sec. 3 and the
    coarse-ratio tables).  variants: on the configuration's problem, the
    coarse problem solved by one V-cycle, by GMRES + V-cycle to 1e-5 (2GV3)
    and by GMRES + block Jacobi to 1e-2, <= 100 steps (2GV2), with the FP64
    and BF16 preconditioners.  ratio: config 1's field on an N_c = args.ratio_nc
    mesh, subdomain grids 8 x 8 .. 64 x 64 (fine nodes per coarse node from
    about N_c^2/64 down to N_c^2/4096), V-cycle and 2GV3, BF16 preconditioner."""
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.inputs import make_problem
    from paper_2310_14649_amd.solver import GpuSG
    variants = []
    pr = make_problem(args.config)
    for prec in ("fp64", "bf16"):
        with GpuSG(pr, prec=prec, coarse="amg", ras_path="auto", local=args.local) as g:
            rho, omega = g.damping()
            for inner, rtol in (("none", 0.0), ("gmres_amg", 1e-5), ("gmres_bj", 1e-2)):
                if inner != "none":
                    g.set_inner(inner, rtol, 100)
                c0, i0, _ = B.amg_inner_stats(g.amg)
                ms, info = _timed_solve(g, pr, omega, torch, ortho=args.ortho)
                c1, i1, _ = B.amg_inner_stats(g.amg)
                row = dict(prec=prec, coarse=inner, inner_rtol=rtol, its=info["iterations"],
                           ms=round(ms, 3), relres=info["true_relres"])
                if inner != "none":
                    # the warm-up solve counted too: the timed solve's share
                    row["inner_steps_per_solve"] = round((i1 - i0) / max(c1 - c0, 1), 2)
                g.set_inner("none")
                log(f"[bench] coarse {prec} {inner}: {row['its']} its {ms:.1f} ms"
                    + (f", {row['inner_steps_per_solve']} inner steps per coarse solve"
                       if inner != "none" else ""))
                variants.append(row)
    ratio = []
    for gx in (8, 16, 32, 64):
        prr = make_problem("c1", nc=args.ratio_nc, sub=(gx, gx))
        for inner in ("none", "gmres_amg"):
            try:
                g = GpuSG(prr, prec="bf16", coarse="amg", ras_path="auto", local=args.local)
            except B.SgError as e:
                ratio.append(dict(sub=gx * gx, coarse=inner, error=str(e)))
                log(f"[bench] ratio {gx}x{gx}: {e}")
                continue
            with g:
                rho, omega = g.damping()
                if inner != "none":
                    g.set_inner(inner, 1e-5, 100)
                ms, info = _timed_solve(g, prr, omega, torch, ortho=args.ortho)
                row = dict(sub=gx * gx, nodes_per_coarse_node=round(prr.mesh.n / (gx * gx), 1),
                           coarse_unknowns=gx * gx * g.P, coarse=inner, its=info["iterations"],
                           ms=round(ms, 3), ras_path=B.ras_path_info(g.ras)[2],
                           amg_levels=B.amg_info(g.amg, gx * gx)[0])
            log(f"[bench] ratio {gx}x{gx} ({row['nodes_per_coarse_node']} nodes per coarse node) "
                f"{inner}: {row['its']} its {row['ms']:.1f} ms")
            ratio.append(row)
    geometric = geometric_ratio_study(args, torch)
    return {"coarse_study": True, "config": args.config, "local_solves": args.local,
            "variants": variants,
            "ratio_nc": args.ratio_nc, "ratio": ratio, "geometric": geometric}


def geometric_ratio_study(args, torch) -> list:
    """The coarse-ratio study with the coarse space of a coarser lattice
    (Eq. coarse; the ratio tables of Sec. 5): config 1's field on an
    N = args.ratio_nc lattice, 16 x 16 fine subdomains, cell ratios r = 2, 4,
    8, 16 (fine:coarse unknowns about 4, 16, 66, 290), the coarse problem
    solved by FGMRES to 1e-5 (<= 100 steps) preconditioned by its own RAS
    (subdomains of about 16 x 16 coarse nodes) with its mean-based Nicolaides
    correction (a third level), and by FGMRES to 1e-2 with its one-level RAS
    (the 2GV2 reading); FP64 and BF16 fine-level preconditioners."""
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.inputs import make_problem
    from paper_2310_14649_amd.solver import Geometric, GpuSG
    rows = []
    prr = make_problem("c1", nc=args.ratio_nc, sub=(16, 16))
    for prec in ("fp64", "bf16"):
        for r in (2, 4, 8, 16):
            for level, rtol in (("mean", 1e-5), ("none", 1e-2)):
                geo = Geometric(r, overlap=1, level_coarse=level, rtol=rtol,
                                max_its=100)
                try:
                    t0 = time.perf_counter()
                    g = GpuSG(prr, prec=prec, coarse=geo, ras_path="auto", local=args.local)
                    setup_ms = (time.perf_counter() - t0) * 1e3
                except B.SgError as e:
                    rows.append(dict(prec=prec, ratio=r, level_coarse=level, error=str(e)))
                    log(f"[bench] geometric r={r}: {e}")
                    continue
                with g:
                    rho, omega = g.damping()
                    nc, nnz_c, om_c = B.amg_geometric_info(g.amg)
                    c0, i0, _ = B.amg_inner_stats(g.amg)
                    ms, info = _timed_solve(g, prr, omega, torch, ortho=args.ortho)
                    c1, i1, _ = B.amg_inner_stats(g.amg)
                    row = dict(prec=prec, ratio=r, unknown_ratio=round(g.n / nc, 2),
                               coarse_nodes=nc, coarse_unknowns=nc * g.P, level_coarse=level,
                               inner_rtol=rtol, its=info["iterations"], ms=round(ms, 3),
                               relres=info["true_relres"], setup_ms=round(setup_ms, 1),
                               coarse_steps_per_solve=round((i1 - i0) / max(c1 - c0, 1), 2),
                               coarse_omega=round(om_c, 4))
                log(f"[bench] geometric {prec} r={r} ({row['unknown_ratio']}:1) {level}: "
                    f"{row['its']} its, {row['coarse_steps_per_solve']} coarse steps, "
                    f"{ms:.1f} ms")
                rows.append(row)
    return rows


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pr, its_gpu: int, sample_its: int, local: str = "mean", omega: float = 0.5):
    """The oracle (plain NumPy/SciPy FP64) on the host: setup, then
    ``sample_its`` FGMRES iterations with the same preconditioner definition
    (mean-based or Kronecker local solves, the GPU solve's damping omega),
    scaled to the iteration count of the GPU FP64 solve."""
    from threadpoolctl import threadpool_info

    from oracle import krylov, system
    from oracle import ras as oras
    m = pr.mesh
    t0 = time.perf_counter()
    S = system.build(m.xy, m.tri, m.dof, m.n, pr.g0, pr.g, pr.M, pr.p_in, pr.p)
    B2, subs, *_ = system.two_level(S, pr.owner, pr.n_sub, pr.overlap, "amg", omega=omega)
    if local == "kron":
        Gt = oras.kron_factor(S.K, S.G)
        B2.M = lambda R: oras.ras_apply_kron(subs, R, Gt)  # noqa: E731
    t_setup = time.perf_counter() - t0
    X = np.random.default_rng(0).standard_normal((m.n, S.P))
    t0 = time.perf_counter()
    S.matvec(X)
    t_mv = time.perf_counter() - t0
    t0 = time.perf_counter()
    krylov.fgmres(S.matvec, S.B, B2, m=50, rtol=1e-8, max_it=sample_its)
    t_its = time.perf_counter() - t0
    per_it = t_its / sample_its
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return dict(per_it_s=per_it, setup_s=t_setup, matvec_s=t_mv, threads=threads,
                est_solve_ms=per_it * its_gpu * 1e3)


def workload(pr, n: int, P: int, mixed: str, local: str = "mean") -> str:
    """The workload named by its sizes."""
    nc = pr.mesh.nc
    mesh = f"{nc}x{nc} P1" + (" (jittered vertices)" if pr.mesh.jittered else "")
    sub = (f"{pr.n_sub} graph-partitioned subdomains" if "partition_seed" in pr.extra
           else f"{pr.n_sub} lattice subdomains")
    return (f"linear SG Poisson {mesh}, M={pr.M} KL vars, order {pr.p} (P={P}), {n * P:,} "
            f"unknowns, RAS on {sub} overlap {pr.overlap} with "
            f"{'Kronecker K0 x Gt' if local == 'kron' else 'mean-based K0 x G0'} local solves "
            f"+ SA-AMG Nicolaides coarse, "
            f"FGMRES({pr.restart}) to {pr.rtol:g}, preconditioner {mixed}")


def config_faithful(pr, args, torch) -> dict:
    """Configs 1 and 2 as they are stated: mean-based local solves
    K_0 (x) G_0 and modified Gram-Schmidt, the FP64 preconditioner against
    the BF16 one (FP32 too), each RAS path autotuned."""
    from paper_2310_14649_amd.solver import GpuSG
    out = {"local_solves": "mean", "ortho": "mgs"}
    ref = None
    for prec in ("fp64", "bf16", "fp32"):
        with GpuSG(pr, prec=prec, coarse="amg", ras_path="auto", local="mean") as g:
            rho, omega = g.damping()
            g.solve(pr.restart, pr.rtol, omega=omega, use_graph=True, ortho="mgs")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=True, ortho="mgs")
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            row = dict(ms=round(ms, 3), iterations=info["iterations"],
                       relres=info["true_relres"], omega=round(omega, 4))
            if ref is None:
                ref = x.clone()
            else:
                row["rel_diff_vs_fp64"] = float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))
            out[prec] = row
            log(f"[bench] config-faithful (mean local, MGS) {prec}: {ms:.1f} ms, "
                f"{info['iterations']} its")
    out["speedup_bf16_vs_fp64"] = round(out["fp64"]["ms"] / out["bf16"]["ms"], 3)
    return out


def config1_geometric(pr, args, torch) -> dict:
    """Config 1's problem with the paper's own coarse space instead of the
    Nicolaides one: a coarser lattice (Eq. coarse) with cell ratio 16 or 32
    (coarse lattices of 31^2 and 15^2 nodes), the coarse problem solved by
    FGMRES to 1e-2 (<= 100 steps) with its one-level RAS (subdomains of about
    16 x 16 coarse nodes), the fine level as in the headline solve."""
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.solver import Geometric, GpuSG
    out = {"coarse": "geometric", "local_solves": args.local, "ortho": args.ortho,
           "coarse_rtol": 1e-2, "rows": []}
    for prec in ("fp64", args.mixed):
        for r in (16, 32):
            geo = Geometric(r, overlap=1, level_coarse="none", rtol=1e-2, max_its=100)
            t0 = time.perf_counter()
            with GpuSG(pr, prec=prec, coarse=geo, ras_path="auto", local=args.local) as g:
                setup_ms = (time.perf_counter() - t0) * 1e3
                rho, omega = g.damping()
                g.solve(pr.restart, pr.rtol, omega=omega, use_graph=True, ortho=args.ortho)
                c0, i0, _ = B.amg_inner_stats(g.amg)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=True,
                                      ortho=args.ortho)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / args.steps
                c1, i1, _ = B.amg_inner_stats(g.amg)
                nc = B.amg_geometric_info(g.amg)[0]
                row = dict(prec=prec, ratio=r, coarse_unknowns=nc * g.P,
                           unknown_ratio=round(g.n / nc, 1), ms=round(ms, 3),
                           iterations=info["iterations"], relres=info["true_relres"],
                           coarse_steps_per_solve=round((i1 - i0) / max(c1 - c0, 1), 2),
                           setup_ms=round(setup_ms, 1))
            out["rows"].append(row)
            log(f"[bench] config 1, geometric coarse r={r} {prec}: {ms:.1f} ms, "
                f"{info['iterations']} its, {row['coarse_steps_per_solve']} coarse steps")
    return out


def bench_config3(args, torch) -> dict:
    """Config 3: the jittered 384 x 384 mesh, M = 6, p = 3 (P = 84, 12.3M
    unknowns), 192 graph-partitioned subdomains of uneven size, FGMRES(50)
    to 1e-8 with graph-captured Arnoldi steps and autotuned RAS paths, in
    FP64 and with the BF16 preconditioner; and its SG matvec (grouped
    kernel) after a cache flush against its algorithmic bytes."""
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.inputs import make_problem
    from paper_2310_14649_amd.solver import GpuSG
    t0 = time.perf_counter()
    pr = make_problem("c3")
    out = {"workload": workload(pr, pr.mesh.n, 84, "bf16", args.local),
           "generate_s": round(time.perf_counter() - t0, 2)}
    ref = None
    for prec in ("fp64", "bf16"):
        t0 = time.perf_counter()
        with GpuSG(pr, prec=prec, coarse="amg", ras_path="auto", local=args.local) as g:
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            rho, omega = g.damping()
            ms, info = _timed_solve(g, pr, omega, torch, ortho=args.ortho)
            row = dict(ms=round(ms, 3), iterations=info["iterations"],
                       relres=info["true_relres"], setup_s=round(setup, 2),
                       ras_path=B.ras_path_info(g.ras)[2], omega=round(omega, 4))
            x = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=True, ortho=args.ortho)[0]
            if ref is None:
                ref = x.clone()
                n, P, L, nnz = g.n, g.P, g.L, g.nnz
                mv_ms, mv_med = time_matvec(g, 20, torch)
                b = matvec_bytes(n, nnz, L, P)
                out["matvec"] = dict(kernel=B.sg_matvec_kernel(g.op), us=round(mv_ms * 1e3, 2),
                                     bytes=b, GBps=round(b / (mv_ms * 1e-3) / 1e9, 1),
                                     frac_hbm_peak=round(b / (mv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
            else:
                row["rel_diff_vs_fp64"] = float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))
            out[prec] = row
            log(f"[bench] config 3 {prec}: {ms:.1f} ms, {info['iterations']} its")
    return out


SWEEP_SHAPES = [(2, 1), (4, 1), (2, 2), (4, 2), (6, 2), (3, 3), (4, 3), (2, 4), (4, 4)]


def jac_apply_part(g, launches: int, torch) -> dict:
    """The Newton Jacobian apply J V of a GpuNewton handle (at the last
    evaluated U), timed alone after a flush (time_launches), against the
    matvec's algorithmic bytes for its L2 values per entry."""
    from paper_2310_14649_amd import binding as B
    jop = B.sg_nl_jac_op(g.nl)
    n, P, L, nnz = B.sg_op_info(jop)
    V = torch.randn(n * P, dtype=torch.float64, device="cuda")
    Y = g.new_vec()
    mean_ms, med_ms = time_launches(lambda: B.sg_nl_jac_apply(g.nl, V, Y), launches, torch)
    b = matvec_bytes(n, nnz, L, P)
    gbs = b / (mean_ms * 1e-3) / 1e9
    return {"kernel": B.sg_matvec_kernel(jop), "L": L, "P": P, "n": n, "nnz": nnz,
            "us": round(mean_ms * 1e3, 2), "median_us": round(med_ms * 1e3, 2), "bytes": b,
            "GBps": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def jac_only(args, torch) -> dict:
    """Config 4's Jacobian apply alone (for counters): the residual at a
    seeded U sets the operator's values, then the flushed launches."""
    from paper_2310_14649_amd.inputs import make_problem
    from paper_2310_14649_amd.solver import GpuNewton
    pr = make_problem("c4")
    with GpuNewton(pr) as g:
        gen = torch.Generator(device="cuda").manual_seed(5)
        U = 0.3 * torch.randn(g.n * g.P, dtype=torch.float64, device="cuda", generator=gen)
        g.residual(U)
        out = jac_apply_part(g, args.mv_launches, torch)
    out["jac_only"] = True
    return out


def bench_newton(args, torch):
    """Config 4: Newton-FGMRES to ||R||/||F|| <= 1e-8 from the zero guess on
    the base draw, then the learned guess: training data from the solver,
    training, and held-out draws solved from the zero and from the learned
    guess."""
    import numpy as np
    from paper_2310_14649_amd.inputs import make_problem
    from paper_2310_14649_amd.learned import LearnedGuess, draw_params
    from paper_2310_14649_amd.solver import GpuNewton

    out = {}
    pr = make_problem("c4")
    with GpuNewton(pr, ortho=args.ortho, ras_path=args.newton_ras) as g:
        U, info = g.solve(tol=1e-8)                      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            U, info = g.solve(tol=1e-8)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        out["jacobian_apply"] = jac_apply_part(g, 20, torch)
        # the coarse hierarchy rebuilt at every Newton step instead of once
        g.solve(tol=1e-8, amg_rebuild=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, info_rb = g.solve(tol=1e-8, amg_rebuild=1)
        torch.cuda.synchronize()
        ms_rb = (time.perf_counter() - t0) * 1e3 / args.steps
    out["coarse_rebuilt_every_step"] = dict(ms=round(ms_rb, 3), krylov_its=info_rb["krylov_its"],
                                            ms_setup=round(info_rb["ms_setup"], 3))
    out["ras_path"] = args.newton_ras
    out["zero_guess"] = dict(ms=round(ms, 3), steps=info["steps"], krylov_its=info["krylov_its"],
                             relres=info["relres"], ms_eval=round(info["ms_eval"], 3),
                             ms_setup=round(info["ms_setup"], 3),
                             ms_krylov=round(info["ms_krylov"], 3),
                             its_per_step=info["krylov_its_per_step"].tolist())
    log(f"[bench] newton c4: {ms:.1f} ms, {info['steps']} steps, {info['krylov_its']} its")
    # the paper's model kappa(u) = 1 + u: its Picard linearisation (stopped at
    # ||dU|| <= 1e-6 ||U||, the paper's criterion) against Newton (to
    # ||R|| / ||F|| <= 1e-8), both from the zero guess
    with GpuNewton(pr, a1=1.0, a2=0.0, ortho=args.ortho, ras_path=args.newton_ras) as gp:
        res, sol = {}, {}
        for meth, kw in (("newton", dict(tol=1e-8)),
                         ("picard", dict(tol=1e-14, du_tol=1e-6, method="picard",
                                         max_steps=100))):
            gp.solve(**kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                Us, inf = gp.solve(**kw)
            torch.cuda.synchronize()
            res[meth] = dict(ms=round((time.perf_counter() - t0) * 1e3 / args.steps, 3),
                             steps=inf["steps"], krylov_its=inf["krylov_its"],
                             relres=inf["relres"], last_du=inf["last_du"],
                             its_per_step=inf["krylov_its_per_step"].tolist())
            sol[meth] = Us
        res["picard_vs_newton_rel_diff"] = float(torch.linalg.norm(sol["picard"] - sol["newton"]) /
                                                 torch.linalg.norm(sol["newton"]))
    out["paper_model_1_plus_u"] = res
    log(f"[bench] kappa = 1 + u, c4: Newton {res['newton']['ms']:.1f} ms, "
        f"{res['newton']['steps']} steps, {res['newton']['krylov_its']} its; Picard "
        f"{res['picard']['ms']:.1f} ms, {res['picard']['steps']} steps, "
        f"{res['picard']['krylov_its']} its; difference {res['picard_vs_newton_rel_diff']:.2e}")
    if args.learned_draws <= 0:
        return out
    lg = LearnedGuess("c4", max_batch=16, seed=0, ortho=args.ortho, ras_path=args.newton_ras)
    try:
        ds = lg.generate(draw_params(args.learned_draws, seed=0))
        lg.fit_output_scale(ds)
        losses, t_train = lg.train(ds, steps=args.learned_steps, batch=16, lr=2e-3, lr_final=2e-5)
        log(f"[bench] learned: {args.learned_draws} solves in {ds.seconds:.1f} s, "
            f"{args.learned_steps} Adam steps in {t_train:.1f} s, loss {np.mean(losses[-20:]):.3e}")
        rows = {"zero": [], "nn": []}
        choices = []
        for s_, e_ in draw_params(args.learned_heldout, seed=1):
            for key, use in (("zero", False), ("nn", True)):
                _, inf = lg.solve(s_, e_, use_nn=use)
                rows[key].append((inf["steps"], inf["krylov_its"], inf["seconds"] * 1e3))
                if use:
                    choices.append(inf["guess_choice"])
        summary = {k: dict(steps=float(np.mean([r[0] for r in v])),
                           krylov_its=float(np.mean([r[1] for r in v])),
                           ms=round(float(np.mean([r[2] for r in v])), 3)) for k, v in rows.items()}
        out["learned"] = dict(train_draws=args.learned_draws, adam_steps=args.learned_steps,
                              gen_s=round(ds.seconds, 2), train_s=round(t_train, 2),
                              final_loss=float(np.mean(losses[-20:])),
                              heldout=args.learned_heldout, guess_choices=choices, **summary)
        log(f"[bench] learned guess on {args.learned_heldout} held-out draws: {summary}")
    finally:
        lg.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--mixed", default="bf16", choices=["fp32", "bf16"])
    ap.add_argument("--also", default="fp32", help="extra preconditioner precisions to time")
    ap.add_argument("--mv-launches", type=int, default=50)
    ap.add_argument("--cpu-sample-its", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=1,
                    help="replay Arnoldi steps from captured HIP graphs (1) or launch eagerly (0)")
    ap.add_argument("--mv-tiles", type=int, default=0, choices=[0, 1, 2, 4],
                    help="with --matvec-only: 64-row tiles per work-group of the staged "
                         "matvec (0 keeps the library default)")
    ap.add_argument("--matrix-free", action="store_true",
                    help="with --matvec-only: time the matrix-free apply")
    ap.add_argument("--matvec-only", action="store_true",
                    help="time only the SG matvec (for counter collection) and print its figures")
    ap.add_argument("--ortho", default="block3",
                    choices=["mgs", "cgs2", "cgs", "block2", "block3", "block4"],
                    help="Arnoldi orthogonalisation")
    ap.add_argument("--ortho-compare", default="block2,block4,cgs,mgs",
                    help="other orthogonalisations timed on the mixed solve (comma list)")
    ap.add_argument("--ras-path", default="auto",
                    choices=["auto", "sweep", "dense", "dense32", "fused"],
                    help="RAS apply path: autotuned per precision, or forced")
    ap.add_argument("--ras-only", action="store_true",
                    help="time only one RAS apply (precision --part-prec) and print its figures")
    ap.add_argument("--jac-only", action="store_true",
                    help="time config 4's Newton Jacobian apply alone (flushed launches)")
    ap.add_argument("--amg-only", action="store_true",
                    help="time only one AMG V-cycle (precision --part-prec) and print its figures")
    ap.add_argument("--part-prec", default="bf16", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--sweep", action="store_true",
                    help="iterations and time against M (2..6) and p (1..4) on one mesh")
    ap.add_argument("--sweep-nc", type=int, default=256)
    ap.add_argument("--local", default="kron", choices=["mean", "kron"],
                    help="RAS local solves: mean-based K_0 (x) G_0 or Kronecker K_0 (x) Gt")
    ap.add_argument("--coarse-study", action="store_true",
                    help="coarse-solve variants (V-cycle, 2GV3, 2GV2) and the coarse-ratio sweep")
    ap.add_argument("--ratio-nc", type=int, default=256)
    ap.add_argument("--geometric-study", action="store_true",
                    help="only the coarse-ratio sweep with the geometric coarse space")
    ap.add_argument("--parts", type=int, default=1,
                    help="also time one RAS apply and one AMG V-cycle of the mixed solver alone")
    ap.add_argument("--newton", type=int, default=1, help="also time config 4 (Newton)")
    ap.add_argument("--newton-ras", default="auto",
                    choices=["auto", "sweep", "dense", "dense32", "fused"],
                    help="RAS apply path of the config-4 solves (auto: the autotuner's pick)")
    ap.add_argument("--geometric", type=int, default=1,
                    help="also time config 1 with the geometric coarse space (ratios 16, 32)")
    ap.add_argument("--faithful", type=int, default=1,
                    help="also time configs 1/2 as stated (mean-based local solves, MGS)")
    ap.add_argument("--c3", type=int, default=1, help="also time config 3 (P = 84, jittered)")
    ap.add_argument("--small-sweep", type=int, default=1,
                    help="also run a few (M, p) shapes of the stochastic sweep")
    ap.add_argument("--small-sweep-nc", type=int, default=128)
    ap.add_argument("--learned-draws", type=int, default=512,
                    help="training solves for the learned Newton guess (0: skip)")
    ap.add_argument("--learned-steps", type=int, default=1500)
    ap.add_argument("--learned-heldout", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(sharding the subdomains over several GPUs is not built)"}))
        return 2

    import torch
    from paper_2310_14649_amd import binding as B
    from paper_2310_14649_amd.inputs import make_problem
    from paper_2310_14649_amd.solver import GpuSG

    B.lib()
    torch.cuda.set_device(0)
    if args.jac_only:
        print(json.dumps(jac_only(args, torch)))
        return 0
    pr = make_problem(args.config)
    log(f"[bench] config {args.config}: n={pr.mesh.n} M={pr.M} p={pr.p} subdomains={pr.n_sub}")
    if args.sweep:
        print(json.dumps(stochastic_sweep(args, torch)))
        return 0
    if args.geometric_study:
        print(json.dumps({"geometric_study": True, "ratio_nc": args.ratio_nc,
                          "local_solves": args.local,
                          "geometric": geometric_ratio_study(args, torch)}))
        return 0
    if args.coarse_study:
        print(json.dumps(coarse_study(args, torch)))
        return 0
    if args.ras_only:
        print(json.dumps(ras_only(pr, args.part_prec, args.ras_path, args.mv_launches, torch,
                                  local=args.local)))
        return 0
    if args.amg_only:
        print(json.dumps(amg_only(pr, args.part_prec, args.mv_launches, torch)))
        return 0
    if args.matvec_only:
        g = GpuSG(pr, prec="fp64", coarse="none")
        if args.matrix_free:
            B.sg_matvec_matrix_free(g.op, True)
        if args.mv_tiles:
            B.sg_matvec_select(g.op, args.mv_tiles)
        n, P, L, nnz = g.n, g.P, g.L, g.nnz
        mv_mean_ms, mv_med_ms = time_matvec(g, args.mv_launches, torch)
        b = (matvec_mf_bytes(n, P, pr.M, pr.mesh.n_tri, not pr.mesh.jittered, 5)
             if args.matrix_free else matvec_bytes(n, nnz, L, P))
        print(json.dumps({"matvec_only": True, "config": args.config,
                          "kernel": B.sg_matvec_kernel(g.op), "tiles": B.sg_matvec_tiles(g.op),
                          "us": round(mv_mean_ms * 1e3, 2),
                          "median_us": round(mv_med_ms * 1e3, 2), "bytes": b,
                          "GBps": round(b / (mv_mean_ms * 1e-3) / 1e9, 1),
                          "flush_bytes_per_launch": 2 * 64 * 1024 * 1024 * 8}))
        g.close()
        return 0
    precs = ["fp64", args.mixed] + [p for p in args.also.split(",") if p and p not in ("fp64", args.mixed)]
    solvers = {}
    setup_s = {}
    ras_paths = {}
    for prec in precs:
        t0 = time.perf_counter()
        solvers[prec] = GpuSG(pr, prec=prec, coarse="amg", ras_path=args.ras_path,
                              local=args.local)
        torch.cuda.synchronize()
        setup_s[prec] = time.perf_counter() - t0
        ras_paths[prec] = dict(path=B.ras_path_info(solvers[prec].ras)[2],
                               ms_sweep_dense_dense32_fused=solvers[prec].ras_ms)
        log(f"[bench] setup {prec}: {setup_s[prec]:.2f} s, RAS {ras_paths[prec]}")
    g64 = solvers["fp64"]
    n, P, L, nnz = g64.n, g64.P, g64.L, g64.nnz
    T = B.sg_basis_info(g64.basis)[2]
    rho, omega = g64.damping()
    log(f"[bench] smoother damping: rho={rho:.4f} omega={omega:.4f}")

    results = {}
    ref_x = None
    for prec in precs:
        g = solvers[prec]
        for _ in range(max(args.warmup, 1 if args.graph else 0)):
            x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=bool(args.graph),
                              ortho=args.ortho)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=bool(args.graph),
                              ortho=args.ortho)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        results[prec] = dict(ms=ms, iterations=info["iterations"], relres=info["true_relres"],
                             converged=info["converged"])
        if prec == "fp64":
            ref_x = x.clone()
        else:
            results[prec]["rel_diff_vs_fp64"] = float(torch.linalg.norm(x - ref_x) /
                                                      torch.linalg.norm(ref_x))
        log(f"[bench] solve {prec}: {ms:.2f} ms, its={info['iterations']}, "
            f"relres={info['true_relres']:.2e}")

    # the solves with the matrix-free operator apply (same preconditioner)
    mf_solves = {}
    for prec in ("fp64", args.mixed):
        g = solvers[prec]
        try:
            B.sg_matvec_matrix_free(g.op, True)
        except B.SgError as e:
            mf_solves = {"error": str(e)}
            break
        try:
            g.solve(pr.restart, pr.rtol, omega=omega, use_graph=bool(args.graph), ortho=args.ortho)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=bool(args.graph),
                                  ortho=args.ortho)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            mf_solves[prec] = dict(ms=round(ms, 3), iterations=info["iterations"],
                                   relres=info["true_relres"],
                                   rel_diff_vs_fp64=float(torch.linalg.norm(x - ref_x) /
                                                          torch.linalg.norm(ref_x)))
            log(f"[bench] solve {prec} with the matrix-free apply: {ms:.2f} ms, "
                f"its={info['iterations']}")
        finally:
            B.sg_matvec_matrix_free(g.op, False)

    # the same mixed solve with the other orthogonalisations, for comparison
    ortho_cmp = {}
    for o in [v for v in args.ortho_compare.split(",") if v and v != args.ortho]:
        g = solvers[args.mixed]
        g.solve(pr.restart, pr.rtol, omega=omega, use_graph=bool(args.graph), ortho=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x, info = g.solve(pr.restart, pr.rtol, omega=omega, use_graph=bool(args.graph), ortho=o)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ortho_cmp[o] = dict(ms=round(ms, 3), iterations=info["iterations"],
                            relres=info["true_relres"])
        log(f"[bench] solve {args.mixed} with {o}: {ms:.2f} ms, its={info['iterations']}")

    mv_family = B.sg_matvec_kernel(g64.op)
    mv_kernel = MV_KERNEL_NAMES[mv_family]
    mv_tiles = B.sg_matvec_tiles(g64.op)
    if mv_family == "staged" and L == 15 and P == 35:
        mv_kernel += f"<4, 2, 3, 5, {mv_tiles}>"
    traffic = MEASURED_TRAFFIC.get((mv_kernel, n, P))
    mv_mean_ms, mv_med_ms = time_matvec(g64, args.mv_launches, torch)
    mv_bytes = matvec_bytes(n, nnz, L, P)
    mv_gbs = mv_bytes / (mv_mean_ms * 1e-3) / 1e9
    log(f"[bench] matvec: {mv_mean_ms * 1e3:.1f} us avg, {mv_gbs:.0f} GB/s algorithmic")
    # the matrix-free apply of the same operator (K values formed per row from
    # the element fields), timed the same way against its own bytes
    mv_mf = None
    try:
        B.sg_matvec_matrix_free(g64.op, True)
        mf_tiles = {}
        for tiles in (1, 2, 4):
            try:
                B.sg_matvec_select(g64.op, tiles)
            except B.SgError:
                continue
            mf_tiles[tiles] = time_matvec(g64, 20, torch)[0]
        best = min(mf_tiles, key=mf_tiles.get)
        B.sg_matvec_select(g64.op, best)
        mf_ms, mf_med = time_matvec(g64, args.mv_launches, torch)
        mf_b = matvec_mf_bytes(n, P, pr.M, pr.mesh.n_tri, not pr.mesh.jittered, 5)
        mv_mf = {"us": round(mf_ms * 1e3, 2), "median_us": round(mf_med * 1e3, 2),
                 "tiles_per_group": best,
                 "us_by_tiles": {k: round(v * 1e3, 2) for k, v in mf_tiles.items()},
                 "bytes": mf_b, "GBps": round(mf_b / (mf_ms * 1e-3) / 1e9, 1),
                 "frac_hbm_peak": round(mf_b / (mf_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 }
        mv_mf["speedup_vs_stored"] = round(mv_mean_ms / mf_ms, 3)
        log(f"[bench] matrix-free matvec: {mf_ms * 1e3:.1f} us ({best} tiles), "
            f"{mv_mf['GBps']:.0f} GB/s of its {mf_b / 1e6:.0f} MB")
    except B.SgError as e:
        mv_mf = {"error": str(e)}
    finally:
        B.sg_matvec_matrix_free(g64.op, False)
        B.sg_matvec_select(g64.op, mv_tiles)
    # the two preconditioner parts alone, on the mixed-precision solver
    parts = {}
    if args.parts:
        parts["ras"] = ras_only(pr, args.mixed, args.ras_path, 20, torch, g=solvers[args.mixed])
        parts["amg_vcycle"] = amg_only(pr, args.mixed, 50, torch, g=solvers[args.mixed])
        log(f"[bench] RAS {parts['ras']['path']}: {parts['ras']['us']:.1f} us, "
            f"{parts['ras']['GBps']:.0f} GB/s; AMG V-cycle {parts['amg_vcycle']['us']:.1f} us")

    cpu = None
    if not args.no_cpu_baseline:
        c = cpu_baseline(pr, results["fp64"]["iterations"], args.cpu_sample_its, args.local,
                         omega)
        cpu = {"value": c["est_solve_ms"], "unit": "ms", "cores": c["threads"], "kind": "oracle",
               "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
               "sample": f"{args.cpu_sample_its} oracle FGMRES(50) iterations of this workload "
                         f"(omega {omega:.4f} as on the GPU) "
                         f"(FP64, same two-grid preconditioner, setup {c['setup_s']:.1f} s "
                         f"excluded) at {c['per_it_s']:.2f} s/iteration, scaled to the "
                         f"{results['fp64']['iterations']} iterations of the GPU FP64 solve; "
                         f"one oracle matvec took {c['matvec_s'] * 1e3:.0f} ms "
                         f"({mv_bytes / c['matvec_s'] / 1e9:.2f} GB/s, scipy.sparse single-threaded)"}
        log(f"[bench] cpu oracle: {c['per_it_s']:.2f} s/it")

    faithful = config_faithful(pr, args, torch) if args.faithful else None
    geometric = config1_geometric(pr, args, torch) if args.geometric else None
    c3 = bench_config3(args, torch) if args.c3 else None
    sweep = (stochastic_sweep(args, torch, SWEEP_SHAPES, nc=args.small_sweep_nc)
             if args.small_sweep else None)
    newton = bench_newton(args, torch) if args.newton else None

    mixed = results[args.mixed]
    out = {
        "metric": "FGMRES time to rel-res 1e-8 (mixed vs FP64 GPU); SG matvec GB/s vs HBM peak",
        "value": round(mixed["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f64 outer / {args.mixed} preconditioner",
        "data": "synthetic",
        "config": {"workload": workload(pr, n, P, args.mixed, args.local),
                   "n": n, "P": P, "L_in": L, "nnz": nnz, "triples": T, "subdomains": pr.n_sub,
                   "graph": bool(args.graph), "ortho": args.ortho},
        "solves": results,
        "speedup_mixed_vs_fp64": round(results["fp64"]["ms"] / mixed["ms"], 3),
        "mixed_other_ortho": ortho_cmp,
        "solves_matrix_free_apply": mf_solves,
        "matvec": {"us": round(mv_mean_ms * 1e3, 2), "median_us": round(mv_med_ms * 1e3, 2),
                   "tiles_per_group": mv_tiles, "autotune_ms_1_2_4_tiles": g64.mv_ms,
                   "GBps": round(mv_gbs, 1), "frac_hbm_peak": round(mv_gbs / HBM_PEAK_GBS, 4),
                   "bytes": mv_bytes, "flops": matvec_flops(n, nnz, L, P, T)},
        "matvec_matrix_free": mv_mf,
        "roofline": {"bound": "hbm", "kernel": mv_kernel, "achieved": round(mv_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(mv_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_unit": "bytes per launch"},
        "roofline_ras": ras_roofline(parts.get("ras"), args.mixed, n, P),
        "parts": parts,
        "setup_s": {k: round(v, 2) for k, v in setup_s.items()},
        "ras_path": ras_paths,
        "local_solves": args.local,
        "omega": omega,
        "cpu_baseline": cpu,
        "config_faithful_mean_mgs": faithful,
        "config1_geometric_coarse": geometric,
        "config3": c3,
        "stochastic_sweep": sweep,
        "newton_c4": newton,
    }
    for g in solvers.values():
        g.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
