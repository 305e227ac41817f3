"""ctypes binding of ``libsgsolve.so``: one Python function per C entry
point, same names, argument marshalling only (host arrays are NumPy, device
arrays are torch tensors on the current HIP device).  Every numerical step
runs in the library's kernels; there is no fallback: importing the library
fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgsolve.so")

SG_OK, SG_NOT_CONVERGED = 0, 1
SG_FP64, SG_FP32, SG_BF16 = 0, 1, 2
SG_COARSE_NONE, SG_COARSE_MEAN_EXACT, SG_COARSE_AMG, SG_COARSE_GEOMETRIC = 0, 1, 2, 3
PREC = {"fp64": SG_FP64, "fp32": SG_FP32, "bf16": SG_BF16}
SG_ORTHO_MGS, SG_ORTHO_CGS_DGKS, SG_ORTHO_CGS, SG_ORTHO_CGS_BLOCK2 = 0, 1, 2, 3
SG_ORTHO_CGS_BLOCK3, SG_ORTHO_CGS_BLOCK4 = 4, 5
ORTHO = {"mgs": SG_ORTHO_MGS, "cgs2": SG_ORTHO_CGS_DGKS, "cgs": SG_ORTHO_CGS,
         "block2": SG_ORTHO_CGS_BLOCK2, "block3": SG_ORTHO_CGS_BLOCK3,
         "block4": SG_ORTHO_CGS_BLOCK4}

_vp = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


class SgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sgsolve error {code}: {msg}")
        self.code = code


class KrylovOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_it", C.c_int), ("rtol", C.c_double),
                ("omega", C.c_double), ("use_graph", C.c_int), ("ortho", C.c_int)]


class KrylovStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("true_relres", C.c_double), ("omega", C.c_double), ("ms_solve", C.c_double),
                ("history", _f64p), ("history_cap", C.c_int), ("history_len", C.c_int)]


NL_RAS_PATHS = {"auto": -1, "sweep": 0, "dense": 1, "dense32": 2, "fused": 3}


class NewtonOpts(C.Structure):
    _fields_ = [("max_steps", C.c_int), ("tol", C.c_double), ("eta_max", C.c_double),
                ("restart", C.c_int), ("max_it", C.c_int), ("omega", C.c_double),
                ("use_graph", C.c_int), ("ortho", C.c_int), ("amg_rebuild", C.c_int),
                ("method", C.c_int), ("du_tol", C.c_double), ("ras_path", C.c_int)]


SG_NEWTON, SG_PICARD = 0, 1
NL_METHODS = {"newton": SG_NEWTON, "picard": SG_PICARD}


class NewtonStats(C.Structure):
    _fields_ = [("steps", C.c_int), ("krylov_its", C.c_int), ("converged", C.c_int),
                ("relres", C.c_double), ("last_lambda", C.c_double), ("last_du", C.c_double),
                ("ms_total", C.c_double),
                ("ms_eval", C.c_double), ("ms_setup", C.c_double), ("ms_krylov", C.c_double),
                ("history", _f64p), ("krylov_its_per_step", _i32p), ("history_cap", C.c_int),
                ("history_len", C.c_int)]


_SIGS = {
    "sg_last_error": (C.c_char_p, []),
    "sg_version": (C.c_int, []),
    "sg_set_allocator": (C.c_int, [_vp, _vp, _vp]),
    "sg_set_arena": (C.c_int, [_vp, C.c_size_t]),
    "sg_arena_reset": (C.c_int, []),
    "sg_memory_stats": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]),
    "sg_memory_reset_peak": (C.c_int, []),
    "sg_build_triples": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(_vp)]),
    "sg_basis_info": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "sg_basis_export": (C.c_int, [_vp, _i32p, _i32p, _f64p]),
    "sg_destroy_basis": (None, [_vp]),
    "sg_assemble": (C.c_int, [_vp, C.c_int, _f64p, C.c_int, _i32p, _i32p, C.c_int, _f64p, _f64p,
                              C.POINTER(_vp), _vp]),
    "sg_op_info": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_int64)]),
    "sg_op_rhs": (C.c_int, [_vp, _vp, _vp]),
    "sg_op_export": (C.c_int, [_vp, _i64p, _i32p, _f64p]),
    "sg_destroy_op": (None, [_vp]),
    "sg_matvec": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sg_matvec_kernel": (C.c_int, [_vp, C.POINTER(C.c_int)]),
    "sg_matvec_autotune": (C.c_int, [_vp, C.c_int, _f64p, _vp]),
    "sg_matvec_select": (C.c_int, [_vp, C.c_int]),
    "sg_matvec_tiles": (C.c_int, [_vp, C.POINTER(C.c_int)]),
    "ras_setup": (C.c_int, [_vp, _i32p, C.c_int, C.c_int, C.c_int, C.POINTER(_vp), _vp]),
    "ras_refactor": (C.c_int, [_vp, _vp, _vp]),
    "ras_select": (C.c_int, [_vp, C.c_int, _vp]),
    "ras_autotune": (C.c_int, [_vp, C.c_int, _f64p, _vp]),
    "ras_path_info": (C.c_int, [_vp, C.POINTER(C.c_int), _i64p]),
    "ras_info": (C.c_int, [_vp, _i32p, _i32p, _i64p]),
    "ras_set_local": (C.c_int, [_vp, _vp, C.c_int, _vp]),
    "ras_local_factor": (C.c_int, [_vp, _f64p]),
    "ras_apply": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sg_destroy_ras": (None, [_vp]),
    "amg_setup": (C.c_int, [_vp, _vp, C.c_int, C.c_int, C.POINTER(_vp), _vp]),
    "amg_info": (C.c_int, [_vp, C.POINTER(C.c_int), _i32p, _i32p]),
    "amg_setup_geometric": (C.c_int, [_vp, C.c_int, _i32p, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_double, C.c_int, C.POINTER(_vp), _vp]),
    "amg_geometric_info": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_double)]),
    "amg_geometric_op": (_vp, [_vp]),
    "amg_vcycle": (C.c_int, [_vp, _vp, _vp, _vp]),
    "amg_set_inner": (C.c_int, [_vp, C.c_int, C.c_double, C.c_int]),
    "amg_inner_stats": (C.c_int, [_vp, _i64p, _i64p, C.POINTER(C.c_int)]),
    "amg_coarse_solve": (C.c_int, [_vp, _vp, _vp, _vp]),
    "amg_level_blocks": (C.c_int, [_vp, C.c_int, _i64p, _i64p, _i64p]),
    "sg_coarse_restrict": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sg_coarse_prolong_add": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sg_destroy_amg": (None, [_vp]),
    "sg_precond_workspace_bytes": (C.c_size_t, [_vp, _vp]),
    "sg_precond_apply": (C.c_int, [_vp, _vp, _vp, C.c_double, _vp, _vp, _vp, C.c_size_t, _vp]),
    "sg_smoother_damping": (C.c_int, [_vp, _vp, C.c_int, _f64p, _f64p, _vp, C.c_size_t, _vp]),
    "fgmres_workspace_bytes": (C.c_size_t, [_vp, _vp, C.c_int]),
    "sg_graph_cache_clear": (C.c_int, []),
    "fgmres_solve": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.POINTER(KrylovOpts),
                               C.POINTER(KrylovStats), _vp, C.c_size_t, _vp]),
    "sg_nl_setup": (C.c_int, [_vp, C.c_int, _f64p, C.c_int, _i32p, _i32p, C.c_int, _f64p, _f64p,
                              C.c_double, C.c_double, C.POINTER(_vp), _vp]),
    "sg_nl_info": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_int64)]),
    "sg_nl_eval": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sg_nl_jac_apply": (C.c_int, [_vp, _vp, _vp, _vp]),
    "sg_nl_export": (C.c_int, [_vp, _i64p, _i32p, _f64p, _f64p]),
    "sg_nl_mean_op": (_vp, [_vp]),
    "sg_nl_jac_op": (_vp, [_vp]),
    "sg_destroy_nl": (None, [_vp]),
    "sg_nl_set_coefficients": (C.c_int, [_vp, _f64p, _f64p, _vp]),
    "newton_guess_workspace_bytes": (C.c_size_t, [_vp]),
    "newton_guess": (C.c_int, [_vp, _vp, _vp, _f64p, C.POINTER(C.c_int), _vp, C.c_size_t, _vp]),
    "nn_create": (C.c_int, [C.c_int, _i32p, C.c_int, C.c_int, C.c_int, C.POINTER(_vp)]),
    "nn_param_count": (C.c_int64, [_vp]),
    "nn_set_params": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "nn_get_params": (C.c_int, [_vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "nn_set_output_map": (C.c_int, [_vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "nn_forward": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp]),
    "sg_matvec_matrix_free": (C.c_int, [_vp, C.c_int, _vp]),
    "sg_matvec_row_tiled": (C.c_int, [_vp, C.c_int]),
    "nn_fit_output_map": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp]),
    "nn_input_fields": (C.c_int, [C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "nn_loss_grad": (C.c_int, [_vp, _vp, _vp, C.c_int, _f64p, _vp]),
    "nn_adam_step": (C.c_int, [_vp, C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    "nn_destroy": (None, [_vp]),
    "sg_precond_apply_noalloc": (C.c_int, [_vp, _vp, _vp, C.c_double, _vp, _vp, _vp]),
    "newton_workspace_bytes": (C.c_size_t, [_vp, C.c_int, C.c_int, C.c_int]),
    "newton_solve": (C.c_int, [_vp, _i32p, C.c_int, C.c_int, C.c_int, C.c_int, _vp,
                               C.POINTER(NewtonOpts), C.POINTER(NewtonStats), _vp, C.c_size_t,
                               _vp]),
}

_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        # torch first: its HIP runtime is then the one the library binds to
        # (loading the library first brings in the system runtime, and torch
        # then finds no GPU)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


# ----------------------------------------------------------------- memory
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
_hooks = None          # the installed callbacks (kept alive while installed)


def memory_stats():
    """(live bytes the library holds, their peak, bytes cut from the arena)."""
    live, peak, used = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().sg_memory_stats(C.byref(live), C.byref(peak), C.byref(used)))
    return live.value, peak.value, used.value


def memory_reset_peak():
    _check(lib().sg_memory_reset_peak())


def use_torch_allocator(enable: bool = True):
    """Take the library's device memory from torch's caching allocator
    (torch.cuda.caching_allocator_alloc / _delete on the current stream), or
    go back to hipMalloc."""
    global _hooks
    if not enable:
        _check(lib().sg_set_allocator(None, None, None))
        _hooks = None
        return
    import torch

    def _alloc(nbytes, device, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device))
        except RuntimeError:
            return None

    def _free(ptr, nbytes, device, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(lib().sg_set_allocator(C.cast(hooks[0], _vp), C.cast(hooks[1], _vp), None))
    _hooks = hooks


class Arena:
    """Context manager: the library cuts its device memory from `buf` (a
    device tensor, caller-owned) while active; on exit arena mode ends (the
    handles made inside keep their memory, which stays valid as long as buf
    lives)."""

    def __init__(self, buf):
        self.buf = buf

    def __enter__(self):
        nbytes = self.buf.numel() * self.buf.element_size()
        _check(lib().sg_set_arena(C.c_void_p(self.buf.data_ptr()), nbytes))
        return self

    def used(self) -> int:
        return memory_stats()[2]

    def reset(self):
        _check(lib().sg_arena_reset())

    def __exit__(self, *exc):
        lib().sg_set_arena(None, 0)


def _check(rc: int) -> int:
    if rc < 0:
        raise SgError(rc, lib().sg_last_error().decode())
    return rc


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _dev(t) -> C.c_void_p:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _stream(stream=None) -> C.c_void_p:
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- basis
def sg_build_triples(M: int, p_in: int, p_out: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().sg_build_triples(M, p_in, p_out, C.byref(h)))
    return h


def sg_basis_info(b):
    P, L, T = C.c_int(), C.c_int(), C.c_int()
    _check(lib().sg_basis_info(b, C.byref(P), C.byref(L), C.byref(T)))
    return P.value, L.value, T.value


def sg_basis_export(b, M: int):
    P, L, T = sg_basis_info(b)
    alpha = np.zeros(P * max(M, 1), dtype=np.int32)
    ijk = np.zeros(T * 3, dtype=np.int32)
    val = np.zeros(T, dtype=np.float64)
    _check(lib().sg_basis_export(b, _ptr(alpha, C.c_int32), _ptr(ijk, C.c_int32),
                                 _ptr(val, C.c_double)))
    return alpha[:P * M].reshape(P, M), ijk.reshape(T, 3), val


def sg_destroy_basis(b):
    lib().sg_destroy_basis(b)


# ---------------------------------------------------------------- operator
def sg_assemble(basis, xy: np.ndarray, tri: np.ndarray, dof: np.ndarray, n: int,
                g0: np.ndarray, g: np.ndarray, stream=None) -> C.c_void_p:
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    dof = np.ascontiguousarray(dof, dtype=np.int32)
    g0 = np.ascontiguousarray(g0, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    h = C.c_void_p()
    gp = _ptr(g, C.c_double) if g.size else None
    _check(lib().sg_assemble(basis, xy.shape[0], _ptr(xy, C.c_double), tri.shape[0],
                             _ptr(tri, C.c_int32), _ptr(dof, C.c_int32), n,
                             _ptr(g0, C.c_double), gp, C.byref(h), _stream(stream)))
    return h


def sg_op_info(op):
    n, P, L, nnz = C.c_int(), C.c_int(), C.c_int(), C.c_int64()
    _check(lib().sg_op_info(op, C.byref(n), C.byref(P), C.byref(L), C.byref(nnz)))
    return n.value, P.value, L.value, nnz.value


def sg_op_rhs(op, B, stream=None):
    _check(lib().sg_op_rhs(op, _dev(B), _stream(stream)))


def sg_op_export(op):
    n, P, L, nnz = sg_op_info(op)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    vals = np.zeros(nnz * L, dtype=np.float64)
    _check(lib().sg_op_export(op, _ptr(rowptr, C.c_int64), _ptr(col, C.c_int32),
                              _ptr(vals, C.c_double)))
    return rowptr, col, vals.reshape(nnz, L)


def sg_destroy_op(op):
    lib().sg_destroy_op(op)


def sg_matvec(op, X, Y, stream=None):
    _check(lib().sg_matvec(op, _dev(X), _dev(Y), _stream(stream)))


MV_KERNELS = {0: "generic", 1: "wide", 2: "pair", 3: "staged", 4: "grouped", 5: "matrix_free",
              6: "row_tiled"}


def sg_matvec_matrix_free(op, enable: bool = True, stream=None):
    _check(lib().sg_matvec_matrix_free(op, 1 if enable else 0, _stream(stream)))


def sg_matvec_row_tiled(op, enable: bool = True):
    _check(lib().sg_matvec_row_tiled(op, 1 if enable else 0))


def sg_matvec_kernel(op) -> str:
    k = C.c_int()
    _check(lib().sg_matvec_kernel(op, C.byref(k)))
    return MV_KERNELS[k.value]


def sg_matvec_autotune(op, reps: int = 10, stream=None):
    """ms per launch for 1, 2 and 4 tiles per work-group (None: does not fit);
    the fastest is kept."""
    ms = np.zeros(3, dtype=np.float64)
    _check(lib().sg_matvec_autotune(op, reps, _ptr(ms, C.c_double), _stream(stream)))
    return [float(v) if v >= 0 else None for v in ms]


def sg_matvec_select(op, tiles: int):
    _check(lib().sg_matvec_select(op, tiles))


def sg_matvec_tiles(op) -> int:
    t = C.c_int()
    _check(lib().sg_matvec_tiles(op, C.byref(t)))
    return t.value


# ---------------------------------------------------------------- RAS
def ras_setup(op, owner: np.ndarray, n_sub: int, overlap: int, prec: int = SG_FP64,
              stream=None):
    owner = np.ascontiguousarray(owner, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().ras_setup(op, _ptr(owner, C.c_int32), n_sub, overlap, prec, C.byref(h),
                           _stream(stream)))
    return h


def ras_refactor(r, op, stream=None):
    _check(lib().ras_refactor(r, op, _stream(stream)))


RAS_PATHS = {"sweep": 0, "dense": 1, "dense32": 2, "fused": 3}


def ras_select(r, dense, stream=None):
    """dense: False/True (sweep / dense with 64 rows per wave) or a path name
    of RAS_PATHS."""
    path = RAS_PATHS[dense] if isinstance(dense, str) else (1 if dense else 0)
    _check(lib().ras_select(r, path, _stream(stream)))


def ras_autotune(r, reps: int = 5, stream=None):
    """ms per apply of the sweep, dense (64 rows per wave), dense32 and fused
    paths (-1 where the fused path does not fit); the fastest is kept."""
    ms = np.zeros(4, dtype=np.float64)
    _check(lib().ras_autotune(r, reps, _ptr(ms, C.c_double), _stream(stream)))
    return tuple(float(v) for v in ms)


def ras_path_info(r):
    """(dense in use, bytes of the dense rows, path name)."""
    d = C.c_int()
    nb = C.c_int64()
    _check(lib().ras_path_info(r, C.byref(d), C.byref(nb)))
    name = {v: k for k, v in RAS_PATHS.items()}[d.value]
    return d.value > 0, nb.value, name


def ras_info(r, n_sub: int):
    nloc = np.zeros(n_sub, dtype=np.int32)
    nlev = np.zeros(n_sub, dtype=np.int32)
    fb = C.c_int64()
    _check(lib().ras_info(r, _ptr(nloc, C.c_int32), _ptr(nlev, C.c_int32), C.byref(fb)))
    return nloc, nlev, fb.value


SG_LOCAL_MEAN, SG_LOCAL_KRON = 0, 1
LOCAL = {"mean": SG_LOCAL_MEAN, "kron": SG_LOCAL_KRON}


def ras_set_local(r, op, mode="mean", stream=None):
    """Local solves: "mean" (K_0 (x) G_0) or "kron" (K_0 (x) Gt, Ullmann)."""
    kind = LOCAL[mode] if isinstance(mode, str) else int(mode)
    _check(lib().ras_set_local(r, op, kind, _stream(stream)))


def ras_local_factor(r, P: int):
    gt = np.zeros(P * P, dtype=np.float64)
    _check(lib().ras_local_factor(r, _ptr(gt, C.c_double)))
    return gt.reshape(P, P)


def ras_apply(r, R, Z, stream=None):
    _check(lib().ras_apply(r, _dev(R), _dev(Z), _stream(stream)))


def sg_destroy_ras(r):
    lib().sg_destroy_ras(r)


# ---------------------------------------------------------------- coarse
def amg_setup(op, ras, kind: int = SG_COARSE_AMG, prec: int = SG_FP64, stream=None):
    h = C.c_void_p()
    _check(lib().amg_setup(op, ras, kind, prec, C.byref(h), _stream(stream)))
    return h


def amg_setup_geometric(op, ratio: int, owner_c, n_sub_c: int, overlap: int,
                        level_coarse: int = SG_COARSE_MEAN_EXACT, prec: int = SG_FP64,
                        rtol: float = 1e-5, max_its: int = 100, stream=None):
    """Geometric coarse space of the N x N lattice operator `op` with
    fine:coarse cell ratio `ratio`; owner_c partitions the coarse unknowns."""
    owner_c = np.ascontiguousarray(owner_c, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().amg_setup_geometric(op, int(ratio), _ptr(owner_c, C.c_int32), int(n_sub_c),
                                     int(overlap), int(level_coarse), int(prec), float(rtol),
                                     int(max_its), C.byref(h), _stream(stream)))
    return h


def amg_geometric_info(a):
    """(coarse unknowns, coarse pattern entries, coarse smoother damping)."""
    n, nnz, om = C.c_int(), C.c_int64(), C.c_double()
    _check(lib().amg_geometric_info(a, C.byref(n), C.byref(nnz), C.byref(om)))
    return n.value, nnz.value, om.value


def amg_geometric_op(a):
    """The coarse operator of a geometric handle (owned by it)."""
    h = lib().amg_geometric_op(a)
    if not h:
        raise SgError(-1, "not a geometric coarse space")
    return C.c_void_p(h)


def amg_info(a, n_sub: int):
    nl = C.c_int()
    nodes = np.zeros(8, dtype=np.int32)
    agg = np.zeros(n_sub, dtype=np.int32)
    _check(lib().amg_info(a, C.byref(nl), _ptr(nodes, C.c_int32), _ptr(agg, C.c_int32)))
    return nl.value, nodes[:nl.value], agg


def amg_level_blocks(a, level: int):
    """(operator, prolongator, restriction) P x P blocks stored on `level`."""
    ab, pb, rb = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().amg_level_blocks(a, level, C.byref(ab), C.byref(pb), C.byref(rb)))
    return ab.value, pb.value, rb.value


def amg_vcycle(a, b_c, x_c, stream=None):
    _check(lib().amg_vcycle(a, _dev(b_c), _dev(x_c), _stream(stream)))


SG_INNER_NONE, SG_INNER_GMRES_AMG, SG_INNER_GMRES_BJ = 0, 1, 2
INNER = {"none": SG_INNER_NONE, "gmres_amg": SG_INNER_GMRES_AMG, "gmres_bj": SG_INNER_GMRES_BJ}


def amg_set_inner(a, inner="none", rtol: float = 1e-5, max_its: int = 100):
    """inner: "none" (one V-cycle), "gmres_amg" (2GV3) or "gmres_bj" (2GV2)."""
    kind = INNER[inner] if isinstance(inner, str) else int(inner)
    _check(lib().amg_set_inner(a, kind, rtol, max_its))


def amg_inner_stats(a):
    """(inner solves, their total steps, steps of the last one)."""
    calls, its, last = C.c_int64(), C.c_int64(), C.c_int()
    _check(lib().amg_inner_stats(a, C.byref(calls), C.byref(its), C.byref(last)))
    return calls.value, its.value, last.value


def amg_coarse_solve(a, b_c, x_c, stream=None):
    _check(lib().amg_coarse_solve(a, _dev(b_c), _dev(x_c), _stream(stream)))


def sg_coarse_restrict(a, R, r_c, stream=None):
    _check(lib().sg_coarse_restrict(a, _dev(R), _dev(r_c), _stream(stream)))


def sg_coarse_prolong_add(a, e_c, Y, stream=None):
    _check(lib().sg_coarse_prolong_add(a, _dev(e_c), _dev(Y), _stream(stream)))


def sg_destroy_amg(a):
    lib().sg_destroy_amg(a)


# ---------------------------------------------------------------- solver
def sg_precond_workspace_bytes(op, amg) -> int:
    return int(lib().sg_precond_workspace_bytes(op, amg))


def sg_precond_apply(op, ras, amg, omega: float, R, Z, ws, stream=None):
    nbytes = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().sg_precond_apply(op, ras, amg, omega, _dev(R), _dev(Z), _dev(ws), nbytes,
                                  _stream(stream)))


SG_NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024


def sg_precond_apply_noalloc(op, ras, amg, omega: float, R, Z, stream=None):
    _check(lib().sg_precond_apply_noalloc(op, ras, amg, omega, _dev(R), _dev(Z),
                                          _stream(stream)))


def sg_smoother_damping(op, ras, its, ws, stream=None):
    rho, om = C.c_double(), C.c_double()
    _check(lib().sg_smoother_damping(op, ras, its, C.byref(rho), C.byref(om), _dev(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)))
    return rho.value, om.value


def fgmres_workspace_bytes(op, amg, restart: int) -> int:
    return int(lib().fgmres_workspace_bytes(op, amg, restart))


def sg_graph_cache_clear() -> int:
    return int(lib().sg_graph_cache_clear())


def fgmres_solve(op, ras, amg, b, x, restart: int, max_it: int, rtol: float, omega: float,
                 ws, history_cap: int = 4096, use_graph: bool = False, ortho: str = "mgs",
                 stream=None):
    opts = KrylovOpts(restart, max_it, rtol, omega, 1 if use_graph else 0, ORTHO[ortho])
    hist = np.zeros(history_cap, dtype=np.float64)
    st = KrylovStats()
    st.history = _ptr(hist, C.c_double)
    st.history_cap = history_cap
    rc = _check(lib().fgmres_solve(op, ras, amg, _dev(b), _dev(x), C.byref(opts), C.byref(st),
                                   _dev(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return dict(status=rc, iterations=st.iterations, restarts=st.restarts,
                converged=bool(st.converged), true_relres=st.true_relres, omega=st.omega,
                ms_solve=st.ms_solve, history=hist[:st.history_len].copy())


# ---------------------------------------------------------------- Newton
def sg_nl_setup(basis, xy: np.ndarray, tri: np.ndarray, dof: np.ndarray, n: int,
                g0: np.ndarray, g: np.ndarray, a2: float = 0.5, a1: float = 0.0,
                stream=None) -> C.c_void_p:
    """kappa(u) = 1 + a1 u + a2 u^2."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    dof = np.ascontiguousarray(dof, dtype=np.int32)
    g0 = np.ascontiguousarray(g0, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    h = C.c_void_p()
    gp = _ptr(g, C.c_double) if g.size else None
    _check(lib().sg_nl_setup(basis, xy.shape[0], _ptr(xy, C.c_double), tri.shape[0],
                             _ptr(tri, C.c_int32), _ptr(dof, C.c_int32), n,
                             _ptr(g0, C.c_double), gp, a1, a2, C.byref(h), _stream(stream)))
    return h


def sg_nl_info(nl):
    n, P, L2, nnz = C.c_int(), C.c_int(), C.c_int(), C.c_int64()
    _check(lib().sg_nl_info(nl, C.byref(n), C.byref(P), C.byref(L2), C.byref(nnz)))
    return n.value, P.value, L2.value, nnz.value


def sg_nl_eval(nl, U, R=None, stream=None):
    _check(lib().sg_nl_eval(nl, _dev(U), _dev(R), _stream(stream)))


def sg_nl_jac_apply(nl, X, Y, stream=None):
    _check(lib().sg_nl_jac_apply(nl, _dev(X), _dev(Y), _stream(stream)))


def sg_nl_export(nl):
    n, P, L2, nnz = sg_nl_info(nl)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    k1 = np.zeros(nnz * L2, dtype=np.float64)
    jac = np.zeros(nnz * L2, dtype=np.float64)
    _check(lib().sg_nl_export(nl, _ptr(rowptr, C.c_int64), _ptr(col, C.c_int32),
                              _ptr(k1, C.c_double), _ptr(jac, C.c_double)))
    return rowptr, col, k1.reshape(nnz, L2), jac.reshape(nnz, L2)


def sg_nl_mean_op(nl) -> C.c_void_p:
    return C.c_void_p(lib().sg_nl_mean_op(nl))


def sg_nl_jac_op(nl) -> C.c_void_p:
    return C.c_void_p(lib().sg_nl_jac_op(nl))


def sg_destroy_nl(nl):
    lib().sg_destroy_nl(nl)


def newton_workspace_bytes(nl, n_sub: int, coarse: int, restart: int) -> int:
    return int(lib().newton_workspace_bytes(nl, n_sub, coarse, restart))


def newton_solve(nl, owner: np.ndarray, n_sub: int, overlap: int, prec: int, coarse: int, U,
                 ws, max_steps: int = 30, tol: float = 1e-8, eta_max: float = 1e-2,
                 restart: int = 50, max_it: int = 1000, omega: float = 0.0,
                 use_graph: bool = False, history_cap: int = 64, ortho: str = "mgs",
                 amg_rebuild: int = 0, method: str = "newton", du_tol: float = 0.0,
                 ras_path: str = "sweep", stream=None):
    """method "newton" or "picard"; du_tol > 0 also stops on ||lambda d|| <= du_tol ||U||;
    ras_path "sweep", "dense", "dense32", "fused" or "auto" (ras_autotune at the
    first step)."""
    owner = np.ascontiguousarray(owner, dtype=np.int32)
    opts = NewtonOpts(max_steps, tol, eta_max, restart, max_it, omega, 1 if use_graph else 0,
                      ORTHO[ortho], amg_rebuild, NL_METHODS[method], du_tol,
                      NL_RAS_PATHS[ras_path])
    hist = np.zeros(history_cap, dtype=np.float64)
    kits = np.zeros(history_cap, dtype=np.int32)
    st = NewtonStats()
    st.history = _ptr(hist, C.c_double)
    st.krylov_its_per_step = _ptr(kits, C.c_int32)
    st.history_cap = history_cap
    rc = _check(lib().newton_solve(nl, _ptr(owner, C.c_int32), n_sub, overlap, prec, coarse,
                                   _dev(U), C.byref(opts), C.byref(st), _dev(ws),
                                   ws.numel() * ws.element_size(), _stream(stream)))
    h = st.history_len
    return dict(status=rc, steps=st.steps, krylov_its=st.krylov_its,
                converged=bool(st.converged), relres=st.relres, last_lambda=st.last_lambda,
                last_du=st.last_du,
                ms_total=st.ms_total, ms_eval=st.ms_eval, ms_setup=st.ms_setup,
                ms_krylov=st.ms_krylov, history=hist[:h].copy(),
                krylov_its_per_step=kits[:max(h - 1, 0)].copy())


def sg_nl_set_coefficients(nl, g0: np.ndarray, g: np.ndarray, stream=None):
    g0 = np.ascontiguousarray(g0, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    gp = _ptr(g, C.c_double) if g.size else None
    _check(lib().sg_nl_set_coefficients(nl, _ptr(g0, C.c_double), gp, _stream(stream)))


def newton_guess_workspace_bytes(nl) -> int:
    return int(lib().newton_guess_workspace_bytes(nl))


def newton_guess(nl, U_pred, U0, ws, stream=None):
    rel = np.zeros(3, dtype=np.float64)
    ch = C.c_int()
    _check(lib().newton_guess(nl, _dev(U_pred), _dev(U0), _ptr(rel, C.c_double), C.byref(ch),
                              _dev(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return ch.value, rel


# ---------------------------------------------------------------- learned predictor
def nn_create(channels, H: int, W: int, max_batch: int):
    ch = np.ascontiguousarray(channels, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().nn_create(len(ch) - 1, _ptr(ch, C.c_int32), H, W, max_batch, C.byref(h)))
    return h


def nn_param_count(nn) -> int:
    return int(lib().nn_param_count(nn))


def nn_set_params(nn, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == nn_param_count(nn)
    _check(lib().nn_set_params(nn, _ptr(p, C.c_float)))


def nn_get_params(nn):
    n = nn_param_count(nn)
    p = np.zeros(n, dtype=np.float32)
    g = np.zeros(n, dtype=np.float32)
    _check(lib().nn_get_params(nn, _ptr(p, C.c_float), _ptr(g, C.c_float)))
    return p, g


def nn_set_output_map(nn, env: np.ndarray, oscale: np.ndarray):
    e = np.ascontiguousarray(env, dtype=np.float32).ravel()
    o = np.ascontiguousarray(oscale, dtype=np.float32).ravel()
    _check(lib().nn_set_output_map(nn, _ptr(e, C.c_float), _ptr(o, C.c_float)))


def nn_fit_output_map(nn, shape, T, B: int, stream=None):
    _check(lib().nn_fit_output_map(nn, _dev(shape), _dev(T), B, _stream(stream)))


def nn_input_fields(npts: int, M: int, g0, g, X, stream=None):
    _check(lib().nn_input_fields(npts, M, _dev(g0), _dev(g) if M else None, _dev(X),
                                 _stream(stream)))


def nn_forward(nn, X, B: int, U, stream=None):
    _check(lib().nn_forward(nn, _dev(X), B, _dev(U), _stream(stream)))


def nn_loss_grad(nn, X, T, B: int, stream=None) -> float:
    loss = C.c_double()
    _check(lib().nn_loss_grad(nn, _dev(X), _dev(T), B, C.byref(loss), _stream(stream)))
    return loss.value


def nn_adam_step(nn, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 stream=None):
    _check(lib().nn_adam_step(nn, lr, beta1, beta2, eps, _stream(stream)))


def nn_destroy(nn):
    lib().nn_destroy(nn)
