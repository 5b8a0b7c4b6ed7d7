"""Thin ctypes binding of the C ABI in include/omm.h (argument marshalling only).

Every function keeps the C name and argument order; matrices are passed as
`BlockArgs` (host index arrays plus values that are either a numpy float64
array or a device tensor exposing `data_ptr()`).  All compute runs in the HIP
library; loading fails loudly when it has not been built.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Any, Optional, Sequence

import numpy as np

from .build import lib_path

OMM_OK, OMM_ERR_ARG, OMM_ERR_STATE, OMM_ERR_NOT_SPD, OMM_ERR_NO_LINE_MIN = 0, 1, 2, 3, 4
OMM_ERR_NOT_CONVERGED, OMM_ERR_ELECTRON_COUNT, OMM_ERR_DEVICE, OMM_ERR_OOM = 5, 6, 7, 8
OMM_DENSE, OMM_DENSE_CHOLESKY, OMM_BLOCK_SPARSE = 0, 1, 2
OMM_FP64, OMM_FP32, OMM_BF16 = 0, 1, 2
OMM_HOST, OMM_DEVICE = 0, 1
OMM_HISTORY_COLS = 11


class omm_matrix(C.Structure):
    _fields_ = [
        ("nbrow", C.c_int32), ("nbcol", C.c_int32),
        ("row_bsz", C.POINTER(C.c_int32)), ("col_bsz", C.POINTER(C.c_int32)),
        ("row_ptr", C.POINTER(C.c_int64)), ("col_idx", C.POINTER(C.c_int32)),
        ("val_off", C.POINTER(C.c_int64)), ("val", C.c_void_p),
        ("nval", C.c_int64), ("memspace", C.c_int32),
    ]


class omm_options(C.Structure):
    _fields_ = [
        ("eta", C.c_double), ("tol_grad", C.c_double), ("rel_tol", C.c_double),
        ("max_iter", C.c_int64), ("filter_eps", C.c_double), ("precision", C.c_int32),
        ("fp64_refine_iters", C.c_int32), ("lowprec_rel_switch", C.c_double),
        ("lowprec_max_iter", C.c_int64), ("graph_iters", C.c_int32), ("history", C.c_int32),
        ("history_max", C.c_int32), ("ne_tol", C.c_double), ("autotune", C.c_int32),
        ("tune_cache", C.c_char_p), ("hip_stream", C.c_void_p),
        ("tile_group", C.c_int32 * 3), ("tile_split", C.c_int32 * 3), ("log_jsonl_path", C.c_char_p),
    ]


class omm_report(C.Structure):
    _fields_ = [
        ("energy", C.c_double), ("energy_band", C.c_double), ("grad_norm", C.c_double),
        ("electron_count", C.c_double), ("iters_total", C.c_int64), ("iters_fp64", C.c_int64),
        ("cg_restarts", C.c_int64), ("status", C.c_int32), ("precision_end", C.c_int32),
        ("seconds", C.c_double),
    ]


class omm_sizes(C.Structure):
    _fields_ = [
        ("m", C.c_int64), ("n", C.c_int64), ("s_nval", C.c_int64), ("c_nval", C.c_int64),
        ("tiles_h", C.c_int64), ("tiles_c", C.c_int64), ("tiles_hc", C.c_int64), ("tiles_w", C.c_int64),
        ("pairs_s1", C.c_int64), ("pairs_s2", C.c_int64), ("pairs_grad", C.c_int64),
        ("flops_alg_iter", C.c_double), ("flops_exec_iter", C.c_double), ("bytes_alg_iter", C.c_double),
        ("flops_alg_step", C.c_double * 3), ("flops_exec_step", C.c_double * 3),
        ("bytes_alg_step", C.c_double * 3), ("tile_group", C.c_int32 * 3), ("tile_split", C.c_int32 * 3),
    ]


_lib: Optional[C.CDLL] = None


def load(path: Optional[str] = None) -> C.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or os.environ.get("OMM_LIBRARY") or lib_path()
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is missing; run paper_2209_05934_amd.build.build() first")
    lib = C.CDLL(p)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    MP = C.POINTER(omm_matrix)
    sig = {
        "omm_default_options": (None, [C.POINTER(omm_options)]),
        "omm_init": (I32, [C.POINTER(P), MP, MP, I64, I32, C.POINTER(omm_options)]),
        "omm_init_batch": (I32, [C.POINTER(P), I32, MP, MP, C.POINTER(I64), C.POINTER(I32),
                                 C.POINTER(D), C.POINTER(omm_options)]),
        "omm_init_complex": (I32, [C.POINTER(P), I32, MP, MP, C.POINTER(I64), C.POINTER(I32),
                                   C.POINTER(D), C.POINTER(omm_options)]),
        "omm_set_coeffs": (I32, [P, I32, MP]),
        "omm_minimize": (I32, [P, C.POINTER(omm_report)]),
        "omm_batch_minimize": (I32, [C.POINTER(P), I32, C.POINTER(omm_report)]),
        "omm_density_matrix": (I32, [P, I32, P, I32]),
        "omm_density_matrix_noalloc": (I32, [P, I32, P]),
        "omm_energy_density": (I32, [P, I32, P, I32]),
        "omm_set_occupied": (I32, [P, I32, I64]),
        "omm_set_preconditioner": (I32, [P, MP, D]),
        "omm_update_hs": (I32, [P, I32, MP, MP]),
        "omm_remap_coeffs": (I32, [MP, MP, MP, P]),
        "omm_write_coeffs": (I32, [C.c_char_p, MP]),
        "omm_read_coeffs": (I32, [C.c_char_p, MP, P]),
        "omm_get_coeffs": (I32, [P, I32, P, I32]),
        "omm_get_projected": (I32, [P, I32, P, P, I32]),
        "omm_get_history": (I32, [P, I32, P, I64, C.POINTER(I64)]),
        "omm_query": (I32, [P, I32, C.POINTER(omm_sizes)]),
        "omm_set_timing": (I32, [P, I32]),
        "omm_kernel_times": (I32, [P, C.POINTER(D), C.POINTER(I64)]),
        "omm_time_step": (I32, [P, I32, I32, C.POINTER(D)]),
        "omm_status_str": (C.c_char_p, [I32]),
        "omm_last_error": (C.c_char_p, [P]),
        "omm_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


EXPORTED = ("omm_default_options", "omm_init", "omm_init_batch", "omm_init_complex", "omm_set_coeffs", "omm_minimize",
            "omm_batch_minimize",
            "omm_density_matrix", "omm_density_matrix_noalloc", "omm_energy_density", "omm_get_coeffs", "omm_get_projected",
            "omm_get_history", "omm_query", "omm_set_occupied", "omm_set_preconditioner", "omm_update_hs",
            "omm_remap_coeffs", "omm_write_coeffs", "omm_read_coeffs", "omm_set_timing", "omm_kernel_times", "omm_time_step",
            "omm_status_str", "omm_last_error", "omm_destroy")


class OmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{omm_status_str(status)}: {msg}")
        self.status = status


# ------------------------------------------------------------------ marshalling helpers
def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class BlockArgs:
    """Keeps the host index arrays alive and exposes an omm_matrix struct."""

    def __init__(self, row_bsz, col_bsz, row_ptr, col_idx, val_off, val: Any):
        self.row_bsz = np.ascontiguousarray(row_bsz, dtype=np.int32)
        self.col_bsz = np.ascontiguousarray(col_bsz, dtype=np.int32)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.val_off = np.ascontiguousarray(val_off, dtype=np.int64)
        if isinstance(val, np.ndarray) and np.iscomplexobj(val):   # complex: interleaved (re, im) doubles
            self.val = np.ascontiguousarray(val, dtype=np.complex128).view(np.float64)
            vptr, nval, space = self.val.ctypes.data, self.val.size // 2, OMM_HOST
        elif isinstance(val, np.ndarray):
            self.val = np.ascontiguousarray(val, dtype=np.float64)
            vptr, nval, space = self.val.ctypes.data, self.val.size, OMM_HOST
        else:   # device tensor
            self.val = val
            vptr, nval, space = int(val.data_ptr()), int(val.numel()), OMM_DEVICE
        self.struct = omm_matrix(
            int(self.row_bsz.size), int(self.col_bsz.size), _ptr(self.row_bsz, C.c_int32),
            _ptr(self.col_bsz, C.c_int32), _ptr(self.row_ptr, C.c_int64), _ptr(self.col_idx, C.c_int32),
            _ptr(self.val_off, C.c_int64), C.c_void_p(vptr), int(nval), space)

    @classmethod
    def from_block_matrix(cls, bm, val=None) -> "BlockArgs":
        return cls(bm.row_bsz, bm.col_bsz, bm.row_ptr, bm.col_idx, bm.val_off, bm.val if val is None else val)


def _addr(buf) -> tuple:
    if isinstance(buf, np.ndarray):
        assert buf.dtype == np.float64 and buf.flags["C_CONTIGUOUS"]
        return buf.ctypes.data, OMM_HOST
    return int(buf.data_ptr()), OMM_DEVICE


# ------------------------------------------------------------------ C-named wrappers
def omm_default_options() -> omm_options:
    o = omm_options()
    load().omm_default_options(C.byref(o))
    return o


def omm_status_str(status: int) -> str:
    return load().omm_status_str(int(status)).decode()


def omm_last_error(ctx) -> str:
    return load().omm_last_error(ctx).decode()


def _check(ctx, rc: int, soft_ok: bool = False) -> int:
    if rc == OMM_OK:
        return rc
    if soft_ok and rc in (OMM_ERR_NOT_CONVERGED, OMM_ERR_ELECTRON_COUNT):
        return rc
    raise OmmError(rc, omm_last_error(ctx))


def omm_init(H: BlockArgs, S: BlockArgs, n_occ: int, mode: int, opt: Optional[omm_options] = None):
    ctx = C.c_void_p()
    rc = load().omm_init(C.byref(ctx), C.byref(H.struct), C.byref(S.struct), int(n_occ), int(mode),
                         C.byref(opt) if opt is not None else None)
    _check(None, rc)
    return ctx


def omm_init_batch(Hs: Sequence[BlockArgs], Ss: Sequence[BlockArgs], n_occ: Sequence[int],
                   modes: Sequence[int], etas: Optional[Sequence[float]] = None,
                   opt: Optional[omm_options] = None):
    count = len(Hs)
    Harr = (omm_matrix * count)(*[h.struct for h in Hs])
    Sarr = (omm_matrix * count)(*[s.struct for s in Ss])
    narr = (C.c_int64 * count)(*[int(v) for v in n_occ])
    marr = (C.c_int32 * count)(*[int(v) for v in modes])
    earr = (C.c_double * count)(*[float(v) for v in etas]) if etas is not None else None
    ctx = C.c_void_p()
    rc = load().omm_init_batch(C.byref(ctx), count, Harr, Sarr, narr, marr, earr,
                               C.byref(opt) if opt is not None else None)
    _check(None, rc)
    return ctx


def omm_init_complex(Hs: Sequence[BlockArgs], Ss: Sequence[BlockArgs], n_occ: Sequence[int],
                     modes: Sequence[int], etas: Optional[Sequence[float]] = None,
                     opt: Optional[omm_options] = None):
    """Complex Hermitian systems (BlockArgs over complex128 values, host memory)."""
    count = len(Hs)
    Harr = (omm_matrix * count)(*[h.struct for h in Hs])
    Sarr = (omm_matrix * count)(*[s.struct for s in Ss])
    narr = (C.c_int64 * count)(*[int(v) for v in n_occ])
    marr = (C.c_int32 * count)(*[int(v) for v in modes])
    earr = (C.c_double * count)(*[float(v) for v in etas]) if etas is not None else None
    ctx = C.c_void_p()
    rc = load().omm_init_complex(C.byref(ctx), count, Harr, Sarr, narr, marr, earr,
                                 C.byref(opt) if opt is not None else None)
    _check(None, rc)
    return ctx


def omm_set_coeffs(ctx, sys: int, C0: BlockArgs) -> int:
    return _check(ctx, load().omm_set_coeffs(ctx, int(sys), C.byref(C0.struct)))


def omm_minimize(ctx, count: int = 1, soft_ok: bool = True):
    reps = (omm_report * count)()
    rc = load().omm_minimize(ctx, reps)
    _check(ctx, rc, soft_ok=soft_ok)
    return rc, list(reps)


def omm_batch_minimize(ctxs, counts, soft_ok: bool = True):
    """ctxs: context handles; counts: systems of each (for the report array)."""
    arr = (C.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    reps = (omm_report * int(sum(counts)))()
    rc = load().omm_batch_minimize(arr, len(ctxs), reps)
    _check(ctxs[0], rc, soft_ok=soft_ok)
    return rc, list(reps)


def omm_density_matrix(ctx, sys: int, out) -> int:
    p, where = _addr(out)
    return _check(ctx, load().omm_density_matrix(ctx, int(sys), C.c_void_p(p), where))


def omm_density_matrix_noalloc(ctx, sys: int, out) -> int:
    """out: a device tensor of s_nval doubles."""
    p, where = _addr(out)
    if where != OMM_DEVICE:
        raise ValueError("omm_density_matrix_noalloc writes device memory only")
    return _check(ctx, load().omm_density_matrix_noalloc(ctx, int(sys), C.c_void_p(p)))


def omm_set_occupied(ctx, sys: int, n_occupied: int) -> int:
    return _check(ctx, load().omm_set_occupied(ctx, int(sys), int(n_occupied)))


def omm_set_preconditioner(ctx, T, tau: float) -> int:
    """T: BlockArgs of the kinetic matrix (None removes the preconditioner)."""
    ref = C.byref(T.struct) if T is not None else None
    return _check(ctx, load().omm_set_preconditioner(ctx, ref, float(tau)))


def omm_update_hs(ctx, sys: int, H, S) -> int:
    """H, S: BlockArgs with the new values on the structure given at init."""
    return _check(ctx, load().omm_update_hs(ctx, int(sys), C.byref(H.struct), C.byref(S.struct)))


def _host_call(rc: int) -> int:
    if rc != OMM_OK:
        raise OmmError(rc, omm_last_error(None))
    return rc


def omm_remap_coeffs(cur, prev, to):
    """Guess on pattern `to` from `cur` (and linear extrapolation with `prev`); block matrices in host memory."""
    a, b, t = (BlockArgs.from_block_matrix(m) if m is not None else None for m in (cur, prev, to))
    out = np.zeros(to.val.size)
    _host_call(load().omm_remap_coeffs(C.byref(a.struct), C.byref(b.struct) if b else None, C.byref(t.struct),
                                       out.ctypes.data))
    return out


def omm_write_coeffs(path: str, Cm) -> None:
    a = BlockArgs.from_block_matrix(Cm)
    _host_call(load().omm_write_coeffs(os.fsencode(path), C.byref(a.struct)))


def omm_read_coeffs(path: str, to):
    t = BlockArgs.from_block_matrix(to)
    out = np.zeros(to.val.size)
    _host_call(load().omm_read_coeffs(os.fsencode(path), C.byref(t.struct), out.ctypes.data))
    return out


def omm_energy_density(ctx, sys: int, out) -> int:
    p, where = _addr(out)
    return _check(ctx, load().omm_energy_density(ctx, int(sys), C.c_void_p(p), where))


def omm_get_coeffs(ctx, sys: int, out) -> int:
    p, where = _addr(out)
    return _check(ctx, load().omm_get_coeffs(ctx, int(sys), C.c_void_p(p), where))


def omm_get_projected(ctx, sys: int, HW, SW) -> int:
    ph, where = _addr(HW)
    ps, _ = _addr(SW)
    return _check(ctx, load().omm_get_projected(ctx, int(sys), C.c_void_p(ph), C.c_void_p(ps), where))


def omm_get_history(ctx, sys: int, max_rows: int) -> np.ndarray:
    out = np.zeros((max(1, max_rows), OMM_HISTORY_COLS))
    rows = C.c_int64(0)
    _check(ctx, load().omm_get_history(ctx, int(sys), C.c_void_p(out.ctypes.data), int(max_rows),
                                       C.byref(rows)))
    return out[:rows.value]


def omm_query(ctx, sys: int = -1) -> omm_sizes:
    z = omm_sizes()
    _check(ctx, load().omm_query(ctx, int(sys), C.byref(z)))
    return z


def omm_set_timing(ctx, enable: bool) -> int:
    return _check(ctx, load().omm_set_timing(ctx, 1 if enable else 0))


def omm_kernel_times(ctx):
    ms = (C.c_double * 3)()
    n = (C.c_int64 * 3)()
    _check(ctx, load().omm_kernel_times(ctx, ms, n))
    return list(ms), list(n)


def omm_time_step(ctx, step: int, reps: int = 20) -> float:
    """Average milliseconds of one launch of product step `step` (see omm.h)."""
    v = C.c_double()
    _check(ctx, load().omm_time_step(ctx, int(step), int(reps), C.byref(v)))
    return v.value


def omm_destroy(ctx) -> None:
    if ctx:
        load().omm_destroy(ctx)
