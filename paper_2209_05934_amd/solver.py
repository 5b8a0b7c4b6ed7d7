"""Convenience layer over the C ABI: one object per context.

Matrices are block-sparse descriptions with the attributes row_bsz, col_bsz,
row_ptr, col_idx, val_off and val (the layout of omm_matrix).  Values may be
replaced by device tensors to hand the library device memory.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Any, List, Optional, Sequence

import numpy as np

from . import omm as L


@dataclass
class Problem:
    H: Any            # block-sparse H (unshifted)
    S: Any            # block-sparse S, same block structure
    C0: Any           # block-sparse initial guess (its pattern is kept fixed)
    n: int            # number of wavefunctions (columns of C)
    mode: int = L.OMM_DENSE
    eta: Optional[float] = None  # Kim shift of this system (None: the context option)
    n_occupied: Optional[int] = None  # occupied states when fewer than n (Kim); None: n
    T: Any = None      # kinetic matrix for preconditioning (dense, single system)
    tau: float = 0.0   # its scale tau_T (> 0 with T)
    T_val: Any = None
    H_val: Any = None  # optional device tensors replacing the host values
    S_val: Any = None
    C0_val: Any = None


def options(**kw) -> L.omm_options:
    o = L.omm_default_options()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k in ("tile_group", "tile_split"):
            v = (L.C.c_int32 * 3)(*v)
        setattr(o, k, v)
    return o


class Context:
    def __init__(self, problems: Sequence[Problem], **opts):
        self.problems = list(problems)
        self.opt = options(**opts)
        self._H = [L.BlockArgs.from_block_matrix(p.H, p.H_val) for p in self.problems]
        self._S = [L.BlockArgs.from_block_matrix(p.S, p.S_val) for p in self.problems]
        self.complex = any(np.iscomplexobj(p.H.val) for p in self.problems)
        if self.complex:    # k-points: complex Hermitian H, S (host values)
            etas = [self.opt.eta if p.eta is None else p.eta for p in self.problems]
            self.ctx = L.omm_init_complex(self._H, self._S, [p.n for p in self.problems],
                                          [p.mode for p in self.problems], etas, self.opt)
        elif len(self.problems) == 1:
            p = self.problems[0]
            if p.eta is not None:
                self.opt.eta = p.eta
            self.ctx = L.omm_init(self._H[0], self._S[0], p.n, p.mode, self.opt)
        else:
            etas = [self.opt.eta if p.eta is None else p.eta for p in self.problems]
            self.ctx = L.omm_init_batch(self._H, self._S, [p.n for p in self.problems],
                                        [p.mode for p in self.problems], etas, self.opt)
        for i, p in enumerate(self.problems):
            self.set_coeffs(i, p.C0, p.C0_val)
            if p.n_occupied is not None:
                L.omm_set_occupied(self.ctx, i, p.n_occupied)
            if p.T is not None:
                self._T = L.BlockArgs.from_block_matrix(p.T, p.T_val)
                L.omm_set_preconditioner(self.ctx, self._T, p.tau)

    @property
    def count(self) -> int:
        return len(self.problems)

    def set_coeffs(self, sys: int, C0, val=None) -> None:
        L.omm_set_coeffs(self.ctx, sys, L.BlockArgs.from_block_matrix(C0, val))

    def minimize(self):
        rc, reps = L.omm_minimize(self.ctx, self.count)
        return rc, reps

    def _host_out(self, size: int, out):
        # complex contexts return complex values: 2 doubles each, viewed as complex128
        if out is not None:
            return out, out
        if self.complex:
            buf = np.zeros(2 * size)
            return buf, buf.view(np.complex128)
        buf = np.zeros(size)
        return buf, buf

    def density_matrix(self, sys: int = 0, out=None) -> np.ndarray:
        buf, res = self._host_out(self.problems[sys].S.val.size, out)
        L.omm_density_matrix(self.ctx, sys, buf)
        return res

    def energy_density(self, sys: int = 0, out=None) -> np.ndarray:
        buf, res = self._host_out(self.problems[sys].S.val.size, out)
        L.omm_energy_density(self.ctx, sys, buf)
        return res

    def coeffs(self, sys: int = 0, out=None) -> np.ndarray:
        buf, res = self._host_out(self.problems[sys].C0.val.size, out)
        L.omm_get_coeffs(self.ctx, sys, buf)
        return res

    def projected(self, sys: int = 0):
        n = self.problems[sys].n
        if self.complex:
            HW, SW = np.zeros(2 * n * n), np.zeros(2 * n * n)
            L.omm_get_projected(self.ctx, sys, HW, SW)
            return HW.view(np.complex128).reshape(n, n), SW.view(np.complex128).reshape(n, n)
        HW, SW = np.zeros((n, n)), np.zeros((n, n))
        L.omm_get_projected(self.ctx, sys, HW, SW)
        return HW, SW

    def history(self, sys: int = 0, max_rows: int = 100000) -> np.ndarray:
        return L.omm_get_history(self.ctx, sys, max_rows)

    def sizes(self, sys: int = -1) -> L.omm_sizes:
        return L.omm_query(self.ctx, sys)

    def set_timing(self, on: bool) -> None:
        L.omm_set_timing(self.ctx, on)

    def kernel_times(self):
        return L.omm_kernel_times(self.ctx)

    def time_step(self, step: int, reps: int = 20) -> float:
        return L.omm_time_step(self.ctx, step, reps)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            L.omm_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def report_dict(r: L.omm_report) -> dict:
    return {k: getattr(r, k) for k, _ in r._fields_}
