"""Shared helpers of the GPU parity tests: run the library and the oracle on one input."""

from __future__ import annotations

from dataclasses import replace

import numpy as np

import oracle as O
from ommgen import config_spec, make_system
from ommgen.systems import SystemSpec, cubic_spec


def system(name: str, **kw):
    if name == "cubic3_dense":
        sp = cubic_spec(3, 31, dense=True)
    elif name == "cubic3_sparse":          # converges fully in ~1.8k iterations
        sp = replace(cubic_spec(3, 11, dense=False), rc=1.2, eta=0.0, filter_eps=0.0)
    elif name == "cubic5_sparse":          # localized, 125 atoms, radius 1.5
        sp = replace(cubic_spec(5, 77, dense=False), rc=1.5, filter_eps=0.0)
    elif name == "chain12_sparse":
        sp = SystemSpec("chain12", (12,), 4, 2, (-1.0, -1.0, 1.0, 1.0), seed=21, rc=1.5, dense=False)
    else:
        sp = config_spec(name)
    if kw:
        sp = replace(sp, **kw)
    return make_system(sp)


def oracle_run(s, mode: str, **kw):
    H, S, C0 = s.H.to_dense(), s.S.to_dense(), s.C0.to_dense()
    kw.setdefault("eta", s.spec.eta)
    if mode == "cholesky":
        return O.cg_minimize_cholesky(H, S, C0, **kw)
    mask = None if mode == "dense" else s.C0.pattern_mask()
    if mode == "sparse" and s.spec.filter_eps > 0 and "filter_eps" not in kw:
        kw["filter_eps"] = 0.0
    return O.cg_minimize(H, S, C0, mask=mask, row_blocks=[s.spec.norb] * s.natoms,
                         col_blocks=[s.spec.wf_per_atom] * s.natoms, **kw)


def rho_values(s, res):
    return s.S.gather_from_dense(O.density_matrix(res.C, res.SW))


def c_values(s, res):
    return s.C0.gather_from_dense(res.C)


def history_array(res) -> np.ndarray:
    rows = [[h["E"], *h["c"], h["x"], h["gnorm"], h["beta"], float(h["restart"])] for h in res.history]
    return np.array(rows) if rows else np.zeros((0, 10))
