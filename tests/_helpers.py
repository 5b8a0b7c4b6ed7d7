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


def hetero_system(seed: int = 9):
    """A 27-atom system whose atoms carry 13, 9 or 5 orbitals (heterogeneous atom
    blocks): the 13-orbital lattice with the last orbitals of some atoms removed
    (rows and columns dropped from H and S, which stay symmetric and positive
    definite), 2 wavefunctions per atom, C localized to radius 1.2 (block pattern
    of the full lattice).  Returns (H, S, C0) as BlockMatrix plus the block sizes."""
    from types import SimpleNamespace
    from ommgen.systems import BlockMatrix
    base = system("cubic3_sparse")
    N, norb, nwf = base.natoms, base.spec.norb, base.spec.wf_per_atom
    sizes = np.array([13, 9, 5])[np.arange(N) % 3].astype(np.int32)
    keep = np.concatenate([a * norb + np.arange(sizes[a]) for a in range(N)])
    H = base.H.to_dense()[np.ix_(keep, keep)]
    S = base.S.to_dense()[np.ix_(keep, keep)]
    C0 = base.C0.to_dense()[keep]
    cpat = np.zeros((N, N), dtype=bool)
    cpat[base.C0.block_rows(), base.C0.col_idx] = True
    hpat = np.zeros((N, N), dtype=bool)
    hpat[base.H.block_rows(), base.H.col_idx] = True

    def pack(A, rbs, cbs, pat):
        ro = np.concatenate([[0], np.cumsum(rbs)])
        co = np.concatenate([[0], np.cumsum(cbs)])
        rp, ci, vo, vals, off = [0], [], [], [], 0
        for i in range(len(rbs)):
            for j in np.nonzero(pat[i])[0]:
                blk = A[ro[i]:ro[i + 1], co[j]:co[j + 1]]
                ci.append(j)
                vo.append(off)
                vals.append(blk.ravel())
                off += blk.size
            rp.append(len(ci))
        return BlockMatrix(row_bsz=np.asarray(rbs, np.int32), col_bsz=np.asarray(cbs, np.int32),
                           row_ptr=np.asarray(rp, np.int64), col_idx=np.asarray(ci, np.int32),
                           val_off=np.asarray(vo, np.int64), val=np.concatenate(vals))

    wbs = np.full(N, nwf, np.int32)
    return SimpleNamespace(H=pack(H, sizes, sizes, hpat), S=pack(S, sizes, sizes, hpat),
                           C0=pack(C0, sizes, wbs, cpat), n=N * nwf, natoms=N, eta=base.spec.eta,
                           row_blocks=sizes, col_blocks=wbs, m=int(sizes.sum()))
