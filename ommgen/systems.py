"""Synthetic tight-binding-like systems in atom-block sparse (BCSR) form.

Model (a stand-in for the DZP boron-nitride Hamiltonians of the paper's tests,
Sec. IV A, which are not available): atoms on a jittered periodic lattice, each
carrying `norb` orbitals and hosting `wf_per_atom` localized wavefunctions.

* on-site block:  H_II = diag(eps) + symmetric N(0, onsite_noise) noise,  S_II = I
* pair (I, J) within `cutoff` (summed over periodic images n, each with its own
  N(0,1) matrices G, Q):
      H_IJ = sum_n hop * exp(-r_n / decay) * G^(n)
      S_IJ = sum_n ovl * exp(-r_n / decay) * Q^(n)
  with H_JI = H_IJ^T and S_JI = S_IJ^T, so both matrices are symmetric.
* the wavefunctions of atom a may expand only on basis atoms b with minimum-image
  distance |R_b - R_a| <= rc (inclusive); rc = None means no localization
  (dense C).
* C0 ~ N(0, sigma^2) inside that pattern with sigma = 0.1 * sqrt(32 / nnz_col),
  nnz_col being the mean number of stored entries per column of C.

All random numbers come from numpy's PCG64 generator seeded with `seed`
(geometry, on-site noise, then G and Q for the pair-image list in sorted
(I, J, image) order) and with `seed + 10**6` for C0, so the output depends only
on the spec.  Atoms of 3D lattices are listed in 2x2x2-brick order (bricks
lexicographic, atoms lexicographic inside a brick) so that consecutive atoms
are spatial neighbours; this is an input ordering choice, like the paper's
remark that block division can follow the chemistry (Sec. IV B, Fig. 7).
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np


# --------------------------------------------------------------------------
# atom-block BCSR container
# --------------------------------------------------------------------------
@dataclass
class BlockMatrix:
    """Atom-block compressed sparse row matrix with row-major dense blocks.

    row_bsz[i], col_bsz[j]  block sizes
    row_ptr[i]..row_ptr[i+1]  the stored blocks of block row i (int64)
    col_idx[k]               block column of stored block k (int32, sorted per row)
    val_off[k]               offset of block k's row-major values in `val` (int64)
    val                      float64 values
    """

    row_bsz: np.ndarray
    col_bsz: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val_off: np.ndarray
    val: np.ndarray

    @property
    def nbrow(self) -> int:
        return int(self.row_bsz.shape[0])

    @property
    def nbcol(self) -> int:
        return int(self.col_bsz.shape[0])

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def shape(self) -> Tuple[int, int]:
        return int(self.row_bsz.sum()), int(self.col_bsz.sum())

    def row_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.row_bsz)]).astype(np.int64)

    def col_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.col_bsz)]).astype(np.int64)

    def block_rows(self) -> np.ndarray:
        """Block-row index of every stored block."""
        return np.repeat(np.arange(self.nbrow, dtype=np.int64), np.diff(self.row_ptr))

    def block(self, k: int) -> np.ndarray:
        i = int(self.block_rows()[k]) if self.nbrow > 1 else 0
        r, c = int(self.row_bsz[i]), int(self.col_bsz[self.col_idx[k]])
        o = int(self.val_off[k])
        return self.val[o:o + r * c].reshape(r, c)

    def to_dense(self) -> np.ndarray:
        ro, co = self.row_offsets(), self.col_offsets()
        out = np.zeros((int(ro[-1]), int(co[-1])), dtype=self.val.dtype)
        rows = self.block_rows()
        for k in range(self.nnzb):
            i, j = int(rows[k]), int(self.col_idx[k])
            r, c = int(self.row_bsz[i]), int(self.col_bsz[j])
            o = int(self.val_off[k])
            out[ro[i]:ro[i] + r, co[j]:co[j] + c] = self.val[o:o + r * c].reshape(r, c)
        return out

    def pattern_mask(self) -> np.ndarray:
        """Boolean element mask of the stored blocks (dense shape)."""
        ro, co = self.row_offsets(), self.col_offsets()
        out = np.zeros((int(ro[-1]), int(co[-1])), dtype=bool)
        rows = self.block_rows()
        for k in range(self.nnzb):
            i, j = int(rows[k]), int(self.col_idx[k])
            out[ro[i]:ro[i + 1], co[j]:co[j + 1]] = True
        return out

    def to_bsr(self):
        """scipy.sparse BSR matrix of the same blocks (uniform block sizes only)."""
        import scipy.sparse
        rb, cb = int(self.row_bsz[0]), int(self.col_bsz[0])
        if np.any(self.row_bsz != rb) or np.any(self.col_bsz != cb):
            raise ValueError("BSR needs uniform block sizes")
        idx = self.val_off[:, None] + np.arange(rb * cb)[None, :]
        data = self.val[idx].reshape(self.nnzb, rb, cb)
        return scipy.sparse.bsr_matrix((data, self.col_idx.astype(np.int32), self.row_ptr.astype(np.int32)),
                                       shape=self.shape)

    def with_values(self, val: np.ndarray) -> "BlockMatrix":
        return replace(self, val=np.ascontiguousarray(
            val, dtype=np.complex128 if np.iscomplexobj(val) else np.float64))

    def gather_from_dense(self, A: np.ndarray) -> np.ndarray:
        """Values of dense A on this matrix's block pattern, in `val` layout."""
        ro, co = self.row_offsets(), self.col_offsets()
        out = np.zeros(self.val.shape, dtype=np.result_type(self.val, A))
        rows = self.block_rows()
        for k in range(self.nnzb):
            i, j = int(rows[k]), int(self.col_idx[k])
            r, c = int(self.row_bsz[i]), int(self.col_bsz[j])
            o = int(self.val_off[k])
            out[o:o + r * c] = A[ro[i]:ro[i] + r, co[j]:co[j] + c].ravel()
        return out


def _uniform_bcsr(nbrow: int, nbcol: int, rb: int, cb: int,
                  rows: np.ndarray, cols: np.ndarray, blocks: np.ndarray) -> BlockMatrix:
    """BCSR from (row, col, block) triples; triples must be sorted by (row, col)."""
    nnzb = rows.shape[0]
    row_ptr = np.zeros(nbrow + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return BlockMatrix(
        row_bsz=np.full(nbrow, rb, dtype=np.int32),
        col_bsz=np.full(nbcol, cb, dtype=np.int32),
        row_ptr=row_ptr.astype(np.int64),
        col_idx=cols.astype(np.int32),
        val_off=(np.arange(nnzb, dtype=np.int64) * rb * cb),
        val=np.ascontiguousarray(blocks.reshape(-1),
                                 dtype=np.complex128 if np.iscomplexobj(blocks) else np.float64),
    )


# --------------------------------------------------------------------------
# specs
# --------------------------------------------------------------------------
@dataclass
class SystemSpec:
    name: str
    dims: Tuple[int, ...]          # lattice size per periodic dimension (1D chain: (8,))
    norb: int                      # orbitals per atom
    wf_per_atom: int               # localized wavefunctions hosted per atom
    onsite: Tuple[float, ...]      # on-site energies (len norb)
    seed: int
    rc: Optional[float] = None     # C localization radius; None = dense C
    eta: float = 0.0               # Kim shift used by runs of this system
    filter_eps: float = 0.0        # product filter threshold used by runs
    dense: bool = True             # solve in dense (cubic-scaling) form
    spacing: float = 1.0
    jitter: float = 0.05
    cutoff: float = 2.5
    hop: float = 0.1
    ovl: float = 0.05
    decay: float = 0.8
    onsite_noise: float = 0.02
    c0_scale: float = 0.1
    c0_ref_nnz: float = 32.0
    occ_per_atom: int = 2          # occupied states per atom (the two low on-site levels)
    kinetic: float = 0.0           # > 0: add a kinetic matrix T (largest level `kinetic`) to H

    @property
    def natoms(self) -> int:
        return int(np.prod(self.dims))

    @property
    def m(self) -> int:
        return self.natoms * self.norb

    @property
    def n(self) -> int:
        return self.natoms * self.wf_per_atom

    @property
    def n_occupied(self) -> int:
        return self.natoms * self.occ_per_atom


def _onsite13() -> Tuple[float, ...]:
    return tuple([-1.0] * 2 + [1.0] * 11)


CONFIG_NAMES = ("chain8", "cubic4_dense", "cubic8_sparse", "cubic16_mixed", "batch64", "cubic8_kim")

# Kim shift inside the gap of the 13-orbital lattices (occupied levels end near
# -0.76, empty ones start near +0.30)
KIM_ETA13 = -0.25


def config_spec(name: str, **overrides) -> SystemSpec:
    """Specs of the named workloads (the batch is built by `batch_specs`)."""
    if name == "chain8":   # periodic 1D chain, 8 atoms x 4 orbitals, dense, eta = 0
        spec = SystemSpec(name, (8,), 4, 2, (-1.0, -1.0, 1.0, 1.0), seed=1)
    elif name == "cubic4_dense":  # 4^3 atoms x 13 orbitals, dense, eta = 0
        spec = SystemSpec(name, (4, 4, 4), 13, 2, _onsite13(), seed=2)
    elif name == "cubic8_sparse":  # 8^3 x 13, rc = 3.0, eta = 1.5, filter 1e-6
        spec = SystemSpec(name, (8, 8, 8), 13, 2, _onsite13(), seed=3, rc=3.0,
                          eta=1.5, filter_eps=1e-6, dense=False)
    elif name == "cubic16_mixed":  # 16^3 x 13, same recipe as cubic8_sparse
        spec = SystemSpec(name, (16, 16, 16), 13, 2, _onsite13(), seed=4, rc=3.0,
                          eta=1.5, filter_eps=1e-6, dense=False)
    elif name == "cubic8_kim":     # 8^3 x 13, 3 wavefunctions per atom for 2 occupied states
        spec = SystemSpec(name, (8, 8, 8), 13, 3, _onsite13(), seed=6, rc=3.0,
                          eta=KIM_ETA13, filter_eps=1e-6, dense=False)
    else:
        raise ValueError(f"unknown config {name!r}")
    return replace(spec, **overrides) if overrides else spec


def cubic_spec(nside: int, seed: int, dense: bool, name: str = "") -> SystemSpec:
    """n^3 x 13 system: dense (eta 0, unlocalized) or sparse (rc 3, eta 1.5, eps 1e-6)."""
    if dense:
        return SystemSpec(name or f"cubic{nside}_dense", (nside,) * 3, 13, 2, _onsite13(), seed)
    return SystemSpec(name or f"cubic{nside}_sparse", (nside,) * 3, 13, 2, _onsite13(), seed,
                      rc=3.0, eta=1.5, filter_eps=1e-6, dense=False)


def batch_specs(count: int = 64, seed: int = 5, nmin: int = 3, nmax: int = 7) -> List[SystemSpec]:
    """`count` uneven systems: lattice side uniform in [nmin, nmax], half dense, half sparse.

    System k has its own generator seed 5000 + k; sizes are drawn from a PCG64
    stream seeded with `seed`.
    """
    rng = np.random.default_rng(seed)
    sides = rng.integers(nmin, nmax + 1, size=count)
    specs = []
    for k in range(count):
        specs.append(cubic_spec(int(sides[k]), 5000 + k, dense=(k < count // 2),
                                name=f"batch{k}"))
    return specs


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def _lattice_points(dims: Sequence[int]) -> np.ndarray:
    """Integer lattice points, 2x2x2-brick order for 3D, natural order otherwise."""
    if len(dims) == 1:
        return np.arange(dims[0], dtype=np.int64)[:, None]
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    key = np.lexsort((pts[:, 0] % 2, pts[:, 1] % 2, pts[:, 2] % 2,
                      pts[:, 0] // 2, pts[:, 1] // 2, pts[:, 2] // 2))
    return pts[key]


@dataclass
class System:
    spec: SystemSpec
    pos: np.ndarray          # (natoms, dim)
    box: np.ndarray          # periodic lengths (dim,)
    H: BlockMatrix           # unshifted Hamiltonian, norb x norb blocks
    S: BlockMatrix           # overlap, same block pattern as H
    C0: BlockMatrix          # initial guess on the C pattern (norb x wf blocks)
    pair_images: int = 0
    T: Optional[BlockMatrix] = None   # kinetic matrix (already part of H), when spec.kinetic > 0
    extra: dict = field(default_factory=dict)

    @property
    def natoms(self) -> int:
        return self.spec.natoms

    @property
    def m(self) -> int:
        return self.spec.m

    @property
    def n(self) -> int:
        return self.spec.n

    @property
    def n_occupied(self) -> int:
        return self.spec.n_occupied


def _min_image(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    return d - box * np.round(d / box)


def make_system(spec: SystemSpec) -> System:
    return _build(spec, None)


def make_bloch_system(spec: SystemSpec, kfrac: Sequence[float]) -> System:
    """The system at the k-point k = 2 pi kfrac / box (kfrac in units of the
    reciprocal lattice of the periodic box, components in [0, 1); kfrac = 0 is
    the Gamma point): every periodic image n of a pair block gets its Bloch phase,
    H(k)_IJ = sum_n exp(i k . R_n) H_IJ^(n), S(k) likewise, with R_n the lattice
    translation of the image and H(k)_JI = H(k)_IJ^dagger, so H(k) and S(k) are
    complex Hermitian (values complex128).  The random numbers are those of
    `make_system` (kfrac = 0 gives the same real matrices); C0 is complex: real
    part `make_system`'s C0 / sqrt 2, imaginary part N(0, sigma^2 / 2) drawn
    after it (the same mean square |C0_ij|^2 as the real guess)."""
    return _build(spec, np.asarray(kfrac, dtype=np.float64))


def _build(spec: SystemSpec, kfrac) -> System:
    rng = np.random.default_rng(spec.seed)
    dim = len(spec.dims)
    N, norb, nwf = spec.natoms, spec.norb, spec.wf_per_atom
    box = np.asarray(spec.dims, dtype=np.float64) * spec.spacing
    pts = _lattice_points(spec.dims).astype(np.float64) * spec.spacing
    pos = pts + rng.uniform(-spec.jitter, spec.jitter, size=pts.shape)
    ntri = norb * (norb + 1) // 2
    onsite_noise = rng.normal(0.0, spec.onsite_noise, size=(N, ntri))

    # pair-image list (I < J), sorted by (I, J, image)
    cut = spec.cutoff
    if np.any(box <= cut + 2 * spec.jitter + 1e-12):
        # self images would fall inside the cutoff
        raise ValueError("lattice too small for the cutoff")
    need_images = bool(np.any(box < 2 * (cut + 2 * spec.jitter)))
    shifts = np.array(np.meshgrid(*([[-1, 0, 1]] * dim), indexing="ij")).reshape(dim, -1).T \
        if need_images else np.zeros((1, dim))
    shifts = shifts[np.lexsort(shifts.T[::-1])]
    I_list, J_list, S_list, R_list = [], [], [], []
    for I in range(N - 1):
        d = _min_image(pos[I + 1:] - pos[I], box)           # (N-I-1, dim)
        dd = d[:, None, :] + shifts[None, :, :] * box        # (.., nshift, dim)
        r = np.sqrt((dd ** 2).sum(-1))
        jj, ss = np.nonzero(r <= cut)
        if jj.size:
            I_list.append(np.full(jj.size, I))
            J_list.append(jj + I + 1)
            S_list.append(ss)
            R_list.append(r[jj, ss])
    if I_list:
        PI = np.concatenate(I_list); PJ = np.concatenate(J_list)
        PS = np.concatenate(S_list); PR = np.concatenate(R_list)
    else:
        PI = PJ = PS = np.zeros(0, dtype=np.int64); PR = np.zeros(0)
    order = np.lexsort((PS, PJ, PI))
    PI, PJ, PS, PR = PI[order], PJ[order], PS[order], PR[order]
    npi = PI.shape[0]
    G = rng.standard_normal((npi, norb, norb))
    Q = rng.standard_normal((npi, norb, norb))
    wH = (spec.hop * np.exp(-PR / spec.decay))[:, None, None]
    wS = (spec.ovl * np.exp(-PR / spec.decay))[:, None, None]
    if kfrac is not None and npi:   # Bloch phase of each image: exp(i k . R), R the lattice translation
        kvec = 2.0 * np.pi * kfrac / box
        d_img = _min_image(pos[PJ] - pos[PI], box) + shifts[PS] * box
        R = d_img - (pos[PJ] - pos[PI])
        ph = np.exp(1j * (R @ kvec))[:, None, None]
        wH = wH * ph
        wS = wS * ph
    # sum images of the same pair
    pair_key = PI * N + PJ
    upair, first = np.unique(pair_key, return_index=True)
    HB = np.add.reduceat(wH * G, first, axis=0) if npi else np.zeros((0, norb, norb))
    SB = np.add.reduceat(wS * Q, first, axis=0) if npi else np.zeros((0, norb, norb))
    UI, UJ = upair // N, upair % N

    # on-site blocks
    iu = np.triu_indices(norb)
    Hd = np.zeros((N, norb, norb))
    Hd[:, iu[0], iu[1]] = onsite_noise
    Hd = Hd + np.transpose(np.triu(Hd, 1), (0, 2, 1))
    Hd[:, np.arange(norb), np.arange(norb)] += np.asarray(spec.onsite)[None, :]
    Sd = np.broadcast_to(np.eye(norb), (N, norb, norb))

    # assemble full (both triangles) block lists sorted by (row, col)
    rows = np.concatenate([np.arange(N), UI, UJ])
    cols = np.concatenate([np.arange(N), UJ, UI])
    Hblk = np.concatenate([Hd, HB, np.conj(np.transpose(HB, (0, 2, 1)))])
    Sblk = np.concatenate([Sd, SB, np.conj(np.transpose(SB, (0, 2, 1)))])
    o = np.lexsort((cols, rows))
    T = None
    if spec.kinetic > 0.0:
        Tblk = _kinetic_blocks(spec, PI, PJ, PR, first, N)
        T = _uniform_bcsr(N, N, norb, norb, rows[o], cols[o], Tblk[o])
        Hblk = Hblk + Tblk
    H = _uniform_bcsr(N, N, norb, norb, rows[o], cols[o], Hblk[o])
    S = _uniform_bcsr(N, N, norb, norb, rows[o], cols[o], Sblk[o])

    # C pattern: rows = basis atoms b, cols = WF atoms a, |R_b - R_a| <= rc
    if spec.rc is None:
        crow = np.repeat(np.arange(N), N)
        ccol = np.tile(np.arange(N), N)
    else:
        cr, cc = [], []
        for b in range(N):
            d = _min_image(pos - pos[b], box)
            a = np.nonzero(np.sqrt((d ** 2).sum(-1)) <= spec.rc)[0]
            cr.append(np.full(a.size, b)); cc.append(a)
        crow = np.concatenate(cr); ccol = np.concatenate(cc)
    nnz_col = crow.shape[0] * norb / N          # mean stored entries per WF column
    sigma = spec.c0_scale * np.sqrt(spec.c0_ref_nnz / nnz_col)
    rng2 = np.random.default_rng(spec.seed + 10**6)
    cblk = rng2.normal(0.0, sigma, size=(crow.shape[0], norb, nwf))
    if kfrac is not None:   # complex entries of the same mean square as the real ones
        cblk = (cblk + 1j * rng2.normal(0.0, sigma, size=cblk.shape)) / np.sqrt(2.0)
    C0 = _uniform_bcsr(N, N, norb, nwf, crow, ccol, cblk)
    return System(spec=spec, pos=pos, box=box, H=H, S=S, C0=C0, pair_images=npi, T=T,
                  extra={"c0_sigma": sigma})


def _kinetic_blocks(spec: SystemSpec, PI, PJ, PR, first, N) -> np.ndarray:
    """Blocks of a synthetic kinetic matrix T on H's pattern, in the block order
    [on-site (N), pairs I<J, their transposes], like H's before sorting.

    The high orbitals carry large kinetic energies (the broad upper spectrum
    behind the ill-conditioning that kinetic preconditioning targets, Sec. II):
    level t_k = kinetic * (0.002 + (k / (norb - 1))^2) for orbital k; pair-image
    blocks (T_IJ)_kl = -0.001 exp(-r / decay) sqrt(t_k t_l) K_kl^(n), K ~ N(0, 1)
    drawn from PCG64 seeded with seed + 2 * 10**6 in pair-image order, summed
    over images; on-site blocks diagonal, t_k plus the absolute sum of the
    row's off-diagonal entries, so T is strictly diagonally dominant and
    therefore positive definite.
    """
    norb = spec.norb
    rng = np.random.default_rng(spec.seed + 2 * 10**6)
    npi = PI.shape[0]
    K = rng.standard_normal((npi, norb, norb))
    t = spec.kinetic * (0.002 + (np.arange(norb) / max(1, norb - 1)) ** 2)
    st = np.sqrt(t)
    wT = (-0.001 * np.exp(-PR / spec.decay))[:, None, None] * (st[:, None] * st[None, :])[None]
    TB = np.add.reduceat(wT * K, first, axis=0) if npi else np.zeros((0, norb, norb))
    upair = (PI * N + PJ)[first] if npi else np.zeros(0, dtype=np.int64)
    UI, UJ = upair // N, upair % N
    rowsum = np.zeros((N, norb))
    np.add.at(rowsum, UI, np.abs(TB).sum(axis=2))
    np.add.at(rowsum, UJ, np.abs(TB).sum(axis=1))
    Td = np.zeros((N, norb, norb))
    Td[:, np.arange(norb), np.arange(norb)] = t[None, :] + rowsum
    return np.concatenate([Td, TB, np.transpose(TB, (0, 2, 1))])
