"""C ABI checks that need no GPU: exported symbols, struct layouts, host-side validation."""

import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from ommgen import config_spec, make_system
from paper_2209_05934_amd import omm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "omm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(omm_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_struct_layouts_match_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "omm.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(omm_matrix), sizeof(omm_options), sizeof(omm_report), sizeof(omm_sizes));
  printf("%zu %zu %zu %zu %zu\n", offsetof(omm_options, hip_stream), offsetof(omm_report, seconds),
         offsetof(omm_sizes, bytes_alg_step), offsetof(omm_sizes, tile_split),
         offsetof(omm_options, log_jsonl_path));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(v) for v in out]
    assert sizes[:4] == [ctypes.sizeof(L.omm_matrix), ctypes.sizeof(L.omm_options),
                         ctypes.sizeof(L.omm_report), ctypes.sizeof(L.omm_sizes)]
    assert sizes[4] == L.omm_options.hip_stream.offset
    assert sizes[5] == L.omm_report.seconds.offset
    assert sizes[6] == L.omm_sizes.bytes_alg_step.offset
    assert sizes[7] == L.omm_sizes.tile_split.offset
    assert sizes[8] == L.omm_options.log_jsonl_path.offset


def test_status_strings_and_defaults():
    assert L.omm_status_str(L.OMM_OK) == "OMM_OK"
    assert L.omm_status_str(L.OMM_ERR_NOT_SPD) == "OMM_ERR_NOT_SPD"
    assert L.omm_status_str(99) == "OMM_UNKNOWN_STATUS"
    o = L.omm_default_options()
    assert o.tol_grad == 1e-9 and o.max_iter == 10000 and o.fp64_refine_iters == 5
    assert o.precision == L.OMM_FP64 and o.graph_iters == 16 and o.hip_stream is None


@pytest.fixture(scope="module")
def chain():
    return make_system(config_spec("chain8"))


def _args(bm, **over):
    d = dict(row_bsz=bm.row_bsz, col_bsz=bm.col_bsz, row_ptr=bm.row_ptr, col_idx=bm.col_idx,
             val_off=bm.val_off, val=bm.val)
    d.update(over)
    return L.BlockArgs(**d)


def _init_rc(H, S, n, mode=L.OMM_DENSE, opt=None):
    ctx = ctypes.c_void_p()
    rc = L.load().omm_init(ctypes.byref(ctx), ctypes.byref(H.struct), ctypes.byref(S.struct), n, mode,
                           ctypes.byref(opt) if opt is not None else None)
    assert not ctx.value
    return rc, L.omm_last_error(None)


def test_unwritable_log_path_rejected_before_the_device(chain):
    # the JSONL iteration log is opened for appending at omm_init, before any HIP call
    opt = L.omm_default_options()
    opt.log_jsonl_path = b"/nonexistent-directory/omm-log.jsonl"
    rc, msg = _init_rc(_args(chain.H), _args(chain.S), chain.n, opt=opt)
    assert rc == L.OMM_ERR_ARG and "log_jsonl_path" in msg


# every rejected call below fails in host-side validation, before any HIP call
def test_rejects_bad_n_occ(chain):
    rc, msg = _init_rc(_args(chain.H), _args(chain.S), 0)
    assert rc == L.OMM_ERR_ARG and "n_occ" in msg
    rc, _ = _init_rc(_args(chain.H), _args(chain.S), chain.m + 1)
    assert rc == L.OMM_ERR_ARG


def test_rejects_pattern_mismatch(chain):
    S = chain.S
    rp = S.row_ptr.copy()
    ci = S.col_idx.copy()
    ci[[1, 2]] = ci[[2, 1]]                    # unsorted columns
    rc, msg = _init_rc(_args(chain.H), _args(S, col_idx=ci), chain.n)
    assert rc == L.OMM_ERR_ARG and "increasing" in msg
    rc, msg = _init_rc(_args(chain.H), _args(S, row_ptr=rp, col_idx=S.col_idx[::-1].copy()), chain.n)
    assert rc == L.OMM_ERR_ARG


def test_rejects_bad_mode_and_offsets(chain):
    rc, msg = _init_rc(_args(chain.H), _args(chain.S), chain.n, mode=7)
    assert rc == L.OMM_ERR_ARG and "mode" in msg
    bad = chain.S.val_off.copy()
    bad[-1] = chain.S.val.size                  # block runs past the value array
    rc, msg = _init_rc(_args(chain.H), _args(chain.S, val_off=bad), chain.n)
    assert rc == L.OMM_ERR_ARG and "val_off" in msg


def test_rejects_unsymmetric_pattern():
    from dataclasses import replace
    s = make_system(replace(config_spec("cubic4_dense"), rc=1.2, dense=False))
    H = s.H
    rows = H.block_rows()
    # drop one off-diagonal block (i, j) but keep (j, i)
    k = next(k for k in range(H.nnzb) if rows[k] != H.col_idx[k])
    keep = np.ones(H.nnzb, dtype=bool)
    keep[k] = False
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=H.nbrow))]).astype(np.int64)
    Hb = _args(H, row_ptr=rp, col_idx=H.col_idx[keep].copy(), val_off=H.val_off[keep].copy())
    Sb = _args(s.S, row_ptr=rp, col_idx=H.col_idx[keep].copy(), val_off=s.S.val_off[keep].copy())
    rc, msg = _init_rc(Hb, Sb, s.n, mode=L.OMM_BLOCK_SPARSE)
    assert rc == L.OMM_ERR_ARG and "symmetric" in msg


def test_rejects_non_square_blocks(chain):
    H = chain.H
    cb = H.col_bsz.copy()
    cb[0] = 3
    rc, _ = _init_rc(_args(H, col_bsz=cb), _args(chain.S, col_bsz=cb), chain.n)
    assert rc == L.OMM_ERR_ARG


def test_null_pointers_rejected():
    lib = L.load()
    assert lib.omm_init(None, None, None, 1, 0, None) == L.OMM_ERR_ARG
    assert lib.omm_minimize(None, None) == L.OMM_ERR_ARG
    lib.omm_destroy(None)


def test_complex_init_rejects_bad_input_before_the_device():
    # k-point contexts: the complex matrices are embedded on the host and checked
    # there; a malformed one (or one in device memory) never reaches HIP
    from ommgen.systems import cubic_spec, make_bloch_system
    z = make_bloch_system(cubic_spec(3, 31, dense=True), (0.25, 0.0, 0.0))
    H, S = _args(z.H), _args(z.S)
    assert H.struct.nval == z.H.val.size and z.H.val.dtype == np.complex128

    def init(Hb, Sb, n):
        ctx = ctypes.c_void_p()
        n_arr = (ctypes.c_int64 * 1)(n)
        m_arr = (ctypes.c_int32 * 1)(L.OMM_DENSE)
        rc = L.load().omm_init_complex(ctypes.byref(ctx), 1, ctypes.byref(Hb.struct), ctypes.byref(Sb.struct),
                                       n_arr, m_arr, None, None)
        assert not ctx.value
        return rc, L.omm_last_error(None)

    bad = z.H.val_off.copy()
    bad[-1] = z.H.val.size
    rc, msg = init(_args(z.H, val_off=bad), S, z.n)
    assert rc == L.OMM_ERR_ARG and "val_off" in msg
    rc, msg = init(H, S, 0)
    assert rc == L.OMM_ERR_ARG and "n_occ" in msg
    Hd = _args(z.H)
    Hd.struct.memspace = L.OMM_DEVICE
    rc, msg = init(Hd, S, z.n)
    assert rc == L.OMM_ERR_ARG and "host" in msg
