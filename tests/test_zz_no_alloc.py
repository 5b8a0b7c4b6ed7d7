"""The allocation-free density-matrix entry point through the C ABI: the same
result as omm_density_matrix, bit for bit, on two calls in a row (the second on
a smaller system, so stale scratch contents would show), in the plain and the
Cholesky-reduced dense forms and for a system of a batch context; a context too
large for the fixed scratch is refused."""

import numpy as np
import pytest
import torch

from _helpers import system
from paper_2209_05934_amd import omm as L
from paper_2209_05934_amd.solver import Context, Problem

pytestmark = pytest.mark.gpu


def _solved(name, mode, **o):
    s = system(name)
    ctx = Context([Problem(s.H, s.S, s.C0, s.n, mode, eta=s.spec.eta)], **o)
    ctx.minimize()
    return s, ctx


def _both(ctx, sys, nval):
    dev = torch.device("cuda:0")
    ref = torch.full((nval,), -1.0, dtype=torch.float64, device=dev)
    got = torch.full((nval,), -2.0, dtype=torch.float64, device=dev)
    L.omm_density_matrix(ctx.ctx, sys, ref)
    L.omm_density_matrix_noalloc(ctx.ctx, sys, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_density_matrix_equals_the_allocating_call():
    # first the larger system, then a smaller one reusing the same scratch
    for name, mode in [("cubic4_dense", L.OMM_DENSE), ("chain8", L.OMM_DENSE), ("cubic3_dense", L.OMM_DENSE_CHOLESKY)]:
        s, ctx = _solved(name, mode)
        ref, got = _both(ctx, 0, s.S.val.size)
        assert np.array_equal(ref, got), name
        assert np.all(np.isfinite(got)) and np.any(got != 0.0)
        ctx.close()
    # a system of a batch context (not the first one)
    a, b = system("chain8"), system("cubic3_sparse")
    ctx = Context([Problem(a.H, a.S, a.C0, a.n, L.OMM_DENSE),
                   Problem(b.H, b.S, b.C0, b.n, L.OMM_BLOCK_SPARSE, eta=b.spec.eta)], max_iter=50)
    ctx.minimize()
    ref, got = _both(ctx, 1, b.S.val.size)
    assert np.array_equal(ref, got)
    ctx.close()


def test_noalloc_density_matrix_refuses_a_context_beyond_the_scratch():
    s, ctx = _solved("cubic8_sparse", L.OMM_BLOCK_SPARSE, max_iter=1, filter_eps=0.0)
    out = torch.zeros(s.S.val.size, dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.OmmError) as e:
        L.omm_density_matrix_noalloc(ctx.ctx, 0, out)
    assert e.value.status == L.OMM_ERR_ARG
    assert "scratch" in L.omm_last_error(ctx.ctx)
    ctx.close()
