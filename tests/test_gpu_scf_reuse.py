"""GPU checks of context reuse across SCF/MD steps (Sec. III A: the solver is called
again at every step): new H and S values on the same structure (omm_update_hs), a
warm start from the previous C, and the reuse functions on device results.

A context updated in place must give what a fresh context gives (same kernels and
plans, so equal to 1e-12 relative); warm starts are checked against the oracle's own
warm start and the generalized eigenvalue result."""

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from _helpers import oracle_run, system
from paper_2209_05934_amd import omm as L
from paper_2209_05934_amd.solver import Context, Problem
from test_gpu_parity import MODES

pytestmark = pytest.mark.gpu


def perturbed(s, seed, amp=0.01):
    """H and S of the next step: symmetric perturbations on their block pattern."""
    rng = np.random.default_rng(seed)
    m = s.m
    mask = s.H.pattern_mask()
    dH = rng.standard_normal((m, m)) * amp
    dS = rng.standard_normal((m, m)) * amp * 0.5
    H = s.H.to_dense() + np.where(mask, dH + dH.T, 0.0)
    S = s.S.to_dense() + np.where(mask, dS + dS.T, 0.0)
    return s.H.with_values(s.H.gather_from_dense(H)), s.S.with_values(s.S.gather_from_dense(S))


@pytest.mark.parametrize("name,mode,prec", [("cubic4_dense", "dense", L.OMM_FP64),
                                            ("cubic3_dense", "cholesky", L.OMM_FP64),
                                            ("cubic5_sparse", "sparse", L.OMM_FP64),
                                            ("cubic3_dense", "dense", L.OMM_FP32)])
def test_update_hs_equals_fresh_context(name, mode, prec):
    s = system(name)
    H2, S2 = perturbed(s, 7)
    kw = dict(max_iter=300, precision=prec)
    ctx = Context([Problem(s.H, s.S, s.C0, s.n, MODES[mode], eta=s.spec.eta)], **kw)
    ctx.minimize()
    L.omm_update_hs(ctx.ctx, 0, L.BlockArgs.from_block_matrix(H2), L.BlockArgs.from_block_matrix(S2))
    rc, reps = ctx.minimize()
    fresh = Context([Problem(H2, S2, s.C0, s.n, MODES[mode], eta=s.spec.eta)], **kw)
    rc2, reps2 = fresh.minimize()
    assert reps[0].iters_total == reps2[0].iters_total
    assert abs(reps[0].energy - reps2[0].energy) <= 1e-12 * abs(reps2[0].energy)
    assert np.max(np.abs(ctx.density_matrix(0) - fresh.density_matrix(0))) <= 1e-12
    ctx.close()
    fresh.close()


def test_warm_start_after_update():
    s = system("cubic4_dense")
    H2, S2 = perturbed(s, 11)
    ctx = Context([Problem(s.H, s.S, s.C0, s.n, L.OMM_DENSE)])
    rc, r1 = ctx.minimize()
    C1 = ctx.coeffs(0)
    L.omm_update_hs(ctx.ctx, 0, L.BlockArgs.from_block_matrix(H2), L.BlockArgs.from_block_matrix(S2))
    with pytest.raises(L.OmmError) as e:          # outputs wait for the next minimize
        ctx.density_matrix(0)
    assert e.value.status == L.OMM_ERR_STATE
    ctx.set_coeffs(0, s.C0.with_values(C1))
    rc, r2 = ctx.minimize()
    # the oracle's own warm start: its converged C of the first step, then the new H, S
    ref1 = oracle_run(s, "dense", tol_grad=1e-9)
    ref2 = O.cg_minimize(H2.to_dense(), S2.to_dense(), ref1.C, tol_grad=1e-9)
    cold = O.cg_minimize(H2.to_dense(), S2.to_dense(), s.C0.to_dense(), tol_grad=1e-9)
    assert r2[0].status == L.OMM_OK and ref2.converged
    assert abs(r2[0].iters_total - ref2.iterations) <= 2 and ref2.iterations < cold.iterations
    w = scipy.linalg.eigh(H2.to_dense(), S2.to_dense(), eigvals_only=True)
    assert abs(r2[0].energy - 2.0 * w[:s.n].sum()) / s.natoms <= 1e-10
    assert abs(r2[0].energy - ref2.energy) / s.natoms <= 1e-10
    ctx.close()


def test_update_hs_in_a_batch_and_errors():
    a, b = system("chain8"), system("cubic5_sparse")
    probs = [Problem(a.H, a.S, a.C0, a.n, L.OMM_DENSE), Problem(b.H, b.S, b.C0, b.n, L.OMM_BLOCK_SPARSE,
                                                                 eta=b.spec.eta)]
    ctx = Context(probs, max_iter=200)
    rc, r1 = ctx.minimize()
    rho_b = ctx.density_matrix(1)
    H2, S2 = perturbed(a, 3)
    L.omm_update_hs(ctx.ctx, 0, L.BlockArgs.from_block_matrix(H2), L.BlockArgs.from_block_matrix(S2))
    rc, r2 = ctx.minimize()
    assert r2[1].iters_total == r1[1].iters_total and r2[1].energy == r1[1].energy
    assert np.array_equal(ctx.density_matrix(1), rho_b)
    w = scipy.linalg.eigh(H2.to_dense(), S2.to_dense(), eigvals_only=True)
    assert abs(r2[0].energy - 2.0 * w[:a.n].sum()) / a.natoms <= 1e-10
    lib = L.load()
    import ctypes
    Hb = L.BlockArgs.from_block_matrix(b.H)
    Ha = L.BlockArgs.from_block_matrix(a.H)
    assert lib.omm_update_hs(ctx.ctx, 0, ctypes.byref(Hb.struct), ctypes.byref(Hb.struct)) == L.OMM_ERR_ARG
    assert lib.omm_update_hs(ctx.ctx, 2, ctypes.byref(Ha.struct), ctypes.byref(Ha.struct)) == L.OMM_ERR_ARG
    ctx.close()
