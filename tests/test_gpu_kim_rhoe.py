"""GPU parity of the energy density (Eq. 6 with the Kim correction of Sec. II) and
of the Kim functional with more wavefunctions than occupied states (Sec. II).

Tolerances as in the other FP64 parity tests: energies within 1e-10 Ha/atom,
per-iteration energies within 1e-11 relative, matrices within 1e-9 absolute.
"""

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from _helpers import oracle_run, system
from ommgen.systems import KIM_ETA13
from paper_2209_05934_amd import omm as L
from paper_2209_05934_amd.solver import Context, Problem
from test_gpu_parity import MODES, check_trajectory

pytestmark = pytest.mark.gpu


def run_both(s, mode, nocc=None, ne_tol=0.0, **kw):
    """The same solve on the GPU (options kw, plus the electron-count check ne_tol) and in the oracle."""
    ctx = Context([Problem(s.H, s.S, s.C0, s.n, MODES[mode], eta=s.spec.eta, n_occupied=nocc)],
                  ne_tol=ne_tol, **kw)
    rc, reps = ctx.minimize()
    ref = oracle_run(s, mode, n_occupied=nocc, **kw)
    return ctx, reps[0], ref


def rho_e_values(s, ref):
    return s.S.gather_from_dense(O.energy_density_matrix(ref.C, ref.HW, ref.SW, s.spec.eta))


@pytest.mark.parametrize("name,mode,eta", [("chain8", "dense", 0.1), ("chain8", "cholesky", 0.1),
                                           ("cubic4_dense", "dense", 0.0), ("cubic3_dense", "cholesky", -0.25)])
def test_energy_density_dense(name, mode, eta):
    s = system(name, eta=eta)
    ctx, r, ref = run_both(s, mode, tol_grad=1e-9)
    assert r.status == L.OMM_OK and ref.converged
    rho_e = ctx.energy_density(0)
    assert np.max(np.abs(rho_e - rho_e_values(s, ref))) <= 1e-9
    # the eigen form at the minimum: 2 sum_i eps_i x_i x_i^T (unshifted eps)
    w, X = scipy.linalg.eigh(s.H.to_dense(), s.S.to_dense())
    Xn = X[:, :s.n]
    assert np.max(np.abs(rho_e - s.S.gather_from_dense(2.0 * Xn @ np.diag(w[:s.n]) @ Xn.T))) <= 1e-8
    # the density matrix is still rho (the shared kernels take other coefficients)
    assert np.max(np.abs(ctx.density_matrix(0) - s.S.gather_from_dense(O.density_matrix(ref.C, ref.SW)))) <= 1e-9
    ctx.close()


def test_energy_density_sparse_and_device_output():
    import torch
    s = system("cubic5_sparse")               # eta 1.5, localized
    ctx, r, ref = run_both(s, "sparse", max_iter=60, tol_grad=1e-9)
    assert r.iters_total == 60 == ref.iterations
    want = rho_e_values(s, ref)
    assert np.max(np.abs(ctx.energy_density(0) - want)) <= 1e-9
    out = torch.zeros(s.S.val.size, dtype=torch.float64, device="cuda:0")
    L.omm_energy_density(ctx.ctx, 0, out)
    assert np.array_equal(out.cpu().numpy(), ctx.energy_density(0))
    ctx.close()


def test_energy_density_call_order():
    s = system("chain8")
    H, S = L.BlockArgs.from_block_matrix(s.H), L.BlockArgs.from_block_matrix(s.S)
    ctx = L.omm_init(H, S, s.n, L.OMM_DENSE)
    out = np.zeros(s.S.val.size)
    assert L.load().omm_energy_density(ctx, 0, out.ctypes.data, L.OMM_HOST) == L.OMM_ERR_STATE
    assert L.load().omm_energy_density(ctx, 1, out.ctypes.data, L.OMM_HOST) == L.OMM_ERR_ARG
    assert L.load().omm_set_occupied(ctx, 0, s.n + 1) == L.OMM_ERR_ARG
    assert L.load().omm_set_occupied(ctx, 0, 0) == L.OMM_ERR_ARG
    L.omm_destroy(ctx)


@pytest.mark.parametrize("name,mode,eta", [("chain8", "dense", 0.1), ("chain8", "cholesky", -0.3),
                                           ("cubic3_dense", "dense", KIM_ETA13)])
def test_kim_more_wavefunctions_dense(name, mode, eta):
    s = system(name, wf_per_atom=3, eta=eta)
    nocc = s.n_occupied
    assert s.n == 3 * s.natoms and nocc == 2 * s.natoms
    ctx, r, ref = run_both(s, mode, nocc=nocc, tol_grad=1e-9, max_iter=5000, ne_tol=1e-7)
    assert r.status == L.OMM_OK and ref.converged             # electron count 2n within 1e-7
    assert abs(r.iters_total - ref.iterations) <= 1
    w, X = scipy.linalg.eigh(s.H.to_dense(), s.S.to_dense())
    assert w[nocc - 1] < eta < w[nocc]
    assert abs(r.energy - ref.energy) / s.natoms <= 1e-10
    assert abs(r.energy - 2.0 * (w[:nocc] - eta).sum()) / s.natoms <= 1e-10
    assert abs(r.energy_band - 2.0 * w[:nocc].sum()) / s.natoms <= 1e-10
    assert abs(r.electron_count - 2 * nocc) <= 1e-7
    check_trajectory(ctx.history(0), ref, k=min(10, ref.iterations))
    Xn = X[:, :nocc]
    assert np.max(np.abs(ctx.density_matrix(0) - s.S.gather_from_dense(2.0 * Xn @ Xn.T))) <= 1e-8
    assert np.max(np.abs(ctx.energy_density(0)
                         - s.S.gather_from_dense(2.0 * Xn @ np.diag(w[:nocc]) @ Xn.T))) <= 1e-8
    HW, SW = ctx.projected(0)
    ev = np.linalg.eigvalsh(SW)
    assert np.max(np.abs(ev[:s.n - nocc])) <= 1e-6 and np.max(np.abs(ev[s.n - nocc:] - 1.0)) <= 1e-8
    ctx.close()


def test_kim_more_wavefunctions_sparse_trajectory():
    s = system("cubic5_sparse", wf_per_atom=3, eta=KIM_ETA13)
    ctx, r, ref = run_both(s, "sparse", nocc=s.n_occupied, max_iter=60, tol_grad=1e-9)
    assert r.iters_total == 60 == ref.iterations
    check_trajectory(ctx.history(0), ref)
    assert abs(r.energy_band - ref.energy_band) / s.natoms <= 1e-10
    assert abs(r.energy_band - r.energy - 2.0 * KIM_ETA13 * s.n_occupied) <= 1e-9 * abs(r.energy)
    assert np.max(np.abs(ctx.density_matrix(0) - s.S.gather_from_dense(O.density_matrix(ref.C, ref.SW)))) <= 1e-9
    assert np.max(np.abs(ctx.energy_density(0) - rho_e_values(s, ref))) <= 1e-9
    ctx.close()
