"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test pins a part of the oracle to something other than itself:
finite differences (gradient), an exact polynomial identity evaluated from
scratch (quartic), a brute-force grid (line search), the generalized
eigendecomposition (converged dense energy and density matrix, Sec. II: the
minimum of Eq. 4 equals the solution of Eq. 2), the identities of Eqs. 1, 2,
5 and Listing 1, the Cholesky reduction (Sec. II) and an independent
quasi-Newton optimizer on tiny localized problems.
"""

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import oracle as O
from ommgen import config_spec, make_system


def _rand_problem(m=10, n=4, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, m))
    H = 0.5 * (A + A.T)
    B = rng.standard_normal((m, m)) * 0.1
    S = np.eye(m) + 0.5 * (B + B.T)
    C = rng.standard_normal((m, n)) * 0.3
    D = rng.standard_normal((m, n)) * 0.3
    return H, S, C, D


def _eigen(H, S, n, eta=0.0):
    w, X = scipy.linalg.eigh(H - eta * S, S)
    return 2.0 * w[:n].sum(), 2.0 * X[:, :n] @ X[:, :n].T, w


@pytest.fixture(scope="module")
def chain():
    s = make_system(config_spec("chain8"))
    return s, s.H.to_dense(), s.S.to_dense(), s.C0.to_dense()


@pytest.fixture(scope="module")
def cube4():
    s = make_system(config_spec("cubic4_dense"))
    return s, s.H.to_dense(), s.S.to_dense(), s.C0.to_dense()


# ------------------------------------------------------------ functional, gradient
def test_gradient_finite_differences():
    H, S, C, _ = _rand_problem()
    G = O.om_gradient(H, S, C)
    h = 1e-5
    num = np.zeros_like(C)
    for idx in np.ndindex(C.shape):
        Cp, Cm = C.copy(), C.copy()
        Cp[idx] += h
        Cm[idx] -= h
        num[idx] = (O.om_energy(H, S, Cp) - O.om_energy(H, S, Cm)) / (2 * h)
    assert np.max(np.abs(num - G)) <= 1e-7 * np.max(np.abs(G))


def test_gradient_chain_fd(chain):
    s, H, S, C0 = chain
    G = O.om_gradient(H, S, C0)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(20):
        i, j = rng.integers(s.m), rng.integers(s.n)
        Cp, Cm = C0.copy(), C0.copy()
        Cp[i, j] += h
        Cm[i, j] -= h
        fd = (O.om_energy(H, S, Cp) - O.om_energy(H, S, Cm)) / (2 * h)
        assert abs(fd - G[i, j]) <= 1e-7 * max(1.0, abs(G[i, j]))


def test_energy_matches_trace_form():
    # Eq. 4 in its expanded form 4 Tr H_W - 2 Tr(S_W H_W); Tr(rho H) equals E~ for any C
    H, S, C, _ = _rand_problem(seed=1)
    HW, SW = C.T @ H @ C, C.T @ S @ C
    E = O.om_energy(H, S, C)
    assert abs(E - (4 * np.trace(HW) - 2 * np.trace(SW @ HW))) < 1e-12 * abs(E)
    rho = O.density_matrix(C, SW)
    assert abs(np.trace(rho @ H) - E) < 1e-11 * max(1, abs(E))
    # Listing 1: n_e = 2 Tr[(2I - S_W) S_W] equals Tr(rho S) for any C
    assert abs(O.electron_count(SW) - np.trace(rho @ S)) < 1e-11 * max(1, abs(np.trace(rho @ S)))


# ------------------------------------------------------------ quartic
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quartic_exact(seed):
    H, S, C, D = _rand_problem(seed=seed)
    c = O.quartic_coefficients(H, S, C, D)
    for x in (-1.0, -0.5, 0.3, 1.0, 2.0):
        ref = O.om_energy(H, S, C + x * D)
        assert abs(O.quartic_value(c, x) - ref) <= 1e-12 * max(1.0, abs(ref)) * 10
    # c1 is the directional derivative <dE/dC, D>
    assert abs(c[1] - np.sum(O.om_gradient(H, S, C) * D)) <= 1e-11 * max(1.0, abs(c[1]))
    # c0 is the functional itself
    assert abs(c[0] - O.om_energy(H, S, C)) <= 1e-12 * max(1.0, abs(c[0]))


def _grid_first_min(c, xmax=50.0, n=2_000_001):
    x = np.linspace(0.0, xmax, n)
    p = c[0] + x * (c[1] + x * (c[2] + x * (c[3] + x * c[4])))
    up = np.nonzero(np.diff(p) > 0)[0]
    if up.size == 0:
        return None, x[1] - x[0]
    return x[up[0]], x[1] - x[0]


def test_line_minimum_vs_grid():
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(400):
        c = rng.standard_normal(5) * np.array([1, 1, 3, 3, 1])
        c[1] = -abs(c[1]) - 0.05
        xg, dx = _grid_first_min(c)
        x, ok = O.line_minimum(c)
        if xg is None or xg >= 49.0:
            assert not ok or x > 49.0
            continue
        assert ok
        assert abs(x - xg) <= 2 * dx
        checked += 1
    assert checked > 200


def test_line_minimum_failures():
    assert not O.line_minimum([0.0, 1.0, 1.0, 0.0, 0.0])[1]           # ascent direction
    assert not O.line_minimum([0.0, -1.0, -1.0, -1.0, -1.0])[1]       # unbounded, no minimum
    x, ok = O.line_minimum([0.0, -2.0, 1.0, 0.0, 0.0])                # pure quadratic
    assert ok and abs(x - 1.0) < 1e-14


# ------------------------------------------------------------ converged dense results
@pytest.mark.parametrize("which", ["chain", "cube4"])
def test_dense_converges_to_eigen_solution(which, request):
    s, H, S, C0 = request.getfixturevalue(which)
    res = O.cg_minimize(H, S, C0, tol_grad=1e-9, max_iter=5000)
    assert res.status == "ok" and res.converged
    Estar, rho_star, _ = _eigen(H, S, s.n)
    assert abs(res.energy - Estar) / s.natoms <= 1e-10
    rho = O.density_matrix(res.C, res.SW)
    assert np.max(np.abs(rho - rho_star)) <= 1e-8
    assert np.max(np.abs(res.SW - np.eye(s.n))) <= 1e-8              # S_W -> I (Sec. II)
    assert abs(np.trace(rho @ S) - 2 * s.n) <= 1e-8                   # 2n electrons
    assert np.max(np.abs(rho @ S @ rho - 2 * rho)) <= 1e-8            # idempotency with spin 2
    assert abs(O.exact_band_energy(H, S, res.C) - res.energy) / s.natoms <= 1e-10   # Eq. 2
    E = [h["E"] for h in res.history]
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(E, E[1:]))    # monotone descent


@pytest.mark.parametrize("which", ["chain", "cube4"])
def test_cholesky_equals_plain(which, request):
    s, H, S, C0 = request.getfixturevalue(which)
    plain = O.cg_minimize(H, S, C0, tol_grad=1e-9)
    chol = O.cg_minimize_cholesky(H, S, C0, tol_grad=1e-9)
    assert chol.converged
    assert abs(chol.energy - plain.energy) / s.natoms <= 1e-10
    rp = O.density_matrix(plain.C, plain.SW)
    rc = O.density_matrix(chol.C, chol.SW)
    assert np.max(np.abs(rp - rc)) <= 1e-8
    # the reduction itself: U^T U = S and U^{-T} H U^{-1} has the generalized spectrum
    Ht, U = O.cholesky_reduce(H, S)
    assert np.max(np.abs(U.T @ U - S)) < 1e-13
    w = scipy.linalg.eigh(H, S, eigvals_only=True)
    assert np.max(np.abs(np.linalg.eigvalsh(0.5 * (Ht + Ht.T)) - w)) < 1e-12


def test_kim_shift_in_gap(chain):
    s, H, S, C0 = chain
    base = O.cg_minimize(H, S, C0, tol_grad=1e-9)
    eta = 0.1                                  # inside the gap
    shifted = O.cg_minimize(H, S, C0, eta=eta, tol_grad=1e-9)
    assert shifted.converged
    assert abs(shifted.energy_band - base.energy) / s.natoms <= 1e-10
    Estar, _, _ = _eigen(H, S, s.n, eta)
    assert abs(shifted.energy - Estar) / s.natoms <= 1e-10


def test_full_mask_equals_dense(chain):
    s, H, S, C0 = chain
    dense = O.cg_minimize(H, S, C0, tol_grad=1e-9)
    masked = O.cg_minimize(H, S, C0, mask=np.ones_like(C0, dtype=bool), tol_grad=1e-9)
    assert masked.iterations == dense.iterations
    assert abs(masked.energy - dense.energy) == 0.0


# ------------------------------------------------------------ localized results
def _tiny_localized(seed=5, natoms=4, norb=3):
    rng = np.random.default_rng(seed)
    m = natoms * norb
    A = rng.standard_normal((m, m)) * 0.1
    H = 0.5 * (A + A.T)
    for a in range(natoms):
        H[a * norb:(a + 1) * norb, a * norb:(a + 1) * norb] += np.diag([-1.0] + [1.0] * (norb - 1))
    B = rng.standard_normal((m, m)) * 0.03
    S = np.eye(m) + 0.5 * (B + B.T)
    # 1 WF per atom, localized on its own atom and the next one (periodic)
    mask = np.zeros((m, natoms), dtype=bool)
    for a in range(natoms):
        for b in (a, (a + 1) % natoms):
            mask[b * norb:(b + 1) * norb, a] = True
    C0 = np.where(mask, rng.standard_normal((m, natoms)) * 0.3, 0.0)
    return H, S, C0, mask


def test_localized_matches_bfgs():
    H, S, C0, mask = _tiny_localized()
    res = O.cg_minimize(H, S, C0, mask=mask, tol_grad=1e-10, max_iter=20000)
    assert res.converged
    free = np.nonzero(mask.ravel())[0]

    def f(v):
        C = np.zeros(mask.size)
        C[free] = v
        C = C.reshape(mask.shape)
        HW, SW = C.T @ H @ C, C.T @ S @ C
        return 2.0 * np.trace((2.0 * np.eye(C.shape[1]) - SW) @ HW)

    opt = scipy.optimize.minimize(f, C0.ravel()[free], method="BFGS",
                                  options=dict(gtol=1e-10, maxiter=20000))
    assert abs(opt.fun - res.energy) <= 1e-8 * abs(res.energy)
    assert np.all(res.C[~mask] == 0.0)
    # variational bound: the constrained minimum lies above the unconstrained one
    Estar, _, _ = _eigen(H, S, mask.shape[1])
    assert res.energy >= Estar - 1e-12


def test_localized_gradient_projection():
    H, S, C0, mask = _tiny_localized(seed=11)
    res = O.cg_minimize(H, S, C0, mask=mask, tol_grad=1e-9, max_iter=20000)
    G = O.om_gradient(H, S, res.C)
    assert np.max(np.abs(G[mask])) <= 1e-9          # stationary on the pattern
    assert np.max(np.abs(G[~mask])) > 1e-6           # but not off it


# ------------------------------------------------------------ filtering, stop rules, failures
def test_filter_blocks_strict():
    A = np.zeros((4, 4))
    A[:2, :2] = 0.5                                 # norm 1.0
    A[2:, 2:] = 0.25                                # norm 0.5
    A[:2, 2:] = [[1e-7, 0], [0, 0]]
    out = O.filter_blocks(A, [2, 2], [2, 2], 0.5)
    assert np.all(out[:2, :2] == 0.5) and np.all(out[2:, 2:] == 0.25)   # norm == eps kept
    assert np.all(out[:2, 2:] == 0)
    assert np.array_equal(O.filter_blocks(A, [2, 2], [2, 2], 0.0), A)


def test_rel_tol_and_max_iter(chain):
    s, H, S, C0 = chain
    r = O.cg_minimize(H, S, C0, tol_grad=0.0, rel_tol=1e-9)
    assert r.converged and r.iterations < 40
    Estar, _, _ = _eigen(H, S, s.n)
    assert abs(r.energy - Estar) / s.natoms < 1e-6
    r2 = O.cg_minimize(H, S, C0, max_iter=3)
    assert r2.status == "not_converged" and r2.iterations == 3 and len(r2.history) == 3


def test_no_line_minimum_failure():
    # H positive definite and an oversized guess: along -G the quartic falls without bound
    m, n = 6, 2
    H = np.eye(m)
    S = np.eye(m)
    C0 = np.zeros((m, n))
    C0[0, 0] = C0[1, 1] = 3.0
    r = O.cg_minimize(H, S, C0)
    assert r.status == "no_line_min" and not r.converged and r.iterations == 0


# ------------------------------------------------------------ rho and rho_E as derivatives
def _sym(rng, m, scale):
    A = rng.standard_normal((m, m)) * scale
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("eta", [0.0, 0.3])
def test_density_matrices_are_derivatives_of_the_functional(eta):
    # E~(C; H - eta S, S) at fixed C: dE~/dH = rho (Eq. 5) and dE~/dS = -rho_E, the
    # energy density of Eq. 6 with the Kim correction rho_E + eta rho (Sec. II); these
    # are the two traces of the force expression (Eq. 6)
    H, S, C, _ = _rand_problem(m=9, n=4, seed=3)
    rng = np.random.default_rng(7)
    dH, dS = _sym(rng, 9, 1.0), _sym(rng, 9, 1.0)
    f = lambda Hm, Sm: O.om_energy(O.kim_shift(Hm, Sm, eta), Sm, C)      # noqa: E731
    h = 1e-5
    dE_dH = (f(H + h * dH, S) - f(H - h * dH, S)) / (2 * h)
    dE_dS = (f(H, S + h * dS) - f(H, S - h * dS)) / (2 * h)
    HW, SW = O.projections(O.kim_shift(H, S, eta), S, C)
    rho = O.density_matrix(C, SW)
    rho_e = O.energy_density_matrix(C, HW, SW, eta)
    assert abs(dE_dH - np.sum(rho * dH)) <= 1e-8 * max(1.0, abs(dE_dH))
    assert abs(dE_dS + np.sum(rho_e * dS)) <= 1e-8 * max(1.0, abs(dE_dS))
    # a dropped Kim term would miss by eta <rho, dS>
    if eta:
        assert abs(eta * np.sum(rho * dS)) > 1e-3


@pytest.mark.parametrize("eta", [0.0, 0.1])
def test_energy_density_at_the_dense_minimum(chain, eta):
    # at the unconstrained minimum rho_E is the energy-weighted density matrix
    # 2 sum_i eps_i x_i x_i^T over the occupied states, eps_i unshifted
    s, H, S, C0 = chain
    res = O.cg_minimize(H, S, C0, eta=eta, tol_grad=1e-9)
    assert res.converged
    w, X = scipy.linalg.eigh(H, S)
    Xn = X[:, :s.n]
    ref = 2.0 * Xn @ np.diag(w[:s.n]) @ Xn.T
    rho_e = O.energy_density_matrix(res.C, res.HW, res.SW, eta)
    assert np.max(np.abs(rho_e - ref)) <= 1e-8
    # pattern restriction keeps exactly the pattern entries
    pat = S != 0.0
    assert np.array_equal(O.energy_density_matrix(res.C, res.HW, res.SW, eta, pat), np.where(pat, rho_e, 0.0))


# ------------------------------------------------------------ Kim functional with n' > n
@pytest.mark.parametrize("eta", [0.1, -0.3])
def test_kim_more_wavefunctions_than_occupied_states(eta):
    # Sec. II: with eta in the gap and n' > n columns, the minimum occupies the n
    # states below eta (shifted energy 2 sum_{i<=n} (eps_i - eta)); the spare columns
    # go to zero norm, so S_W has n eigenvalues 1 and n' - n eigenvalues 0 and the
    # electron count is 2n
    from dataclasses import replace
    s = make_system(replace(config_spec("chain8"), wf_per_atom=3))
    n, nocc = s.n, s.n_occupied
    assert (n, nocc) == (24, 16)
    H, S, C0 = s.H.to_dense(), s.S.to_dense(), s.C0.to_dense()
    w, X = scipy.linalg.eigh(H, S)
    assert w[nocc - 1] < eta < w[nocc]
    res = O.cg_minimize(H, S, C0, eta=eta, tol_grad=1e-9, max_iter=20000, n_occupied=nocc)
    assert res.converged
    assert abs(res.energy - 2.0 * (w[:nocc] - eta).sum()) / s.natoms <= 1e-10
    assert abs(res.energy_band - 2.0 * w[:nocc].sum()) / s.natoms <= 1e-10
    ev = np.linalg.eigvalsh(res.SW)
    assert np.max(np.abs(ev[:n - nocc])) <= 1e-6 and np.max(np.abs(ev[n - nocc:] - 1.0)) <= 1e-8
    assert abs(O.electron_count(res.SW) - 2 * nocc) <= 1e-8
    Xn = X[:, :nocc]
    assert np.max(np.abs(O.density_matrix(res.C, res.SW) - 2.0 * Xn @ Xn.T)) <= 1e-8
    rho_e = O.energy_density_matrix(res.C, res.HW, res.SW, eta)
    assert np.max(np.abs(rho_e - 2.0 * Xn @ np.diag(w[:nocc]) @ Xn.T)) <= 1e-8


# ------------------------------------------------------------ kinetic preconditioning (Eq. 7)
@pytest.fixture(scope="module")
def kinetic4():
    from dataclasses import replace
    s = make_system(replace(config_spec("cubic4_dense"), kinetic=30.0))
    return s, s.H.to_dense(), s.S.to_dense(), s.C0.to_dense(), s.T.to_dense()


def test_identity_preconditioner_is_plain_cg(chain):
    s, H, S, C0 = chain
    plain = O.cg_minimize(H, S, C0, tol_grad=1e-9)
    ident = O.cg_minimize(H, S, C0, tol_grad=1e-9, precon=np.eye(s.m))
    assert ident.iterations == plain.iterations
    for a, b in zip(plain.history, ident.history):
        assert a["E"] == b["E"] and a["x"] == b["x"] and a["beta"] == b["beta"]


def test_preconditioned_cg_reaches_the_same_minimum_faster(kinetic4):
    # Sec. II: preconditioning changes the path, not the minimum; with the kinetic
    # scale of Table 1's default order it needs far fewer CG iterations here
    s, H, S, C0, T = kinetic4
    P = O.kinetic_preconditioner(S, T, 5.0)
    assert np.max(np.abs(P @ (S + T / 5.0) - np.eye(s.m))) <= 1e-10
    plain = O.cg_minimize(H, S, C0, tol_grad=1e-9, max_iter=5000)
    pre = O.cg_minimize(H, S, C0, tol_grad=1e-9, max_iter=5000, precon=P)
    assert plain.converged and pre.converged
    Estar, rho_star, _ = _eigen(H, S, s.n)
    assert abs(pre.energy - Estar) / s.natoms <= 1e-10
    assert np.max(np.abs(O.density_matrix(pre.C, pre.SW) - rho_star)) <= 1e-8
    assert pre.iterations * 2 < plain.iterations
    # every step is a descent step: c1 = <dE/dC, D> < 0
    assert all(h["c"][1] < 0.0 for h in pre.history)


# Preconditioned CG with P = (U^T U)^-1 is plain CG on the problem transformed by U
# (Sec. II, Eq. 7 and the Cholesky reduction): with C = U^-1 C~ the functional is
# the same, the gradient maps as G~ = U^-T G, so -G~ + beta D~ maps back to
# -P G + beta D and the plain Polak-Ribiere ratio <G~, G~ - G~_old>/<G~_old, G~_old>
# equals <P G, G - G_old>/<P G_old, G_old>.  Step lengths, energies and betas must
# agree iteration by iteration.
def _same_trajectory(a, b, k, rtol=1e-9):
    assert len(a.history) == len(b.history) == k
    for ha, hb in zip(a.history, b.history):
        assert abs(ha["E"] - hb["E"]) <= 1e-12 * abs(hb["E"])
        assert abs(ha["x"] - hb["x"]) <= rtol * abs(hb["x"])
        assert abs(ha["beta"] - hb["beta"]) <= rtol * max(abs(hb["beta"]), 1e-3)


def _transformed_plain_cg(H, S, C0, U, k):
    """Plain CG on H~ = U^-T H U^-1, S~ = U^-T S U^-1 from C~0 = U C0 (oracle, no preconditioner)."""
    Ui = scipy.linalg.solve_triangular(U, np.eye(U.shape[0]), lower=False)
    Ht = Ui.T @ H @ Ui
    St = Ui.T @ S @ Ui
    return O.cg_minimize(0.5 * (Ht + Ht.T), 0.5 * (St + St.T), U @ C0, tol_grad=0.0, max_iter=k)


@pytest.mark.parametrize("which", ["chain", "cube4"])
def test_preconditioner_inverse_overlap_is_the_cholesky_path(which, request):
    s, H, S, C0 = request.getfixturevalue(which)
    k = 12
    pre = O.cg_minimize(H, S, C0, tol_grad=0.0, max_iter=k, precon=np.linalg.inv(S))
    chol = O.cg_minimize_cholesky(H, S, C0, tol_grad=0.0, max_iter=k)
    _same_trajectory(pre, chol, k)


def test_kinetic_preconditioner_is_plain_cg_on_the_transformed_problem(kinetic4):
    s, H, S, C0, T = kinetic4
    k = 10
    U = scipy.linalg.cholesky(S + T / 5.0, lower=False)
    pre = O.cg_minimize(H, S, C0, tol_grad=0.0, max_iter=k, precon=O.kinetic_preconditioner(S, T, 5.0))
    ref = _transformed_plain_cg(H, S, C0, U, k)
    _same_trajectory(pre, ref, k)
    # the iterate maps back: C = U^-1 C~
    Cb = scipy.linalg.solve_triangular(U, ref.C, lower=False)
    assert np.max(np.abs(pre.C - Cb)) <= 1e-10 * np.max(np.abs(Cb))


def test_wrong_preconditioned_beta_is_detected(kinetic4):
    # the pin above separates the preconditioned Polak-Ribiere ratio from a
    # plausible slip: <P G, G - G_old> / <G_old, G_old> (unpreconditioned denominator)
    s, H, S, C0, T = kinetic4
    k = 6
    P = O.kinetic_preconditioner(S, T, 5.0)
    U = scipy.linalg.cholesky(S + T / 5.0, lower=False)
    ref = _transformed_plain_cg(H, S, C0, U, k)
    C = C0.copy()
    G = O.om_gradient(H, S, C)
    D = -(P @ G)
    hist = []
    for it in range(k):
        c = O.quartic_coefficients(H, S, C, D)
        x, ok = O.line_minimum(c)
        assert ok
        C = C + x * D
        E, Gn = O.om_energy(H, S, C), O.om_gradient(H, S, C)
        Z = P @ Gn
        beta = max(0.0, float(np.sum(Z * (Gn - G))) / float(np.sum(G * G)))   # the slip
        hist.append(dict(E=E, x=x, beta=beta))
        D = -Z + beta * D
        G = Gn
    with pytest.raises(AssertionError):
        assert len(hist) == k
        for ha, hb in zip(hist, ref.history):
            assert abs(ha["E"] - hb["E"]) <= 1e-12 * abs(hb["E"])
            assert abs(ha["x"] - hb["x"]) <= 1e-9 * abs(hb["x"])
            assert abs(ha["beta"] - hb["beta"]) <= 1e-9 * max(abs(hb["beta"]), 1e-3)


# ------------------------------------------------------------ block-sparse form of the oracle
# The scipy.sparse form (used where dense m x n matrices do not fit, the 4096-atom
# lattice) computes the same iterates as the plain dense form, which the tests above
# pin; it must follow it step for step on localized systems.
@pytest.mark.parametrize("name,k", [("cubic3_sparse", 25), ("cubic5_sparse", 12)])
def test_block_sparse_form_follows_the_dense_oracle(name, k):
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from _helpers import history_array, oracle_run, system
    s = system(name)
    ref = oracle_run(s, "sparse", tol_grad=0.0, max_iter=k)
    sp = O.cg_minimize_sparse(s.H.to_bsr(), s.S.to_bsr(), s.C0.to_bsr(), eta=s.spec.eta, tol_grad=0.0,
                              max_iter=k)
    a = history_array(ref)
    b = np.array([[h["E"], *h["c"], h["x"], h["gnorm"], h["beta"], float(h["restart"])] for h in sp.history])
    assert a.shape == b.shape == (k, 10)
    assert np.all(np.abs(a[:, 0] - b[:, 0]) <= 1e-12 * np.abs(a[:, 0]))            # E
    assert np.all(np.abs(a[:, 6] - b[:, 6]) <= 1e-9 * np.abs(a[:, 6]))             # x
    scale = np.max(np.abs(a[:, 1:6]), axis=0)
    assert np.all(np.abs(a[:, 1:6] - b[:, 1:6]) <= 1e-10 * scale)                   # c0..c4
    assert np.all(np.abs(a[:, 7] - b[:, 7]) <= 1e-9 * np.abs(a[:, 7]))             # ||G||
    assert np.array_equal(a[:, 9], b[:, 9])
    assert np.max(np.abs(sp.C.toarray() - ref.C)) <= 1e-12 * np.max(np.abs(ref.C))
    assert abs(sp.energy - ref.energy) <= 1e-12 * abs(ref.energy)


# ------------------------------------------------------------ filtering definition (Sec. V)
def test_filtered_method_at_threshold_zero_is_the_plain_method():
    import os
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from _helpers import history_array, system
    s = system("cubic3_sparse")
    H, S, C0, mask = s.H.to_dense(), s.S.to_dense(), s.C0.to_dense(), s.C0.pattern_mask()
    blocks = dict(row_blocks=[s.spec.norb] * s.natoms, col_blocks=[s.spec.wf_per_atom] * s.natoms)
    k = 30
    plain = O.cg_minimize(H, S, C0, mask=mask, eta=s.spec.eta, tol_grad=0.0, max_iter=k)
    filt = O.cg_minimize_filtered(H, S, C0, mask=mask, eta=s.spec.eta, tol_grad=0.0, max_iter=k, filter_eps=0.0,
                                  **blocks)
    a, b = history_array(plain), history_array(filt)
    assert np.all(np.abs(a[:, 0] - b[:, 0]) <= 1e-12 * np.abs(a[:, 0]))
    assert np.all(np.abs(a[:, 6] - b[:, 6]) <= 1e-9 * np.abs(a[:, 6]))
    assert np.max(np.abs(plain.C - filt.C)) <= 1e-12


def test_filtered_method_keeps_projections_symmetric_and_drops_small_blocks():
    import os
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from _helpers import system
    s = system("cubic3_sparse")
    H, S, C0, mask = s.H.to_dense(), s.S.to_dense(), s.C0.to_dense(), s.C0.pattern_mask()
    rb, cb = [s.spec.norb] * s.natoms, [s.spec.wf_per_atom] * s.natoms
    eps = 3e-3
    r = O.cg_minimize_filtered(H, S, C0, mask=mask, eta=s.spec.eta, tol_grad=0.0, max_iter=10, filter_eps=eps,
                               row_blocks=rb, col_blocks=cb)
    assert np.array_equal(r.SW, r.SW.T) and np.array_equal(r.HW, r.HW.T)
    # the start-up S_W is the filtered C^T f(S C) with its upper triangle mirrored: no
    # block of it (off the zero blocks) is below the threshold, some are zero
    SC = O.filter_blocks(S @ C0, rb, cb, eps)
    SW0 = O.upper_mirror(O.filter_blocks(C0.T @ SC, cb, cb, eps))
    n = SW0.shape[0]
    norms = np.sqrt((SW0.reshape(n // 2, 2, n // 2, 2) ** 2).sum(axis=(1, 3)))
    assert np.all((norms == 0.0) | (norms >= eps)) and np.any(norms == 0.0)
    # and the filtered run differs from the plain one
    p = O.cg_minimize(H, S, C0, mask=mask, eta=s.spec.eta, tol_grad=0.0, max_iter=10)
    assert abs(p.energy - r.energy) > 1e-9 * abs(p.energy)


# ------------------------------------------------------------ complex Hermitian (k-points)
def _rand_complex_problem(m=9, n=3, seed=3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    H = 0.5 * (A + A.conj().T)
    B = 0.1 * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    S = np.eye(m) + 0.5 * (B + B.conj().T)
    C = 0.3 * (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    D = 0.3 * (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    return H, S, C, D


def test_complex_gradient_finite_differences():
    # dE = Re <G, dC>: the real and imaginary parts of G are the derivatives along
    # the real and imaginary parts of each entry of C
    H, S, C, _ = _rand_complex_problem()
    G = O.om_gradient_complex(H, S, C)
    h = 1e-5
    num = np.zeros_like(C)
    for idx in np.ndindex(C.shape):
        for unit in (1.0, 1j):
            Cp, Cm = C.copy(), C.copy()
            Cp[idx] += h * unit
            Cm[idx] -= h * unit
            d = (O.om_energy_complex(H, S, Cp) - O.om_energy_complex(H, S, Cm)) / (2 * h)
            num[idx] += d * unit
    assert np.max(np.abs(num - G)) <= 1e-7 * np.max(np.abs(G))


def test_complex_quartic_exact():
    H, S, C, D = _rand_complex_problem(seed=4)
    c = O.quartic_coefficients_complex(H, S, C, D)
    for x in (-1.0, -0.5, 0.3, 1.0, 2.0):
        E = O.om_energy_complex(H, S, C + x * D)
        assert abs(O.quartic_value(c, x) - E) <= 1e-11 * max(1.0, abs(E))
    # c1 is the directional derivative Re <G, D>
    assert abs(c[1] - float(np.real(np.vdot(O.om_gradient_complex(H, S, C), D)))) <= 1e-10 * abs(c[1])


def test_complex_form_on_real_input_is_the_real_method(chain):
    s, H, S, C0 = chain
    k = 15
    a = O.cg_minimize(H, S, C0, tol_grad=0.0, max_iter=k)
    b = O.cg_minimize_complex(H.astype(complex), S.astype(complex), C0.astype(complex), tol_grad=0.0, max_iter=k)
    for ha, hb in zip(a.history, b.history):
        assert abs(ha["E"] - hb["E"]) <= 1e-13 * abs(ha["E"])
        assert abs(ha["x"] - hb["x"]) <= 1e-9 * abs(ha["x"])
    assert np.max(np.abs(a.C - b.C)) <= 1e-12


@pytest.mark.parametrize("kfrac", [(0.25, 0.0, 0.0), (0.25, 0.25, 0.5)])
def test_complex_k_point_converges_to_the_eigen_solution(kfrac):
    # Sec. II at a k-point: the minimum of Eq. 4 is 2 sum of the n lowest eigenvalues of
    # the Hermitian pencil (H(k), S(k)), with rho = 2 X X^+ (S-orthonormal X)
    from ommgen.systems import cubic_spec, make_bloch_system
    s = make_bloch_system(cubic_spec(3, 31, dense=True), kfrac)
    H, S, C0 = s.H.to_dense(), s.S.to_dense(), s.C0.to_dense()
    assert np.max(np.abs(H - H.conj().T)) == 0.0 and np.max(np.abs(H.imag)) > 1e-3
    r = O.cg_minimize_complex(H, S, C0, tol_grad=1e-9, max_iter=5000)
    assert r.converged
    w, X = scipy.linalg.eigh(H, S)
    n = s.n
    assert abs(r.energy - 2.0 * w[:n].sum()) / s.natoms <= 1e-10
    rho = O.density_matrix_complex(r.C, r.SW)
    assert np.max(np.abs(rho - 2.0 * X[:, :n] @ X[:, :n].conj().T)) <= 1e-8
    assert np.max(np.abs(r.SW - np.eye(n))) <= 1e-8
