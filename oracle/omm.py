"""CPU FP64 oracle: Ordejon-Mauri / Kim functional minimized by conjugate gradients.

TEST INFRASTRUCTURE ONLY (imported by tests/, __graft_entry__.smoke() and
bench.py's cpu_baseline leg; never by the GPU library, with which it shares no
code).  Plain NumPy/SciPy in float64.  Every product is recomputed from C and D
at every iteration; nothing is updated incrementally, blocked or fused.

Notation follows the paper (arXiv 2209.05934, Sec. II): H, S are the m x m
Hamiltonian and overlap in the atomic-orbital basis, C is the m x n coefficient
matrix (columns = wavefunctions, Eq. 3), H_W = C^T H C and S_W = C^T S C
(Eq. 3), and the functional is E~ = 2 Tr[(2I - S_W) H_W] (Eq. 4).  Matrices are
real (Gamma point, Sec. IV A).  H and S may be dense numpy arrays or
scipy.sparse matrices; C-shaped matrices are dense.

Readings where the paper is silent:
* gradient: the real gradient dE~/dC = 8HC - 4(HC S_W + SC H_W); the paper's
  G = dE~/d(C*) (Sec. III B) is half of it.  With an exact line search the CG
  iterates do not depend on that factor; only the norm threshold does.
* the gradient is projected on the sparsity pattern of the initial C
  ("keep_sparsity", Sec. III B); products are never restricted otherwise.
* CG direction update: Polak-Ribiere, beta = max(0, <G, G - G_old>/<G_old, G_old>);
  with kinetic preconditioning (Eq. 7) the gradient is multiplied by P, the
  direction follows -P G and beta = max(0, <P G, G - G_old>/<P G_old, G_old>).
* line search: the exact minimum of the quartic E~(C + xD) (Sec. I, ref. to
  the analytic quartic) reached by going downhill from x = 0: the smallest
  positive critical point with positive curvature.  When the quartic has no
  such minimum or the direction is not a descent direction (the failure mode
  of Sec. IV C), the step is x = 0 and the next direction is the steepest
  descent -G; if that already was the direction, the run fails.
* stop: projected gradient Frobenius norm <= tol_grad, or (if rel_tol > 0) the
  paper's relative energy change |2(E_n - E_{n-1})/(E_n + E_{n-1})| < rel_tol
  (Table 1, OMM.RelTol).
* Kim correction: the reported band energy is E~ + 2 eta n (2n electrons,
  Sec. II), i.e. the paper's "E~ + eta n" with its spin factor; n counts the
  occupied states, which may be fewer than the n' columns of C.  The energy
  density gets the matching correction rho_E + eta rho.
* filtering (Sec. V): the paper filters the block products it forms; which
  products a CG iteration forms is libOMM's business (only cited).  The reading
  taken (`cg_minimize_filtered`): each iteration forms the direction products
  H D, S D and the n x n projections C^T S D, C^T H D, D^T S D, D^T H D, and
  filters each of them (atom blocks of Frobenius norm < eps set to zero); H C,
  S C, H_W and S_W are formed and filtered once from C0 and afterwards follow
  the line steps as exact sums of those filtered products.  The n x n products
  that are symmetric without filtering (H_W, S_W, D^T H D, D^T S D) are kept
  symmetric, as in symmetric block storage: their blocks on and above the
  block diagonal are formed and filtered, each block below is the transpose of
  its mirror.  C, D, G, H and S are never filtered.  With eps = 0 this is the
  plain method.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg
import scipy.sparse


# ---------------------------------------------------------------- helpers
def _frob(A, B) -> float:
    """Frobenius inner product <A, B> = sum_ij A_ij B_ij."""
    if scipy.sparse.issparse(A):
        return float(A.multiply(B).sum())
    if scipy.sparse.issparse(B):
        return float(B.multiply(A).sum())
    return float(np.sum(np.asarray(A) * np.asarray(B)))


def _trace(A) -> float:
    return float(A.diagonal().sum())


def _dense(A) -> np.ndarray:
    return A.toarray() if scipy.sparse.issparse(A) else np.asarray(A)


# ---------------------------------------------------------------- Sec. II
def kim_shift(H, S, eta: float):
    """Kim functional, step (1) of Sec. II: eigenspectrum shift H -> H - eta S."""
    return H - eta * S


def projections(H, S, C) -> Tuple[np.ndarray, np.ndarray]:
    """H_W = C^T H C and S_W = C^T S C (Eq. 3, real C)."""
    return _dense(C.T @ (H @ C)), _dense(C.T @ (S @ C))


def om_energy(H, S, C) -> float:
    """Ordejon-Mauri functional E~ = 2 Tr[(2I - S_W) H_W] (Eq. 4)."""
    HW, SW = projections(H, S, C)
    n = HW.shape[0]
    return 2.0 * float(np.trace((2.0 * np.eye(n) - SW) @ HW))


def om_gradient(H, S, C) -> np.ndarray:
    """Real gradient of Eq. 4 with respect to C for symmetric H, S.

    E~ = 4 Tr(C^T H C) - 2 Tr(C^T S C C^T H C), so
    dE~/dC = 8 HC - 4 (HC S_W + SC H_W).
    """
    HC = _dense(H @ C)
    SC = _dense(S @ C)
    HW = C.T @ HC
    SW = C.T @ SC
    return 8.0 * HC - 4.0 * (HC @ SW + SC @ HW)


def project(G: np.ndarray, mask: Optional[np.ndarray]) -> np.ndarray:
    """Keep only the entries inside the pattern of the initial C (Sec. III B)."""
    return G if mask is None else np.where(mask, G, 0.0)


def exact_band_energy(H, S, C) -> float:
    """E = 2 Tr[S_W^{-1} H_W] (Eq. 2)."""
    HW, SW = projections(H, S, C)
    return 2.0 * float(np.trace(np.linalg.solve(SW, HW)))


def electron_count(SW: np.ndarray) -> float:
    """n_e = 2 Tr[(2I - S_W) S_W] (Listing 1)."""
    n = SW.shape[0]
    return 2.0 * float(np.trace((2.0 * np.eye(n) - SW) @ SW))


def density_matrix(C: np.ndarray, SW: np.ndarray, pattern: Optional[np.ndarray] = None) -> np.ndarray:
    """rho = 2 C (2I - S_W) C^T (Eq. 5), kept on S's pattern when given (Sec. III B)."""
    n = SW.shape[0]
    rho = 2.0 * C @ (2.0 * np.eye(n) - SW) @ C.T
    return rho if pattern is None else np.where(pattern, rho, 0.0)


def energy_density_matrix(C: np.ndarray, HW: np.ndarray, SW: np.ndarray, eta: float = 0.0,
                          pattern: Optional[np.ndarray] = None) -> np.ndarray:
    """rho_E = 2 C H_W C^T (Eq. 6), plus eta rho under the Kim shift (Sec. II, step 3).

    H_W here is C^T (H - eta S) C, the projection of the shifted Hamiltonian the
    functional is minimized with.  Kept on S's pattern when given (Sec. III B).
    """
    rho_e = 2.0 * C @ HW @ C.T + eta * density_matrix(C, SW)
    return rho_e if pattern is None else np.where(pattern, rho_e, 0.0)


# ---------------------------------------------------------------- filtering
def filter_blocks(A: np.ndarray, row_bsz: Optional[Sequence[int]],
                  col_bsz: Optional[Sequence[int]], eps: float) -> np.ndarray:
    """Zero every block whose Frobenius norm is strictly below eps (Sec. V)."""
    if eps <= 0.0 or row_bsz is None or col_bsz is None:
        return A
    ro = np.concatenate([[0], np.cumsum(row_bsz)])
    co = np.concatenate([[0], np.cumsum(col_bsz)])
    out = np.array(A, copy=True)
    for i in range(len(row_bsz)):
        for j in range(len(col_bsz)):
            blk = out[ro[i]:ro[i + 1], co[j]:co[j + 1]]
            if np.sqrt(np.sum(blk * blk)) < eps:
                blk[...] = 0.0
    return out


# ---------------------------------------------------------------- quartic
def quartic_coefficients(H, S, C, D, filt=None) -> np.ndarray:
    """Coefficients c0..c4 with E~(C + xD) = sum_k c_k x^k exactly.

    Substituting C + xD into Eq. 4:
      H_W(x) = H0 + x H1 + x^2 H2,  S_W(x) = S0 + x S1 + x^2 S2 with
      H0 = C^T H C, H1 = C^T H D + D^T H C, H2 = D^T H D (S likewise), and
      E~(x) = 4 Tr H_W(x) - 2 <S_W(x), H_W(x)>.
    `filt` (optional) = (f_mn, f_nn) filters applied to the m x n and n x n products.
    """
    f_mn, f_nn = filt if filt is not None else (lambda A: A, lambda A: A)
    HC, SC = f_mn(_dense(H @ C)), f_mn(_dense(S @ C))
    HD, SD = f_mn(_dense(H @ D)), f_mn(_dense(S @ D))
    H0, S0 = f_nn(C.T @ HC), f_nn(C.T @ SC)
    H1 = f_nn(C.T @ HD) + f_nn(D.T @ HC)
    S1 = f_nn(C.T @ SD) + f_nn(D.T @ SC)
    H2, S2 = f_nn(D.T @ HD), f_nn(D.T @ SD)
    return quartic_from_projections(H0, S0, H1, S1, H2, S2)


def quartic_from_projections(H0, S0, H1, S1, H2, S2) -> np.ndarray:
    """c0..c4 of E~(x) = 4 Tr H_W(x) - 2 <S_W(x), H_W(x)> (Eq. 4) for
    H_W(x) = H0 + x H1 + x^2 H2 and S_W(x) = S0 + x S1 + x^2 S2, collected by powers of x."""
    c0 = 4.0 * np.trace(H0) - 2.0 * _frob(S0, H0)
    c1 = 4.0 * np.trace(H1) - 2.0 * (_frob(S0, H1) + _frob(S1, H0))
    c2 = 4.0 * np.trace(H2) - 2.0 * (_frob(S0, H2) + _frob(S1, H1) + _frob(S2, H0))
    c3 = -2.0 * (_frob(S1, H2) + _frob(S2, H1))
    c4 = -2.0 * _frob(S2, H2)
    return np.array([c0, c1, c2, c3, c4], dtype=np.float64)


def quartic_value(c: Sequence[float], x: float) -> float:
    return float(c[0] + x * (c[1] + x * (c[2] + x * (c[3] + x * c[4]))))


def _dp(c, x):
    return c[1] + x * (2.0 * c[2] + x * (3.0 * c[3] + x * 4.0 * c[4]))


def _d2p(c, x):
    return 2.0 * c[2] + x * (6.0 * c[3] + x * 12.0 * c[4])


def line_minimum(c: Sequence[float]) -> Tuple[float, bool]:
    """First minimum of the quartic p(x) = sum c_k x^k along the descent direction.

    The step is the exact line minimum of Eq. 4 along D (Sec. I: the quartic's
    parameters are computed analytically).  With p'(0) = c1 < 0 the minimum
    reached by going downhill from x = 0 is the smallest positive root of the
    cubic p'(x) at which p'' > 0; farther minima lie where the Ordejon-Mauri
    functional is unbounded below and are not taken.  Roots come from the
    companion matrix (numpy.roots) and are polished by Newton steps.
    Returns (x*, True), or (nan, False) when c1 >= 0 or no such minimum exists
    (the failure mode of Sec. IV C).
    """
    if not c[1] < 0.0:
        return float("nan"), False
    coeffs = [4.0 * c[4], 3.0 * c[3], 2.0 * c[2], c[1]]
    roots = np.roots(coeffs)
    cands: List[float] = []
    for r in roots:
        if abs(r.imag) > 1e-7 * max(1.0, abs(r.real)):
            continue
        x = float(r.real)
        for _ in range(4):
            d2 = _d2p(c, x)
            if d2 == 0.0:
                break
            x -= _dp(c, x) / d2
        if x > 0.0 and _d2p(c, x) > 0.0:
            cands.append(x)
    if not cands:
        return float("nan"), False
    return min(cands), True


# ---------------------------------------------------------------- CG
@dataclass
class CGResult:
    C: np.ndarray
    energy: float              # shifted functional E~ at the final C
    energy_band: float         # E~ + 2 eta n
    iterations: int
    converged: bool
    status: str                # "ok", "not_converged", "no_line_min"
    grad_norm: float
    restarts: int
    HW: np.ndarray
    SW: np.ndarray
    history: List[dict] = field(default_factory=list)


def _block_filters(filter_eps, row_blocks, col_blocks):
    if filter_eps <= 0.0 or row_blocks is None or col_blocks is None:
        return None
    f_mn = lambda A: filter_blocks(A, row_blocks, col_blocks, filter_eps)   # noqa: E731
    f_nn = lambda A: filter_blocks(A, col_blocks, col_blocks, filter_eps)   # noqa: E731
    return f_mn, f_nn


def _energy_and_gradient(H, S, C, mask, filt):
    f_mn, f_nn = filt if filt is not None else (lambda A: A, lambda A: A)
    HC, SC = f_mn(_dense(H @ C)), f_mn(_dense(S @ C))
    HW, SW = f_nn(C.T @ HC), f_nn(C.T @ SC)
    n = HW.shape[0]
    E = 2.0 * float(np.trace((2.0 * np.eye(n) - SW) @ HW))
    G = project(8.0 * HC - 4.0 * (HC @ SW + SC @ HW), mask)
    return E, G, HW, SW


def cg_minimize(H, S, C0: np.ndarray, *, mask: Optional[np.ndarray] = None, eta: float = 0.0,
                tol_grad: float = 1e-9, rel_tol: float = 0.0, max_iter: int = 10000,
                filter_eps: float = 0.0, row_blocks=None, col_blocks=None,
                keep_history: bool = True, n_occupied: Optional[int] = None,
                precon: Optional[np.ndarray] = None) -> CGResult:
    """Minimize E~ (Eq. 4, with the Kim shift of Sec. II) by conjugate gradients.

    H, S: unshifted Hamiltonian and overlap; the shift H - eta S is applied here.
    C0: initial guess; `mask` is its sparsity pattern (None = dense).  Its
    column count n' may exceed the number n_occupied of occupied states (Kim
    functional, Sec. II step 2); n_occupied (default n') only enters the
    reported band energy E~ + 2 eta n_occupied.
    row_blocks/col_blocks: atom block sizes of the basis and of the
    wavefunctions, used only by filtering.
    precon: an m x m preconditioning matrix P (Eq. 7, `kinetic_preconditioner`)
    that multiplies the gradient (Sec. II); the direction then follows -P G and
    beta uses the preconditioned products <P G, G - G_old> / <P G_old, G_old>.
    """
    filt = _block_filters(filter_eps, row_blocks, col_blocks)
    if filt is not None:
        if precon is not None:
            raise ValueError("filtering applies to the block-sparse method, preconditioning to the dense one")
        return cg_minimize_filtered(H, S, C0, mask=mask, eta=eta, tol_grad=tol_grad, rel_tol=rel_tol,
                                    max_iter=max_iter, filter_eps=filter_eps, row_blocks=row_blocks,
                                    col_blocks=col_blocks, keep_history=keep_history, n_occupied=n_occupied)
    Heta = kim_shift(H, S, eta)
    C = project(np.array(C0, dtype=np.float64, copy=True), mask)
    n = C.shape[1] if n_occupied is None else int(n_occupied)
    E, G, HW, SW = _energy_and_gradient(Heta, S, C, mask, filt)
    pre = (lambda A: A) if precon is None else (lambda A: precon @ A)      # noqa: E731
    Z = pre(G)
    D = -Z
    steepest = True
    gg = _frob(G, G)
    zg = _frob(Z, G)
    history: List[dict] = []
    status, converged, it, restarts = "not_converged", False, 0, 0
    if np.sqrt(gg) <= tol_grad:
        status, converged = "ok", True
    while not converged and it < max_iter:
        it += 1
        c = quartic_coefficients(Heta, S, C, D, filt)
        x, ok = line_minimum(c)
        restart = False
        if not ok or c[1] >= 0.0:
            if steepest:
                status = "no_line_min"
                it -= 1
                break
            x, restart = 0.0, True
            restarts += 1
        C = C + x * D
        E_old = E
        E, G_new, HW, SW = _energy_and_gradient(Heta, S, C, mask, filt)
        gg_new = _frob(G_new, G_new)
        Z = pre(G_new)
        zg_new = _frob(Z, G_new)
        beta = 0.0 if restart else max(0.0, _frob(Z, G_new - G) / zg)
        if keep_history:
            history.append(dict(E=E, c=c.copy(), x=x, gnorm=np.sqrt(gg_new), beta=beta,
                                restart=restart))
        G, gg, zg = G_new, gg_new, zg_new
        if np.sqrt(gg) <= tol_grad:
            status, converged = "ok", True
            break
        if rel_tol > 0.0 and not restart and (E + E_old) != 0.0 and \
                abs(2.0 * (E - E_old) / (E + E_old)) < rel_tol:
            status, converged = "ok", True
            break
        D = -Z + beta * D
        steepest = (beta == 0.0)
    return CGResult(C=C, energy=E, energy_band=E + 2.0 * eta * n, iterations=it,
                    converged=converged, status=status, grad_norm=float(np.sqrt(gg)),
                    restarts=restarts, HW=HW, SW=SW, history=history)


# ---------------------------------------------------------------- filtered method (Sec. V)
def upper_mirror(A: np.ndarray) -> np.ndarray:
    """The symmetric matrix holding A's upper triangle (diagonal included): what a
    symmetric product keeps when only its blocks on and above the block diagonal
    are stored (blocks are contiguous, so that is the element-wise upper triangle)."""
    return np.triu(A) + np.triu(A, 1).T


def cg_minimize_filtered(H, S, C0: np.ndarray, *, mask: Optional[np.ndarray] = None, eta: float = 0.0,
                         tol_grad: float = 1e-9, rel_tol: float = 0.0, max_iter: int = 10000,
                         filter_eps: float = 0.0, row_blocks=None, col_blocks=None,
                         keep_history: bool = True, n_occupied: Optional[int] = None) -> CGResult:
    """CG on Eq. 4 with filtering of the block products (Sec. V), in the form that
    forms each iteration only the products the line search needs.

    Start: HC = f(H C), SC = f(S C), H_W = u(f(C^T HC)), S_W = u(f(C^T SC)).
    Iteration: HD = f(H D), SD = f(S D); X = f(C^T SD), Y = f(C^T HD),
    S2 = u(f(D^T SD)), H2 = u(f(D^T HD)); the quartic of Eq. 4 along D has
    H1 = Y + Y^T, S1 = X + X^T (the symmetric H, S make D^T HC = (C^T HD)^T);
    u keeps the products that are symmetric without filtering symmetric
    (`upper_mirror`, after the block filter), so H_W and S_W stay symmetric;
    after the step x,
    C += x D, HC += x HD, SC += x SD, H_W += x H1 + x^2 H2, S_W += x S1 + x^2 S2,
    and the energy and projected gradient G = P[8 HC - 4 (HC S_W + SC H_W)] are
    those of the maintained products.  f zeroes the atom blocks of Frobenius norm
    below filter_eps (m x n products: basis x wavefunction blocks; n x n:
    wavefunction x wavefunction blocks).  Line search, beta and stop rules as in
    `cg_minimize`.  With filter_eps = 0 this is the plain method up to rounding.
    """
    f_mn = (lambda A: filter_blocks(A, row_blocks, col_blocks, filter_eps))   # noqa: E731
    f_nn = (lambda A: filter_blocks(A, col_blocks, col_blocks, filter_eps))   # noqa: E731
    f_sym = (lambda A: upper_mirror(f_nn(A)))                                # noqa: E731
    Heta = kim_shift(H, S, eta)
    C = project(np.array(C0, dtype=np.float64, copy=True), mask)
    n = C.shape[1] if n_occupied is None else int(n_occupied)
    HC, SC = f_mn(_dense(Heta @ C)), f_mn(_dense(S @ C))
    HW, SW = f_sym(C.T @ HC), f_sym(C.T @ SC)

    def energy_gradient():
        E = 4.0 * float(np.trace(HW)) - 2.0 * _frob(SW, HW)
        return E, project(8.0 * HC - 4.0 * (HC @ SW + SC @ HW), mask)

    E, G = energy_gradient()
    D = -G
    steepest = True
    gg = _frob(G, G)
    history: List[dict] = []
    status, converged, it, restarts = "not_converged", False, 0, 0
    if np.sqrt(gg) <= tol_grad:
        status, converged = "ok", True
    while not converged and it < max_iter:
        it += 1
        HD, SD = f_mn(_dense(Heta @ D)), f_mn(_dense(S @ D))
        X, Y = f_nn(C.T @ SD), f_nn(C.T @ HD)
        S2, H2 = f_sym(D.T @ SD), f_sym(D.T @ HD)
        H1, S1 = Y + Y.T, X + X.T
        c = quartic_from_projections(HW, SW, H1, S1, H2, S2)
        x, ok = line_minimum(c)
        restart = False
        if not ok or c[1] >= 0.0:
            if steepest:
                status = "no_line_min"
                it -= 1
                break
            x, restart = 0.0, True
            restarts += 1
        C = C + x * D
        HC, SC = HC + x * HD, SC + x * SD
        HW, SW = HW + x * H1 + x * x * H2, SW + x * S1 + x * x * S2
        E_old = E
        E, G_new = energy_gradient()
        gg_new = _frob(G_new, G_new)
        beta = 0.0 if restart else max(0.0, _frob(G_new, G_new - G) / gg)
        if keep_history:
            history.append(dict(E=E, c=c.copy(), x=x, gnorm=np.sqrt(gg_new), beta=beta, restart=restart))
        G, gg = G_new, gg_new
        if np.sqrt(gg) <= tol_grad:
            status, converged = "ok", True
            break
        if rel_tol > 0.0 and not restart and (E + E_old) != 0.0 and \
                abs(2.0 * (E - E_old) / (E + E_old)) < rel_tol:
            status, converged = "ok", True
            break
        D = -G + beta * D
        steepest = (beta == 0.0)
    return CGResult(C=C, energy=E, energy_band=E + 2.0 * eta * n, iterations=it,
                    converged=converged, status=status, grad_norm=float(np.sqrt(gg)),
                    restarts=restarts, HW=HW, SW=SW, history=history)


# ---------------------------------------------------------------- kinetic preconditioning
def kinetic_preconditioner(S, T, tau: float) -> np.ndarray:
    """P = (S + T / tau_T)^-1 (Eq. 7): T the kinetic-energy matrix, tau_T its scale
    (Table 1, OMM.TPreconScale).  Dense; cubic-scaling OMM only (Sec. II)."""
    return np.linalg.inv(_dense(S) + _dense(T) / tau)


# ---------------------------------------------------------------- Cholesky variant
def cholesky_reduce(H, S) -> Tuple[np.ndarray, np.ndarray]:
    """Reduce the generalized problem to standard form (Sec. II, Cholesky factorization).

    S = U^T U with U upper triangular, H~ = U^{-T} H U^{-1}.  Returns (H~, U).
    """
    Hd, Sd = _dense(H), _dense(S)
    U = scipy.linalg.cholesky(Sd, lower=False)
    A = scipy.linalg.solve_triangular(U, Hd, trans="T", lower=False)       # U^{-T} H
    Ht = scipy.linalg.solve_triangular(U, A.T, trans="T", lower=False).T   # (U^{-T} A^T)^T
    return Ht, U


def cg_minimize_cholesky(H, S, C0: np.ndarray, *, eta: float = 0.0, **kw) -> CGResult:
    """Cubic-scaling OMM on the Cholesky-reduced problem (dense only, Sec. II/III B).

    The shifted Hamiltonian H - eta S is reduced, the guess is mapped to
    C~0 = U C0, CG runs with S~ = I, and the result is mapped back C = U^{-1} C~.
    """
    Ht, U = cholesky_reduce(kim_shift(H, S, eta), S)
    m = Ht.shape[0]
    Ct0 = U @ np.asarray(C0, dtype=np.float64)
    res = cg_minimize(Ht, np.eye(m), Ct0, eta=0.0, **kw)
    C = scipy.linalg.solve_triangular(U, res.C, lower=False)
    n = kw.get("n_occupied") or C.shape[1]
    res.C = C
    res.energy_band = res.energy + 2.0 * eta * n
    return res


# ---------------------------------------------------------------- block-sparse form
# The same CG for a localized C held as a scipy.sparse BSR matrix (atom blocks,
# Sec. III B: zero blocks not stored), for systems whose dense m x n matrices
# are too large for the plain form above (the 4096-atom lattice).  Every
# product is still recomputed from C and D at every iteration; the only
# difference from `cg_minimize` is that the products of H and S with C and D
# are scipy.sparse products and that the projected gradient is evaluated only
# on the stored blocks of C (which is what the projection keeps).  No filtering
# (threshold 0) and no preconditioner.
def _bsr_on(P, data):
    """A BSR matrix with the block structure of P and the given block values."""
    return scipy.sparse.bsr_matrix((data, P.indices, P.indptr), shape=P.shape)


def _nn(A, B) -> np.ndarray:
    """A^T B as a dense n x n array (A, B sparse m x n)."""
    return (A.T @ B).toarray()


def _projected_gradient_blocks(P, HC, SC, HW, SW) -> np.ndarray:
    """Blocks of G = 8 HC - 4 (HC S_W + SC H_W) at the stored blocks of P (Sec. III B).

    Block row I of G needs row I of HC and SC (their stored WF blocks b) and the
    rows b, columns a (a the WF blocks of P in row I) of the dense S_W, H_W.
    """
    rb, cb = P.blocksize
    out = np.zeros_like(P.data)
    for I in range(P.shape[0] // rb):
        a_blk = P.indices[P.indptr[I]:P.indptr[I + 1]]
        if a_blk.size == 0:
            continue
        h0, h1 = HC.indptr[I], HC.indptr[I + 1]
        b_blk = HC.indices[h0:h1]
        assert np.array_equal(b_blk, SC.indices[SC.indptr[I]:SC.indptr[I + 1]])
        hc = HC.data[h0:h1].transpose(1, 0, 2).reshape(rb, -1)      # the blocks side by side: rb x (cb |b|)
        sc = SC.data[h0:h1].transpose(1, 0, 2).reshape(rb, -1)
        bcols = (b_blk[:, None] * cb + np.arange(cb)[None, :]).ravel()
        acols = (a_blk[:, None] * cb + np.arange(cb)[None, :]).ravel()
        g = -4.0 * (hc @ SW[np.ix_(bcols, acols)] + sc @ HW[np.ix_(bcols, acols)])
        pos = np.searchsorted(b_blk, a_blk)                         # P's blocks inside HC's row
        assert np.array_equal(b_blk[pos], a_blk), "C pattern outside H C's pattern"
        g += 8.0 * HC.data[h0:h1][pos].transpose(1, 0, 2).reshape(rb, -1)
        out[P.indptr[I]:P.indptr[I + 1]] = g.reshape(rb, a_blk.size, cb).transpose(1, 0, 2)
    return out


def cg_minimize_sparse(H, S, C0, *, eta: float = 0.0, tol_grad: float = 1e-9, rel_tol: float = 0.0,
                       max_iter: int = 10000, keep_history: bool = True) -> CGResult:
    """`cg_minimize` for a localized C given as a scipy.sparse BSR matrix (atom blocks).

    H, S: unshifted Hamiltonian and overlap as BSR matrices with square atom
    blocks; C0: BSR with blocks (basis atom) x (wavefunction atom), whose block
    pattern is kept fixed (Sec. III B).  Same functional (Eq. 4 with the Kim
    shift of Sec. II), gradient projection, quartic line search, Polak-Ribiere
    beta and stop rules as `cg_minimize`; the returned CGResult holds C as a
    BSR matrix and H_W, S_W as dense arrays.
    """
    Heta = scipy.sparse.bsr_matrix(H - eta * S, blocksize=H.blocksize)
    S = scipy.sparse.bsr_matrix(S, blocksize=H.blocksize)
    P = scipy.sparse.bsr_matrix(C0)
    P.sort_indices()
    C = _bsr_on(P, np.array(P.data, dtype=np.float64, copy=True))

    def energy_gradient(C):
        HC, SC = Heta @ C, S @ C
        HC.sort_indices()
        SC.sort_indices()
        HW, SW = _nn(C, HC), _nn(C, SC)
        n = HW.shape[0]
        E = 4.0 * np.trace(HW) - 2.0 * _frob(SW, HW)
        return E, _bsr_on(P, _projected_gradient_blocks(P, HC, SC, HW, SW)), HW, SW, n

    E, G, HW, SW, n = energy_gradient(C)
    D = _bsr_on(P, -G.data)
    steepest = True
    gg = float(np.sum(G.data * G.data))
    history: List[dict] = []
    status, converged, it, restarts = "not_converged", False, 0, 0
    if np.sqrt(gg) <= tol_grad:
        status, converged = "ok", True
    t_prev = time.perf_counter()
    while not converged and it < max_iter:
        it += 1
        HC, SC, HD, SD = Heta @ C, S @ C, Heta @ D, S @ D
        c = quartic_from_projections(_nn(C, HC), _nn(C, SC), _nn(C, HD) + _nn(D, HC),
                                     _nn(C, SD) + _nn(D, SC), _nn(D, HD), _nn(D, SD))
        x, ok = line_minimum(c)
        restart = False
        if not ok or c[1] >= 0.0:
            if steepest:
                status = "no_line_min"
                it -= 1
                break
            x, restart = 0.0, True
            restarts += 1
        C = _bsr_on(P, C.data + x * D.data)
        E_old = E
        E, G_new, HW, SW, n = energy_gradient(C)
        gg_new = float(np.sum(G_new.data * G_new.data))
        beta = 0.0 if restart else max(0.0, float(np.sum(G_new.data * (G_new.data - G.data))) / gg)
        t_now = time.perf_counter()
        if keep_history:   # `seconds`: wall time of the iteration (instrumentation only)
            history.append(dict(E=E, c=c.copy(), x=x, gnorm=np.sqrt(gg_new), beta=beta, restart=restart,
                                seconds=t_now - t_prev))
        t_prev = t_now
        G, gg = G_new, gg_new
        if np.sqrt(gg) <= tol_grad:
            status, converged = "ok", True
            break
        if rel_tol > 0.0 and not restart and (E + E_old) != 0.0 and \
                abs(2.0 * (E - E_old) / (E + E_old)) < rel_tol:
            status, converged = "ok", True
            break
        D = _bsr_on(P, -G.data + beta * D.data)
        steepest = (beta == 0.0)
    return CGResult(C=C, energy=E, energy_band=E + 2.0 * eta * n, iterations=it,
                    converged=converged, status=status, grad_norm=float(np.sqrt(gg)),
                    restarts=restarts, HW=HW, SW=SW, history=history)


# ---------------------------------------------------------------- complex Hermitian (k-points)
# The functional of Eq. 4 for complex Hermitian H, S (a k-point; the paper writes
# C^dagger throughout, Sec. II-III): H_W = C^dagger H C, S_W = C^dagger S C and
# E~ = 2 Tr[(2I - S_W) H_W], which is real.  The variables are the real and
# imaginary parts of C; with the real inner product Re <A, B> = Re sum conj(A) B
# the gradient is G = 8 HC - 4 (HC S_W + SC H_W) (dE~ = Re <G, dC>), twice the
# Wirtinger derivative dE~/dC*.  CG, line search and stop rules as in
# `cg_minimize`, with every inner product taken as Re <., .>.
def _rdot(A, B) -> float:
    """Re <A, B> = Re sum_ij conj(A_ij) B_ij."""
    return float(np.real(np.vdot(A, B)))


def _trace_prod(A, B) -> float:
    """Re Tr(A B) = Re sum_ij A_ij B_ji."""
    return float(np.real(np.sum(A * B.T)))


def quartic_coefficients_complex(H, S, C, D) -> np.ndarray:
    """c0..c4 with E~(C + xD) = sum_k c_k x^k for complex Hermitian H, S: H_W(x) =
    H0 + x H1 + x^2 H2 with H0 = C^+ H C, H1 = C^+ H D + D^+ H C, H2 = D^+ H D
    (S likewise) and E~(x) = 4 Re Tr H_W(x) - 2 Re Tr(S_W(x) H_W(x))."""
    Ch, Dh = C.conj().T, D.conj().T
    HC, SC, HD, SD = H @ C, S @ C, H @ D, S @ D
    H0, S0 = Ch @ HC, Ch @ SC
    H1, S1 = Ch @ HD + Dh @ HC, Ch @ SD + Dh @ SC
    H2, S2 = Dh @ HD, Dh @ SD
    tr = lambda A: float(np.real(np.trace(A)))   # noqa: E731
    c0 = 4.0 * tr(H0) - 2.0 * _trace_prod(S0, H0)
    c1 = 4.0 * tr(H1) - 2.0 * (_trace_prod(S0, H1) + _trace_prod(S1, H0))
    c2 = 4.0 * tr(H2) - 2.0 * (_trace_prod(S0, H2) + _trace_prod(S1, H1) + _trace_prod(S2, H0))
    c3 = -2.0 * (_trace_prod(S1, H2) + _trace_prod(S2, H1))
    c4 = -2.0 * _trace_prod(S2, H2)
    return np.array([c0, c1, c2, c3, c4], dtype=np.float64)


def om_energy_complex(H, S, C) -> float:
    """E~ = 2 Tr[(2I - S_W) H_W] with H_W = C^+ H C, S_W = C^+ S C (Eq. 3-4), real part."""
    Ch = C.conj().T
    HW, SW = Ch @ H @ C, Ch @ S @ C
    n = HW.shape[0]
    return 2.0 * float(np.real(np.trace((2.0 * np.eye(n) - SW) @ HW)))


def om_gradient_complex(H, S, C) -> np.ndarray:
    """G = 8 HC - 4 (HC S_W + SC H_W): dE~ = Re <G, dC> for Hermitian H, S."""
    HC, SC = H @ C, S @ C
    Ch = C.conj().T
    return 8.0 * HC - 4.0 * (HC @ (Ch @ SC) + SC @ (Ch @ HC))


def cg_minimize_complex(H, S, C0: np.ndarray, *, mask: Optional[np.ndarray] = None, eta: float = 0.0,
                        tol_grad: float = 1e-9, rel_tol: float = 0.0, max_iter: int = 10000,
                        keep_history: bool = True, n_occupied: Optional[int] = None) -> CGResult:
    """`cg_minimize` for complex Hermitian H, S (dense arrays) and complex C0."""
    Heta = np.asarray(H, dtype=np.complex128) - eta * np.asarray(S, dtype=np.complex128)
    S = np.asarray(S, dtype=np.complex128)
    C = project(np.array(C0, dtype=np.complex128, copy=True), mask)
    n = C.shape[1] if n_occupied is None else int(n_occupied)

    def energy_gradient(C):
        HC, SC = Heta @ C, S @ C
        Ch = C.conj().T
        HW, SW = Ch @ HC, Ch @ SC
        E = 4.0 * float(np.real(np.trace(HW))) - 2.0 * _trace_prod(SW, HW)
        return E, project(8.0 * HC - 4.0 * (HC @ SW + SC @ HW), mask), HW, SW

    E, G, HW, SW = energy_gradient(C)
    D = -G
    steepest = True
    gg = _rdot(G, G)
    history: List[dict] = []
    status, converged, it, restarts = "not_converged", False, 0, 0
    if np.sqrt(gg) <= tol_grad:
        status, converged = "ok", True
    while not converged and it < max_iter:
        it += 1
        c = quartic_coefficients_complex(Heta, S, C, D)
        x, ok = line_minimum(c)
        restart = False
        if not ok or c[1] >= 0.0:
            if steepest:
                status = "no_line_min"
                it -= 1
                break
            x, restart = 0.0, True
            restarts += 1
        C = C + x * D
        E_old = E
        E, G_new, HW, SW = energy_gradient(C)
        gg_new = _rdot(G_new, G_new)
        beta = 0.0 if restart else max(0.0, _rdot(G_new, G_new - G) / gg)
        if keep_history:
            history.append(dict(E=E, c=c.copy(), x=x, gnorm=np.sqrt(gg_new), beta=beta, restart=restart))
        G, gg = G_new, gg_new
        if np.sqrt(gg) <= tol_grad:
            status, converged = "ok", True
            break
        if rel_tol > 0.0 and not restart and (E + E_old) != 0.0 and \
                abs(2.0 * (E - E_old) / (E + E_old)) < rel_tol:
            status, converged = "ok", True
            break
        D = -G + beta * D
        steepest = (beta == 0.0)
    return CGResult(C=C, energy=E, energy_band=E + 2.0 * eta * n, iterations=it,
                    converged=converged, status=status, grad_norm=float(np.sqrt(gg)),
                    restarts=restarts, HW=HW, SW=SW, history=history)


def density_matrix_complex(C: np.ndarray, SW: np.ndarray) -> np.ndarray:
    """rho = 2 C (2I - S_W) C^+ (Eq. 5 with C^dagger)."""
    n = SW.shape[0]
    return 2.0 * C @ (2.0 * np.eye(n) - SW) @ C.conj().T
