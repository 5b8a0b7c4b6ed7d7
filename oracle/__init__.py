"""Plain, slow CPU FP64 oracle for the conjugate-gradient orbital minimization method.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import it; the GPU library never does and
shares no code with it.  Every function cites the passage of arXiv 2209.05934
(Lebedeva, Garcia, Artacho, Ordejon) it follows.

Pins (see tests/test_oracle_*.py): finite-difference gradient, exactness of
the quartic along a line, line-search root choice against a brute-force grid,
converged dense energy and density matrix against the generalized
eigendecomposition (also with more wavefunctions than occupied states, Kim
functional), the energy density as minus the derivative of the functional with
respect to S and its eigen form at the minimum, the identities of Eqs. 1, 2, 5
and Listing 1, Cholesky
variant == plain variant, unlimited localization radius == dense, and a
brute-force BFGS minimum on tiny localized inputs.  Product filtering with a
positive threshold follows one definition (`cg_minimize_filtered`): at
threshold 0 it is the plain method; above it, "parity unpinned" against any
closed form (the difference from the unfiltered minimum is only reported).
"""

from .omm import (  # noqa: F401
    kim_shift,
    projections,
    om_energy,
    om_gradient,
    project,
    quartic_coefficients,
    quartic_from_projections,
    quartic_value,
    line_minimum,
    cg_minimize,
    cg_minimize_sparse,
    cg_minimize_filtered,
    cg_minimize_complex,
    quartic_coefficients_complex,
    om_energy_complex,
    om_gradient_complex,
    density_matrix_complex,
    cholesky_reduce,
    kinetic_preconditioner,
    cg_minimize_cholesky,
    density_matrix,
    energy_density_matrix,
    electron_count,
    exact_band_energy,
    filter_blocks,
    upper_mirror,
    CGResult,
)
