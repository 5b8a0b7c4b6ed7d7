"""Seeded synthetic inputs for orbital-minimization (OMM) runs.

This package only builds inputs: atom positions, the Hamiltonian H and overlap
S of a tight-binding-like model in atom-block sparse form, the localization
pattern of the coefficient matrix C and a random initial guess C0 inside it.
It holds none of the method's arithmetic (no functional, gradient, line search,
shift or factorisation); both the CPU oracle and the GPU library consume its
output.
"""

from .systems import (  # noqa: F401
    BlockMatrix,
    System,
    SystemSpec,
    make_system,
    config_spec,
    batch_specs,
    CONFIG_NAMES,
)
