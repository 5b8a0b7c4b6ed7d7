"""MI355X (gfx950) conjugate-gradient orbital minimization (arXiv 2209.05934).

The product is the C-ABI library built from `csrc/` (header `include/omm.h`);
`omm` is its thin ctypes binding and `solver` a convenience layer over it.
"""

from . import omm  # noqa: F401
from .build import build, lib_path  # noqa: F401
