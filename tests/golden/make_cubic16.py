"""Write the reference values of the first CG iterations of the 4096-atom system.

    python tests/golden/make_cubic16.py [iterations]

16x16x16 lattice, 4096 atoms x 13 orbitals (N_basis 53248), 2 wavefunctions
per atom (N_occ 8192), C localized to radius 3.0, Kim shift eta = 1.5, no
product filtering (threshold 0), C0 from the generator's seed.  The oracle's
block-sparse form (every product recomputed from C and D each iteration) runs
the first iterations and this script stores, per iteration, the energy, the
quartic coefficients c0..c4, the step x, the gradient norm and beta in
cubic16_first_iterations.json next to it.  It calls only the oracle and the
input generator; it takes about ten minutes on one CPU core.
"""

from __future__ import annotations

import json
import os
import sys
import time

# the gradient's many small dense products run fastest on one BLAS thread
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("OMP_NUM_THREADS", "1")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O                       # noqa: E402
from ommgen import config_spec, make_system   # noqa: E402


def main(k: int = 3) -> None:
    spec = config_spec("cubic16_mixed", filter_eps=0.0)
    t0 = time.time()
    s = make_system(spec)
    res = O.cg_minimize_sparse(s.H.to_bsr(), s.S.to_bsr(), s.C0.to_bsr(), eta=spec.eta, tol_grad=0.0,
                               max_iter=k)
    rows = [[h["E"], *[float(v) for v in h["c"]], h["x"], float(h["gnorm"]), h["beta"], float(h["restart"])]
            for h in res.history]
    out = {
        "what": "first CG iterations of the oracle's block-sparse form on the 4096-atom lattice",
        "system": {"name": spec.name, "dims": list(spec.dims), "norb": spec.norb,
                   "wf_per_atom": spec.wf_per_atom, "seed": spec.seed, "rc": spec.rc, "eta": spec.eta,
                   "filter_eps": 0.0, "N_basis": s.m, "N_occ": s.n},
        "columns": ["E", "c0", "c1", "c2", "c3", "c4", "x", "grad_norm", "beta", "restart"],
        "history": rows,
        "written_by": "tests/golden/make_cubic16.py (oracle.cg_minimize_sparse)",
        "cpu_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "cubic16_first_iterations.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["history"]), flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 3)
