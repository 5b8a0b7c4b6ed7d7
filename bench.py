#!/usr/bin/env python3
"""Throughput of the conjugate-gradient OMM hot path on one MI355X.

Default workload: the 4096-atom lattice (16x16x16 atoms x 13 orbitals, N_basis
53248, N_occ 8192, C localized to radius 3.0, eta 1.5, filter 1e-6).  A step is
a fixed number of CG iterations (20) from the initial guess held in HBM: C
reset, the iterations through the C ABI, the density matrix (Eq. 5) into device
memory.  `value` = FP64 CG iterations per second over the timed steps.  Beside
it, for the block-sparse workloads, `to_accuracy` times the FP64, FP32 + FP64
and BF16 + FP64 forms to the same stop rule (relative energy change < 1e-9)
and gives each one's energy/atom error against the FP64 result, while the CPU
oracle times one CG iteration of the same system in a child process.  Prints
one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision fp64|fp32|bf16]
"""

from __future__ import annotations

import argparse
import collections
from dataclasses import replace
import tempfile
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "OMM CG iters/s & block GFLOP/s, FP64 vs mixed/batched at fixed E/atom err"

# workloads: generator config, solver form, stop rule
WORKLOADS = {
    "cubic4_dense": dict(cfg="cubic4_dense", mode="dense", max_iter=10000,
                         desc="4x4x4 periodic cubic lattice, 64 atoms x 13 orbitals, N_basis 832, "
                              "N_occ 128, dense cubic-scaling OMM, eta 0, CG to ||G||_F <= 1e-9"),
    "cubic4_cholesky": dict(cfg="cubic4_dense", mode="cholesky", max_iter=10000,
                            desc="same 64-atom system, dense OMM on the Cholesky-reduced problem, "
                                 "CG to ||G||_F <= 1e-9"),
    "cubic4_precon": dict(cfg="cubic4_dense", mode="dense", max_iter=10000, spec={"kinetic": 30.0}, tau=5.0,
                          desc="64-atom dense system with a synthetic kinetic matrix T (levels up to 30) added "
                               "to H, N_basis 832, N_occ 128, kinetic preconditioning P = (S + T/5)^-1, "
                               "CG to ||G||_F <= 1e-9"),
    "chain8": dict(cfg="chain8", mode="dense", max_iter=10000,
                   desc="periodic chain of 8 atoms x 4 orbitals, N_basis 32, N_occ 16, dense, "
                        "CG to ||G||_F <= 1e-9"),
    "cubic8_sparse": dict(cfg="cubic8_sparse", mode="sparse", max_iter=200,
                          desc="8x8x8 lattice, 512 atoms x 13 orbitals, N_basis 6656, N_occ 1024, "
                               "atom-block sparse, C radius 3.0, eta 1.5, filter 1e-6, 200 CG iterations"),
    "cubic8_kim": dict(cfg="cubic8_kim", mode="sparse", max_iter=200,
                       desc="8x8x8 lattice, 512 atoms x 13 orbitals, N_basis 6656, Kim functional with "
                            "3 wavefunctions per atom (1536) for N_occ 1024, atom-block sparse, C radius 3.0, "
                            "eta -0.25 (in the gap), filter 1e-6, 200 CG iterations"),
    "cubic16_mixed": dict(cfg="cubic16_mixed", mode="sparse", max_iter=20,
                          desc="16x16x16 lattice, 4096 atoms x 13 orbitals, N_basis 53248, N_occ 8192, "
                               "atom-block sparse, C radius 3.0, eta 1.5, filter 1e-6, 20 CG iterations "
                               "per step from the initial guess"),
}

BATCH_DESC = ("64 independent systems, n^3 cubic lattices with n uniform in 3..7 (27-343 atoms x 13 "
              "orbitals, 2 wavefunctions/atom), 32 dense (eta 0) + 32 block-sparse (C radius 3.0, eta 1.5, "
              "filter 1e-6), FP32 products then 5 FP64 iterations, at most 200 CG iterations each")

PEAKS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense TFLOP/s of MI355X

# HBM bytes per launch of a product step from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (calibrated against a plain device copy), keyed by workload, precision, step,
# group width and split, and valid only for the kernel sources they were taken
# with (sha256 prefix of the step's source file, tile_sched.hpp and tile_ops.hpp)
MEASURED_TRAFFIC = {
    ("cubic4_dense", "fp64", 0, 1, 1): (3.6204e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 1, 2): (3.6204e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 1, 4): (3.6240e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 1, 8): (3.7836e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 2, 1): (3.6149e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 2, 2): (3.6178e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 2, 4): (3.6162e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 2, 8): (3.6102e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 4, 1): (2.8091e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 4, 2): (2.8983e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 0, 4, 4): (2.9456e+07, "7f6ec2575e98f052"),
    ("cubic4_dense", "fp64", 1, -2, 1): (1.0626e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, -2, 2): (1.0635e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, -2, 4): (1.0589e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 1, 1): (1.6137e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 1, 2): (1.6144e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 1, 4): (1.6065e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 1, 8): (1.6011e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 2, 1): (1.6244e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 2, 2): (1.6268e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 2, 4): (1.6214e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 4, 1): (9.2210e+06, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 4, 2): (1.6353e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 1, 4, 4): (1.6428e+07, "abdca07b294c4edf"),
    ("cubic4_dense", "fp64", 2, 1, 1): (7.8307e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 1, 2): (7.8379e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 1, 4): (7.8215e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 1, 8): (7.8256e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 2, 1): (7.8150e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 2, 2): (7.8485e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 2, 4): (7.8413e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 2, 8): (8.2663e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 4, 1): (6.6911e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 4, 2): (6.9353e+06, "816809e26cfbb54b"),
    ("cubic4_dense", "fp64", 2, 4, 4): (7.0569e+06, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 0, 1, 1): (1.7805e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 1, 2): (1.8321e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 1, 4): (1.8490e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 1, 8): (1.8005e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 2, 1): (1.9325e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 2, 2): (1.7469e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 2, 4): (1.7972e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 2, 8): (1.7241e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 4, 1): (1.4959e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 4, 2): (1.4576e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 0, 4, 4): (1.6270e+10, "7f6ec2575e98f052"),
    ("cubic16_mixed", "fp64", 1, -2, 1): (4.4001e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, -2, 2): (4.2122e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, -2, 4): (4.1246e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 1, 1): (5.5531e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 1, 2): (5.4272e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 1, 4): (5.4060e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 1, 8): (5.3467e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 2, 1): (5.5304e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 2, 2): (5.4095e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 2, 4): (5.3789e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 4, 1): (5.6985e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 4, 2): (5.5591e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 1, 4, 4): (5.4714e+10, "abdca07b294c4edf"),
    ("cubic16_mixed", "fp64", 2, 1, 1): (1.6601e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 1, 2): (2.3474e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 1, 4): (3.2561e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 1, 8): (3.2583e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 2, 1): (2.6804e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 2, 2): (2.6253e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 2, 4): (3.2106e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 2, 8): (3.0459e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 4, 1): (3.3387e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 4, 2): (3.2287e+10, "816809e26cfbb54b"),
    ("cubic16_mixed", "fp64", 2, 4, 4): (3.2124e+10, "816809e26cfbb54b"),
}


STEP_SOURCES = ("dir_products.hip", "proj_products.hip", "grad_products.hip")


def kernel_source_hash(step: int) -> str:
    """Hash of the sources of one tile-product step's kernel (stored traffic is valid only for them)."""
    import hashlib
    h = hashlib.sha256()
    for f in (STEP_SOURCES[step], "tile_sched.hpp", "tile_ops.hpp"):
        with open(os.path.join(ROOT, "paper_2209_05934_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
HBM_PEAK = 8000.0                                         # GB/s
TIMING_REPS = 20                                          # back-to-back launches per timed product step


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 10; 20 for the small workloads)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 2; 3 for the small workloads)")
    ap.add_argument("--workload", default="cubic16_mixed", choices=sorted(WORKLOADS) + ["batch64"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--max-iter", type=int, default=None)
    ap.add_argument("--graph-iters", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run 5 device-to-device copies of BYTES (HBM counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the heuristic work split of the tile products instead of timing the variants")
    ap.add_argument("--to-accuracy", action="store_true",
                    help="only the time-to-accuracy comparison (FP64, FP32 + FP64, BF16 + FP64 to the stop rule "
                         "|dE/E| < 1e-9), as its own JSON line")
    ap.add_argument("--filter-eps", type=float, default=None,
                    help="product filter threshold of the block-sparse workloads (default: the workload's, 1e-6)")
    ap.add_argument("--no-to-accuracy", action="store_true",
                    help="skip the time-to-accuracy comparison of the block-sparse workloads")
    args = ap.parse_args()
    small = args.workload not in ("cubic16_mixed", "batch64")
    if args.steps is None:
        args.steps = 20 if small else 10
    if args.warmup is None:
        args.warmup = 3 if small else 2
    return args


def _scipy_csr(bm):
    """scipy.sparse CSR of an atom-block matrix (input conversion for the CPU leg)."""
    import numpy as np
    import scipy.sparse
    ro, co = bm.row_offsets(), bm.col_offsets()
    rows = bm.block_rows()
    r_list, c_list = [], []
    for k in range(bm.nnzb):
        i, j = int(rows[k]), int(bm.col_idx[k])
        rr, cc = np.meshgrid(np.arange(ro[i], ro[i + 1]), np.arange(co[j], co[j + 1]), indexing="ij")
        r_list.append(rr.ravel())
        c_list.append(cc.ravel())
    order = np.concatenate([np.arange(bm.val_off[k], bm.val_off[k] + (ro[int(rows[k]) + 1] - ro[int(rows[k])])
                                      * (co[int(bm.col_idx[k]) + 1] - co[int(bm.col_idx[k])]))
                            for k in range(bm.nnzb)])
    return scipy.sparse.csr_matrix((bm.val[order], (np.concatenate(r_list), np.concatenate(c_list))),
                                   shape=(int(ro[-1]), int(co[-1])))


def _cpu_info():
    import platform
    threads, blas = os.cpu_count() or 1, "unknown"
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
        blas = ", ".join(sorted({f"{i.get('internal_api')} {i.get('version')}" for i in info
                                 if i.get("user_api") == "blas"})) or blas
    except Exception:
        pass
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    return threads, blas, cpu


def cpu_baseline(system, spec, mode, max_iter, budget_s, tau=0.0):
    """The CPU oracle as it stands on a bounded sample of a dense workload: full
    solves of the same system, as many as fit the time budget."""
    import numpy as np
    import oracle as O
    threads, blas, cpu = _cpu_info()
    H, S = system.H.to_dense(), system.S.to_dense()
    C0 = system.C0.to_dense()
    kw = dict(eta=spec.eta, tol_grad=1e-9, max_iter=max_iter, keep_history=False)
    if tau > 0.0:
        kw["precon"] = O.kinetic_preconditioner(S, system.T.to_dense(), tau)
    iters, runs, t0 = 0, 0, time.perf_counter()
    while True:
        if mode == "cholesky":
            r = O.cg_minimize_cholesky(H, S, C0, **kw)
        else:
            r = O.cg_minimize(H, S, C0, **kw)
        iters += r.iterations
        runs += 1
        if time.perf_counter() - t0 >= budget_s or runs >= 200:
            break
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "CG iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{runs} full solve(s) of the same workload ({iters} CG iterations, {dt:.1f} s) with the "
                      f"NumPy/SciPy FP64 oracle, every product recomputed each iteration",
            "cpu": cpu, "blas": blas}


def cpu_leg_child(workload, out_path, budget_s):
    """Child process of the block-sparse workloads: the oracle's block-sparse form
    (scipy.sparse products, every product recomputed from C and D each
    iteration) on the same system from the same C0, one BLAS thread: the start-up
    evaluation, then CG iterations until the time budget is spent (at least
    one).  Writes the JSON of the cpu_baseline object to out_path."""
    import oracle as O
    from ommgen import config_spec, make_system
    wl = WORKLOADS[workload]
    spec = config_spec(wl["cfg"])
    system = make_system(spec)
    threads, blas, cpu = _cpu_info()
    H, S, C0 = system.H.to_bsr(), system.S.to_bsr(), system.C0.to_bsr()
    t0 = time.perf_counter()
    k = 1
    while True:   # runs of 1, 2, 4 ... iterations: the iteration times come from the history
        r = O.cg_minimize_sparse(H, S, C0, eta=spec.eta, tol_grad=0.0, max_iter=k)
        if time.perf_counter() - t0 >= budget_s or k >= wl["max_iter"]:
            break
        k *= 2
    secs = sum(h["seconds"] for h in r.history)
    out = {"value": len(r.history) / secs, "unit": "CG iters/s", "cores": 1, "kind": "oracle",
           "sample": f"{len(r.history)} CG iteration(s) of the same {system.natoms}-atom system from the same "
                     f"C0 with the oracle's block-sparse form (scipy.sparse products, every product "
                     f"recomputed from C and D each iteration, filter 0, one BLAS thread), {secs:.1f} s of "
                     f"iterations (the start-up evaluation before them not counted; "
                     f"{time.perf_counter() - t0:.0f} s of oracle time in all), run in a child process "
                     f"beside the GPU legs",
           "cpu": cpu, "blas": blas, "threads_available": os.cpu_count()}
    with open(out_path, "w") as f:
        json.dump(out, f)


def start_cpu_leg(workload, budget_s):
    import subprocess
    out = os.path.join(tempfile.gettempdir(), f"omm_cpu_leg_{os.getpid()}.json")
    env = dict(os.environ, OPENBLAS_NUM_THREADS="1", OMP_NUM_THREADS="1", MKL_NUM_THREADS="1")
    p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-leg", workload, out,
                          str(budget_s)], env=env, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)
    return p, out


def finish_cpu_leg(handle, timeout_s=600.0):
    p, out = handle
    try:
        _, err = p.communicate(timeout=timeout_s)
    except Exception:
        p.kill()
        p.communicate()
        return None
    if p.returncode != 0 or not os.path.exists(out):
        print(f"cpu leg failed: {err.decode(errors='replace')[-400:]}", file=sys.stderr)
        return None
    with open(out) as f:
        res = json.load(f)
    os.remove(out)
    return res


def batch_main(args):
    """64 uneven systems in one context (block-diagonal batch, graph replay) vs one context each."""
    import torch
    from ommgen import batch_specs, make_system
    from paper_2209_05934_amd import omm as L
    from paper_2209_05934_amd.solver import Context, Problem

    specs = batch_specs()
    systems = [make_system(sp) for sp in specs]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    prec = {"fp64": L.OMM_FP64, "fp32": L.OMM_FP32, "bf16": L.OMM_BF16}[
        args.precision if args.precision != "fp64" else "fp32"]
    max_iter = args.max_iter or 200
    probs, c0s = [], []
    for s in systems:
        hv, sv, cv = (torch.from_numpy(a).to(dev) for a in (s.H.val, s.S.val, s.C0.val))
        mode = L.OMM_DENSE if s.spec.dense else L.OMM_BLOCK_SPARSE
        probs.append(Problem(s.H, s.S, s.C0, s.n, mode, eta=s.spec.eta, H_val=hv, S_val=sv, C0_val=cv))
        c0s.append(cv)
    opts = dict(tol_grad=1e-9, max_iter=max_iter, precision=prec, fp64_refine_iters=5,
                lowprec_max_iter=max_iter - 10, filter_eps=1e-6, graph_iters=args.graph_iters, history=0,
                hip_stream=stream.cuda_stream, autotune=0 if args.no_autotune else 1)
    batch = Context(probs, **opts)
    singles = [Context([p], **opts) for p in probs]

    def run_batch():
        for i, s in enumerate(systems):
            batch.set_coeffs(i, s.C0, c0s[i])
        rc, reps = batch.minimize()
        return sum(r.iters_total for r in reps), reps

    def run_seq():
        tot, reps = 0, []
        for i, (s, c) in enumerate(zip(systems, singles)):
            c.set_coeffs(0, s.C0, c0s[i])
            rc, r = c.minimize()
            tot += r[0].iters_total
            reps.append(r[0])
        return tot, reps

    for _ in range(args.warmup):
        run_batch()
        run_seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_b = 0
    for _ in range(args.steps):
        n, reps_b = run_batch()
        it_b += n
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    it_s = 0
    for _ in range(args.steps):
        n, reps_s = run_seq()
        it_s += n
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    dE = max(abs(a.energy - b.energy) / s.natoms for a, b, s in zip(reps_b, reps_s, systems))
    sz = batch.sizes(-1)
    flops_iter_avg = sz.flops_alg_iter / len(systems)
    out = {
        "metric": METRIC, "value": it_b / dt_b, "unit": "CG iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt_b / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products (then 5 f64 iterations), f64 traces/line search",
        "data": "synthetic",
        "config": {"workload": "batch64: " + BATCH_DESC, "systems": len(systems),
                   "atoms_total": int(sum(s.natoms for s in systems))},
        "cg_iters_per_step": it_b / args.steps,
        "sequential": {"value": it_s / dt_s, "ms_per_step": dt_s / args.steps * 1e3,
                       "what": "the same 64 systems, one context each, solved one after another"},
        "speedup_vs_sequential": (it_b / dt_b) / (it_s / dt_s),
        "max_abs_dE_per_atom_batch_vs_sequential": dE,
        "avg_alg_flops_per_iter_per_system": flops_iter_avg,
        # a fixed iteration budget, not a fixed accuracy: how far each system of the batch got
        "status_counts": dict(collections.Counter(L.omm_status_str(r.status) for r in reps_b)),
        "grad_norm_max": max(r.grad_norm for r in reps_b),
        "per_system": [{"atoms": int(s.natoms), "dense": bool(s.spec.dense), "iters": int(r.iters_total),
                        "iters_fp64": int(r.iters_fp64), "status": L.omm_status_str(r.status),
                        "grad_norm": r.grad_norm} for r, s in zip(reps_b, systems)],
        "roofline": None, "cpu_baseline": None,
    }
    for c in singles:
        c.close()
    batch.close()
    print(json.dumps(out), flush=True)


def to_accuracy_legs(args, system, spec, Hv, Sv, C0v, stream):
    """Time to the same accuracy: FP64, FP32 + FP64 and BF16 + FP64 solves of one
    block-sparse system to the stop rule |2(E_n - E_n-1)/(E_n + E_n-1)| < 1e-9,
    each energy/atom against the FP64 one (the mixed-precision target is 1e-5
    Ha/atom).  A low-precision run switches to FP64 when its relative energy
    change falls below its switch point (1e-9 FP32, 1e-5 BF16) and ends after
    5 FP64 iterations or the stop rule.  Each solve is timed from a fresh context,
    minus the time of a one-iteration solve of the same kind (set-up: symbolic
    phase, graph capture)."""
    import torch
    from paper_2209_05934_amd import omm as L
    from paper_2209_05934_amd.solver import Context, Problem

    max_iter = 20000
    cache = os.path.join(tempfile.gettempdir(), f"omm_tune_{os.getpid()}.txt")
    prec_of = {"fp64": L.OMM_FP64, "fp32": L.OMM_FP32, "bf16": L.OMM_BF16}

    def solve(prec, mi):
        prob = Problem(system.H, system.S, system.C0, system.n, L.OMM_BLOCK_SPARSE, H_val=Hv, S_val=Sv,
                       C0_val=C0v)
        ctx = Context([prob], eta=spec.eta, tol_grad=1e-9, rel_tol=1e-9, max_iter=mi, precision=prec_of[prec],
                      filter_eps=spec.filter_eps, fp64_refine_iters=5, lowprec_max_iter=max(1, mi - 10),
                      graph_iters=args.graph_iters, history=0, hip_stream=stream.cuda_stream,
                      autotune=0 if args.no_autotune else 1, tune_cache=cache.encode())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_coeffs(0, system.C0, C0v)
        reps = (L.omm_report * 1)()      # a failed solve (e.g. no line minimum) is reported, not raised
        L.load().omm_minimize(ctx.ctx, reps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.close()
        return dt, reps[0]

    res = {}
    for prec in ("fp64", "fp32", "bf16"):
        solve(prec, 2)                   # fills the autotune cache for this precision
        t1, _ = solve(prec, 1)
        tn, r = solve(prec, max_iter)
        res[prec] = {"seconds": tn - t1, "iters": int(r.iters_total), "iters_fp64": int(r.iters_fp64),
                     "energy_per_atom": r.energy / system.natoms, "grad_norm": r.grad_norm,
                     "status": L.omm_status_str(r.status)}
        print(f"{prec}: {res[prec]['iters']} iterations in {res[prec]['seconds']:.2f} s", file=sys.stderr,
              flush=True)
    e64 = res["fp64"]["energy_per_atom"]
    for prec, v in res.items():
        v["abs_dE_per_atom_vs_fp64"] = abs(v["energy_per_atom"] - e64)
        v["within_1e-5"] = v["abs_dE_per_atom_vs_fp64"] <= 1e-5
        v["speedup_vs_fp64"] = res["fp64"]["seconds"] / v["seconds"]
        v["cg_iters_per_s"] = v["iters"] / v["seconds"]
    try:
        os.remove(cache)
    except OSError:
        pass
    return res


def accuracy_main(args):
    """Only the time-to-accuracy comparison, as its own JSON line."""
    import torch
    from ommgen import config_spec, make_system

    wl = WORKLOADS[args.workload]
    if wl["mode"] != "sparse":
        raise SystemExit("--to-accuracy applies to the block-sparse workloads")
    spec = config_spec(wl["cfg"])
    if args.filter_eps is not None:
        spec = replace(spec, filter_eps=args.filter_eps)
    system = make_system(spec)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    Hv, Sv, C0v = (torch.from_numpy(a).to(dev) for a in (system.H.val, system.S.val, system.C0.val))
    res = to_accuracy_legs(args, system, spec, Hv, Sv, C0v, stream)
    out = {
        "metric": METRIC, "value": res["fp32"]["cg_iters_per_s"], "unit": "CG iters/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": res["fp32"]["seconds"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 products (then f64 iterations), f64 traces/line search", "data": "synthetic",
        "config": {"workload": args.workload + ": " + wl["desc"].rsplit(", ", 1)[0]
                   + ", each precision to the stop rule |dE/E| < 1e-9", "atoms": int(system.natoms)},
        "to_accuracy": res,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    if len(sys.argv) == 5 and sys.argv[1] == "--cpu-leg":   # child process of the CPU leg
        cpu_leg_child(sys.argv[2], sys.argv[3], float(sys.argv[4]))
        return
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        import torch
        n = args.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 5}), flush=True)
        return
    if args.workload == "batch64":
        return batch_main(args)
    if args.to_accuracy:
        return accuracy_main(args)
    import numpy as np
    import torch
    from ommgen import config_spec, make_system
    from paper_2209_05934_amd import omm as L
    from paper_2209_05934_amd.solver import Context, Problem

    wl = WORKLOADS[args.workload]
    spec = config_spec(wl["cfg"], **wl.get("spec", {}))
    if args.filter_eps is not None and wl["mode"] == "sparse":
        spec = replace(spec, filter_eps=args.filter_eps)
    system = make_system(spec)
    tau = wl.get("tau", 0.0)
    mode = {"dense": L.OMM_DENSE, "cholesky": L.OMM_DENSE_CHOLESKY, "sparse": L.OMM_BLOCK_SPARSE}[wl["mode"]]
    prec = {"fp64": L.OMM_FP64, "fp32": L.OMM_FP32, "bf16": L.OMM_BF16}[args.precision]
    max_iter = args.max_iter or wl["max_iter"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    # inputs resident in HBM before the timed region
    Hv = torch.from_numpy(system.H.val).to(dev)
    Sv = torch.from_numpy(system.S.val).to(dev)
    C0v = torch.from_numpy(system.C0.val).to(dev)
    rho = torch.zeros(system.S.val.size, dtype=torch.float64, device=dev)
    prob = Problem(system.H, system.S, system.C0, system.n, mode, H_val=Hv, S_val=Sv, C0_val=C0v,
                   n_occupied=system.n_occupied, T=system.T if tau > 0.0 else None, tau=tau)
    ctx = Context([prob], eta=spec.eta, tol_grad=1e-9, max_iter=max_iter, precision=prec,
                  filter_eps=spec.filter_eps, graph_iters=args.graph_iters, history=0,
                  hip_stream=stream.cuda_stream, autotune=0 if args.no_autotune else 1)
    from paper_2209_05934_amd import omm as LL

    def step():
        ctx.set_coeffs(0, system.C0, C0v)
        reps = (LL.omm_report * 1)()     # a failed solve (e.g. no line minimum) shows in "status"
        LL.load().omm_minimize(ctx.ctx, reps)
        LL.omm_density_matrix(ctx.ctx, 0, rho)
        return reps[0]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    last = None
    for _ in range(args.steps):
        last = step()
        iters += last.iters_total
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sz = ctx.sizes(0)
    value = iters / dt
    flops_iter = sz.flops_alg_iter

    plain_cg = None
    if tau > 0.0:   # the same solves without the preconditioner, for the time to solution
        pctx = Context([Problem(system.H, system.S, system.C0, system.n, mode, H_val=Hv, S_val=Sv, C0_val=C0v)],
                       eta=spec.eta, tol_grad=1e-9, max_iter=max_iter, graph_iters=args.graph_iters, history=0,
                       hip_stream=stream.cuda_stream, autotune=0 if args.no_autotune else 1)
        for _ in range(args.warmup):
            pctx.minimize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pit = 0
        for _ in range(args.steps):
            rc, preps = pctx.minimize()
            pit += preps[0].iters_total
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t1
        plain_cg = {"cg_iters_per_solve": pit / args.steps, "ms_per_solve": pdt / args.steps * 1e3,
                    "cg_iters_per_s": pit / pdt, "energy": preps[0].energy,
                    "solve_time_ratio_plain_over_preconditioned": pdt / dt}
        pctx.close()

    # the two density outputs of a finished solve (Eq. 5 and the energy density of
    # Eq. 6), each a blocking call into a device buffer, host-timed
    rho_e = torch.zeros_like(rho)
    outputs_ms = {}
    for name, fn, buf in (("rho", LL.omm_density_matrix, rho), ("rho_E", LL.omm_energy_density, rho_e)):
        fn(ctx.ctx, 0, buf)
        t1 = time.perf_counter()
        for _ in range(5):
            fn(ctx.ctx, 0, buf)
        outputs_ms[name] = (time.perf_counter() - t1) / 5 * 1e3

    # per-launch device time of each product step with HIP events on the
    # library's stream: TIMING_REPS launches back to back (the tuned shape, the
    # operands of the last solve)
    roof = None
    if not args.no_kernel_timing:
        names = ["direction products (H D, S D)", "n x n projections", "gradient products"]
        avg_ms = [ctx.time_step(i, TIMING_REPS) for i in range(3)]
        k = int(np.argmax(avg_ms))
        avg_s = avg_ms[k] / 1e3
        if args.precision == "bf16":
            achieved = sz.bytes_alg_step[k] / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK, "traffic": None}
        else:
            achieved = sz.flops_alg_step[k] / avg_s / 1e12
            peak = PEAKS[args.precision]
            roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "traffic": None}
        tk = (args.workload, args.precision, k, int(sz.tile_group[k]), int(sz.tile_split[k]))
        if tk in MEASURED_TRAFFIC and MEASURED_TRAFFIC[tk][1] == kernel_source_hash(k):
            roof["traffic"] = MEASURED_TRAFFIC[tk][0]
        roof.update({"kernel": names[k], "tile_group": int(sz.tile_group[k]), "tile_split": int(sz.tile_split[k]),
                     "avg_launch_us": avg_s * 1e6, "launches": TIMING_REPS,
                     "alg_flops_per_launch": sz.flops_alg_step[k],
                     "exec_flops_per_launch": sz.flops_exec_step[k],
                     "alg_bytes_per_launch": sz.bytes_alg_step[k],
                     "step_us": {names[i]: avg_ms[i] * 1e3 for i in range(3)},
                     # every product step against the peak of its arithmetic: algorithmic
                     # (unpadded atom blocks) and executed (16 x 16 tiles) flops per launch
                     "steps": {names[i]: {"us": avg_ms[i] * 1e3, "alg_flops": sz.flops_alg_step[i],
                                          "exec_flops": sz.flops_exec_step[i],
                                          "alg_frac": sz.flops_alg_step[i] / (avg_ms[i] * 1e-3) / 1e12
                                          / PEAKS[args.precision],
                                          "exec_frac": sz.flops_exec_step[i] / (avg_ms[i] * 1e-3) / 1e12
                                          / PEAKS[args.precision],
                                          "alg_bytes": sz.bytes_alg_step[i]} for i in range(3)}})

    sparse = wl["mode"] == "sparse"
    cpu_leg = None
    if sparse and not args.no_cpu_baseline:    # the oracle runs beside the GPU legs below
        cpu_leg = start_cpu_leg(args.workload, args.cpu_seconds)
    to_acc = None
    if sparse and not args.no_to_accuracy:
        to_acc = to_accuracy_legs(args, system, spec, Hv, Sv, C0v, stream)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "CG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 products, f64 traces/line search",
                  "bf16": "bf16 products (f32 accumulate), f64 traces/line search"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + wl["desc"].replace("filter 1e-6", f"filter {spec.filter_eps:g}"),
                   "mode": wl["mode"],
                   "filter_eps": spec.filter_eps if wl["mode"] == "sparse" else None,
                   "precision": args.precision, "N_basis": int(system.m), "N_occ": int(system.n_occupied),
                   "N_wf": int(system.n), "atoms": int(system.natoms)},
        "cg_iters_per_step": iters / args.steps,
        "gflops_alg": flops_iter * value / 1e9,
        "alg_flops_per_iter": flops_iter,
        "exec_flops_per_iter": sz.flops_exec_iter,
        "energy": last.energy,
        "energy_per_atom": last.energy / system.natoms,
        "energy_band_per_atom": last.energy_band / system.natoms,
        "electron_count": last.electron_count,
        "status": LL.omm_status_str(last.status),
        "output_call_ms": outputs_ms,
        "plain_cg": plain_cg,
        "to_accuracy": to_acc,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if cpu_leg is not None:
        out["cpu_baseline"] = finish_cpu_leg(cpu_leg)
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(system, spec, wl["mode"], max_iter, args.cpu_seconds, tau)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
