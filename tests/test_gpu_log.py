"""The per-iteration JSONL log (omm_options.log_jsonl_path) against the history rows and the report."""

import json

import numpy as np
import pytest

from _helpers import oracle_run, history_array, system
from paper_2209_05934_amd import omm as L
from paper_2209_05934_amd.solver import Context, Problem

pytestmark = pytest.mark.gpu


def test_jsonl_log_matches_history_and_report(tmp_path):
    s = system("chain8")
    path = tmp_path / "omm.jsonl"
    ctx = Context([Problem(s.H, s.S, s.C0, s.n, L.OMM_DENSE)], eta=s.spec.eta, history=0,
                  log_jsonl_path=str(path).encode())
    rc, reps = ctx.minimize()
    r = reps[0]
    assert r.status == L.OMM_OK
    rows = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(rows) == r.iters_total
    assert [q["iter"] for q in rows] == list(range(1, r.iters_total + 1))
    assert all(q["solve"] == 1 and q["system"] == 0 and q["fp64"] for q in rows)
    h = ctx.history(0)          # the log turned history on: the same rows, as numbers
    assert h.shape[0] == r.iters_total
    for q, hr in zip(rows, h):
        assert q["energy"] == hr[0] and q["c"] == list(hr[1:6]) and q["x"] == hr[6]
        assert q["grad_norm"] == hr[7] and q["beta"] == hr[8] and q["restart"] == int(hr[9])
    assert rows[-1]["grad_norm"] == r.grad_norm <= 1e-9
    # the oracle's trajectory, as for the history rows
    ref = oracle_run(s, "dense", tol_grad=1e-9)
    ho = history_array(ref)
    k = min(10, len(ho))
    assert np.allclose([q["energy"] for q in rows[:k]], ho[:k, 0], rtol=1e-11, atol=1e-12)
    # a second solve appends its own rows
    ctx.set_coeffs(0, s.C0)
    ctx.minimize()
    rows2 = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(rows2) == 2 * r.iters_total and rows2[-1]["solve"] == 2
    ctx.close()
