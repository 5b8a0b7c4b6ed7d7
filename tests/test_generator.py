"""Seeded synthetic inputs: determinism, symmetry, definiteness, pattern radius."""

import numpy as np
import pytest

from ommgen import batch_specs, config_spec, make_system
from ommgen.systems import cubic_spec, _min_image


@pytest.fixture(scope="module")
def chain():
    return make_system(config_spec("chain8"))


@pytest.fixture(scope="module")
def cube4():
    return make_system(config_spec("cubic4_dense"))


def test_deterministic(chain):
    again = make_system(config_spec("chain8"))
    assert np.array_equal(chain.H.val, again.H.val)
    assert np.array_equal(chain.S.val, again.S.val)
    assert np.array_equal(chain.C0.val, again.C0.val)
    other = make_system(config_spec("chain8", seed=11))
    assert not np.array_equal(chain.H.val, other.H.val)


@pytest.mark.parametrize("name", ["chain8", "cubic4_dense"])
def test_symmetric_spd_gap(name):
    s = make_system(config_spec(name))
    H, S = s.H.to_dense(), s.S.to_dense()
    assert np.array_equal(H, H.T) and np.array_equal(S, S.T)
    assert np.linalg.eigvalsh(S)[0] > 0.5
    import scipy.linalg
    w = scipy.linalg.eigh(H, S, eigvals_only=True)
    assert w[s.n] - w[s.n - 1] > 1.0          # insulating gap around N_occ


def test_block_counts(chain, cube4):
    assert chain.H.nnzb == 8 * 5                 # self + 2 neighbours each side
    assert cube4.H.nnzb == 64 * 54               # 84% block fill (images summed)
    assert chain.m == 32 and chain.n == 16 and cube4.m == 832 and cube4.n == 128
    assert chain.C0.nnzb == 64 and cube4.C0.nnzb == 64 * 64
    assert abs(chain.extra["c0_sigma"] - 0.1) < 1e-15


def test_on_site_blocks(chain):
    H = chain.H.to_dense()
    d = np.diag(H)
    assert np.all(np.abs(d[0::4] + 1) < 0.1) and np.all(np.abs(d[2::4] - 1) < 0.1)
    S = chain.S.to_dense()
    assert np.array_equal(S[:4, :4], np.eye(4))


def test_c_pattern_radius():
    spec = cubic_spec(5, 123, dense=False)
    s = make_system(spec)
    rows = s.C0.block_rows()
    stored = set(zip(rows.tolist(), s.C0.col_idx.tolist()))
    for b in range(s.natoms):
        d = _min_image(s.pos - s.pos[b], s.box)
        r = np.sqrt((d ** 2).sum(-1))
        for a in range(s.natoms):
            assert ((b, a) in stored) == (r[a] <= spec.rc)


def test_hopping_cutoff(cube4):
    # every stored off-diagonal block belongs to a pair with an image within the cutoff
    s = cube4
    rows = s.H.block_rows()
    for k in range(0, s.H.nnzb, 7):
        i, j = int(rows[k]), int(s.H.col_idx[k])
        if i == j:
            continue
        d = _min_image(s.pos[j] - s.pos[i], s.box)
        assert np.sqrt((d ** 2).sum()) <= s.spec.cutoff


def test_batch_specs():
    specs = batch_specs()
    assert len(specs) == 64
    sides = [sp.dims[0] for sp in specs]
    assert min(sides) >= 3 and max(sides) <= 7
    assert sum(sp.dense for sp in specs) == 32
    assert len({sp.seed for sp in specs}) == 64


def test_kinetic_matrix():
    from dataclasses import replace
    base = make_system(config_spec("chain8"))
    s = make_system(replace(config_spec("chain8"), kinetic=10.0))
    T = s.T.to_dense()
    assert np.array_equal(T, T.T)
    assert np.linalg.eigvalsh(T).min() > 0.0
    # T has H's block pattern and is the only change to the inputs
    assert np.array_equal(s.T.col_idx, s.H.col_idx) and np.array_equal(s.T.row_ptr, s.H.row_ptr)
    assert np.allclose(s.H.to_dense() - base.H.to_dense(), T, atol=1e-14, rtol=0)
    assert np.array_equal(s.S.val, base.S.val) and np.array_equal(s.C0.val, base.C0.val)
    assert base.T is None
