"""The seeded input generators: determinism, structure and symmetry."""
import numpy as np
import pytest

from workloads import make_config, random_cube, sc_lattice, zincblende_sphere, random_pattern
from workloads.core import shuffle_columns
from test_oracle_pins import dense_of


def test_same_seed_same_bits():
    a, va = make_config("C1", scale=0.2, nrhs=3)
    b, vb = make_config("C1", scale=0.2, nrhs=3)
    assert np.array_equal(a.values, b.values) and np.array_equal(a.col_idx, b.col_idx)
    assert np.array_equal(va["X"], vb["X"])


def test_c2_lattice_has_19_blocks_per_row():
    op = sc_lattice(5, 2, seed=2)
    assert np.all(np.diff(op.row_ptr) == 19)
    assert op.nnzb == 19 * 125
    # distances are exactly 0, 1, sqrt(2)
    assert set(np.round(op.dist, 12)) == {0.0, 1.0, round(np.sqrt(2.0), 12)}


def _brute_pairs(pos, L, rc):
    n = pos.shape[0]
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(-1))
    i, j = np.nonzero((r < rc) & (np.arange(n)[:, None] < np.arange(n)[None, :]))
    return set(zip(i.tolist(), j.tolist()))


def test_random_cube_neighbours_match_brute_force():
    op = random_cube(250, 0.05, [(4, 125), (9, 125)], 6.0, 2.0, seed=17)
    rng = np.random.default_rng(17)
    L = op.meta["box"]
    pos = rng.uniform(0.0, L, size=(250, 3))   # same first draw as the generator
    want = _brute_pairs(pos, L, 6.0)
    rows = op.block_rows
    got = {(int(i), int(j)) for i, j in zip(rows, op.col_idx) if i < j}
    assert got == want
    assert np.all(op.col_idx[op.row_ptr[:-1]] <= np.arange(250))  # sorted, self present
    assert sorted(np.bincount(op.b)[[4, 9]].tolist()) == [125, 125]


def test_operators_are_symmetric():
    for op in (random_cube(120, 0.05, [(1, 30), (4, 40), (9, 50)], 5.0, 2.0, seed=3),
               sc_lattice(3, 3, seed=4),
               zincblende_sphere(9.0, 5.87, 13, 9, 5.37, seed=5),
               random_pattern(6, 25, density=0.3, symmetric=True)):
        D = dense_of(op)
        assert np.array_equal(D, D.T)


def test_zincblende_shells_and_passivation():
    op = zincblende_sphere(14.0, 5.87, 13, 9, 5.37, seed=3)
    b = op.b
    rows = op.block_rows
    # passivating atoms couple to themselves and exactly one host
    for i in np.nonzero(b == 1)[0]:
        cols = op.col_idx[op.row_ptr[i]:op.row_ptr[i + 1]]
        assert len(cols) == 2 and i in cols
        host = int(cols[cols != i][0])
        assert b[host] in (13, 9)
    # interior atoms have self + 4 + 12 + 12 = 29 blocks
    counts = np.diff(op.row_ptr)
    assert counts.max() == 29
    d = np.round(op.dist[(b[rows] != 1) & (b[op.col_idx] != 1) & (op.dist > 0)] / (5.87 / 4), 6)
    assert set(np.round(d ** 2, 4)) <= {3.0, 8.0, 11.0}


def test_shuffled_columns_same_operator():
    op = random_pattern(8, 15, density=0.4)
    sh = shuffle_columns(op, np.random.default_rng(1))
    assert not np.array_equal(op.col_idx, sh.col_idx)
    assert np.array_equal(dense_of(op), dense_of(sh))


@pytest.mark.parametrize("name", ["C1", "C5", "FD50"])
def test_species_counts_are_exact(name):
    op, _ = make_config(name, scale=0.1 if name != "FD50" else 1.0, nrhs=1)
    cnt = np.bincount(op.b)
    if name == "C1":
        assert cnt[4] == cnt[9] == op.n // 2
    elif name == "FD50":
        assert (cnt[1], cnt[4], cnt[9]) == (10, 20, 20)
    else:
        assert cnt[1] + cnt[4] + cnt[9] == op.n and abs(cnt[4] - 2 * cnt[1]) <= 2
