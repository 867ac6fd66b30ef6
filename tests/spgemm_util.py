"""Helpers for the block-product tests: random operators on given atoms and
a dense assembly of block results (test-side, no library arithmetic)."""
import numpy as np

from workloads.core import Operator


def operator_on(b, seed, density=0.3, empty_rows=0, unsorted=False, scale_rows=None):
    """Random block pattern over the atoms ``b`` (values U[-1, 1]).

    ``scale_rows`` multiplies the blocks of row i by ``scale_rows[i]`` so that
    block norms spread over several decades (threshold tests)."""
    b = np.asarray(b, dtype=np.int32)
    n = b.shape[0]
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    if empty_rows:
        mask[rng.choice(n, size=min(empty_rows, n), replace=False), :] = False
    rows, cols = np.nonzero(mask)
    if unsorted:
        order = np.lexsort((rng.random(rows.shape[0]), rows))
        rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    sizes = b[rows].astype(np.int64) * b[cols].astype(np.int64)
    values = rng.uniform(-1.0, 1.0, size=int(sizes.sum()))
    if scale_rows is not None:
        values *= np.repeat(np.asarray(scale_rows)[rows], sizes)
    return Operator("pattern", b, row_ptr, cols.astype(np.int32), values,
                    np.zeros(cols.shape[0]), {"seed": seed})


def dense_of_blocks(b, rows, rp, col, values):
    """Dense matrix of a block result given per row ``rows[t]`` the columns
    ``col[rp[t]:rp[t+1]]`` and row-major blocks back to back in ``values``."""
    b = np.asarray(b, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(b)])
    D = np.zeros((off[-1], off[-1]))
    pos = 0
    for t, i in enumerate(rows):
        for c in range(rp[t], rp[t + 1]):
            j = col[c]
            sz = b[i] * b[j]
            D[off[i]:off[i + 1], off[j]:off[j + 1]] = values[pos:pos + sz].reshape(b[i], b[j])
            pos += sz
    assert pos == len(values)
    return D


def blocks_dict(op):
    """{(i, j): dense block} of an operator."""
    out = {}
    base = op.block_base
    r = op.block_rows
    for k in range(op.nnzb):
        i, j = int(r[k]), int(op.col_idx[k])
        out[(i, j)] = op.values[base[k]:base[k + 1]].reshape(int(op.b[i]), int(op.b[j]))
    return out
