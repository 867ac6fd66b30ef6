"""Translation-resolved (periodic) operators: input generation only.

A periodic real-space operator is a set of images O(R), one block-sparse
operator per integer lattice translation R, over the atoms of one cell
(paper, section 3.3).  Here it is one block graph whose blocks carry an image
index: block (i, j, m) couples atom i of the home cell to atom j of the cell
shifted by shifts[m].  The same (i, j) may appear under several images.
``tau`` holds the atoms' fractional positions in the cell (the R + tau phase
convention).  No operator arithmetic lives here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ImageOperator:
    name: str
    b: np.ndarray          # int32 [n]
    row_ptr: np.ndarray    # int64 [n+1]
    col_idx: np.ndarray    # int32 [nnzb]
    image: np.ndarray      # int32 [nnzb]
    shifts: np.ndarray     # int32 [n_images, 3]
    values: np.ndarray     # float64, graph order, row-major blocks
    tau: np.ndarray        # float64 [n, 3]

    @property
    def n(self):
        return int(self.b.shape[0])

    @property
    def N(self):
        return int(self.b.astype(np.int64).sum())

    @property
    def nnzb(self):
        return int(self.col_idx.shape[0])

    @property
    def block_rows(self):
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    @property
    def block_sizes(self):
        r = self.block_rows
        return self.b[r].astype(np.int64) * self.b[self.col_idx].astype(np.int64)

    @property
    def nnz(self):
        return int(self.block_sizes.sum())


def from_cube(op) -> ImageOperator:
    """The periodic form of a ``random_cube`` operator with the box as the
    unit cell: block (i, j) couples atom i to the minimum image of atom j,
    which lies in the cell shifted by R = -round((p_j - p_i) / L)."""
    pos, L = op.meta["pos"], op.meta["box"]
    rows = op.block_rows
    d = pos[op.col_idx] - pos[rows]
    R = -np.round(d / L).astype(np.int32)
    shifts, image = np.unique(R, axis=0, return_inverse=True)
    return ImageOperator(op.name + "-periodic", op.b, op.row_ptr, op.col_idx,
                         image.astype(np.int32).ravel(), shifts.astype(np.int32), op.values,
                         pos / L)


def random_images(seed: int, n: int, n_shifts: int = 3, bset=(1, 2, 4, 9, 13),
                  density: float = 0.15, hermitian: bool = True, empty_rows: int = 0,
                  unsorted: bool = True, name: str = "random_images") -> ImageOperator:
    """Random periodic operator: images R = 0 and +-R_1 .. +-R_{n_shifts}
    (random integer vectors), random block patterns with overlapping (i, j)
    across images, U[-1, 1] values.  ``hermitian`` makes O(-R) = O(R)^T."""
    rng = np.random.default_rng(seed)
    b = rng.choice(np.asarray(bset, dtype=np.int32), size=n).astype(np.int32)
    sh = [np.zeros(3, np.int32)]
    while len(sh) < 1 + 2 * n_shifts:
        r = rng.integers(-2, 3, size=3).astype(np.int32)
        if not any(np.array_equal(r, x) or np.array_equal(-r, x) for x in sh):
            sh += [r, -r]
    shifts = np.array(sh, dtype=np.int32)
    masks = [None] * len(sh)
    masks[0] = rng.random((n, n)) < density
    if hermitian:
        masks[0] = np.triu(masks[0]) | np.triu(masks[0]).T
    for m in range(1, len(sh), 2):
        masks[m] = rng.random((n, n)) < density
        masks[m + 1] = masks[m].T.copy() if hermitian else rng.random((n, n)) < density
    if empty_rows:
        er = rng.choice(n, size=min(empty_rows, n), replace=False)
        for M in masks:
            M[er, :] = False
            if hermitian:
                M[:, er] = False
    ent = []  # (i, j, m)
    for m, M in enumerate(masks):
        ii, jj = np.nonzero(M)
        ent += list(zip(ii.tolist(), jj.tolist(), [m] * ii.size))
    ent.sort()
    if unsorted:
        rng.shuffle(ent)
        ent.sort(key=lambda t: t[0])
    rows = np.array([e[0] for e in ent], dtype=np.int64)
    cols = np.array([e[1] for e in ent], dtype=np.int32)
    imgs = np.array([e[2] for e in ent], dtype=np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    sizes = b[rows].astype(np.int64) * b[cols].astype(np.int64)
    base = np.zeros(len(ent) + 1, dtype=np.int64)
    np.cumsum(sizes, out=base[1:])
    values = rng.uniform(-1, 1, size=int(base[-1]))
    if hermitian:
        pos = {e: t for t, e in enumerate(ent)}
        partner = {0: 0}
        for m in range(1, len(sh), 2):
            partner[m], partner[m + 1] = m + 1, m
        for t, (i, j, m) in enumerate(ent):
            u = pos[(j, i, partner[m])]
            if (i, j, m) < (j, i, partner[m]) or t == u:
                blk = values[base[t]:base[t + 1]].reshape(b[i], b[j])
                if t == u:
                    blk = np.triu(blk) + np.triu(blk, 1).T
                    values[base[t]:base[t + 1]] = blk.ravel()
                else:
                    values[base[u]:base[u + 1]] = blk.T.ravel()
    tau = rng.uniform(0, 1, size=(n, 3))
    return ImageOperator(name, b, row_ptr, cols, imgs, shifts, values, tau)
