"""Geometry, neighbour graphs and symmetric block values (input generation only)."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree


@dataclass
class Operator:
    """A square block-sparse operator in graph order.

    ``b``        int32 [n]      orbitals per atom (block size)
    ``row_ptr``  int64 [n+1]    block-row pointers (block units)
    ``col_idx``  int32 [nnzb]   block column (atom) indices, ascending per row
    ``values``   float64 [nnz]  block values, graph order, each block row-major
    ``dist``     float64 [nnzb] pair distance of each stored block (0 for self)
    """
    name: str
    b: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    dist: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.b.shape[0])

    @property
    def off(self) -> np.ndarray:
        o = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(self.b, out=o[1:])
        return o

    @property
    def N(self) -> int:
        return int(self.b.astype(np.int64).sum())

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def block_rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    @property
    def block_sizes(self) -> np.ndarray:
        """int64 [nnzb]: b_i * b_j of every stored block, graph order."""
        r = self.block_rows
        return self.b[r].astype(np.int64) * self.b[self.col_idx].astype(np.int64)

    @property
    def nnz(self) -> int:
        return int(self.block_sizes.sum())

    @property
    def block_base(self) -> np.ndarray:
        """int64 [nnzb+1]: start of every block in ``values``."""
        s = np.zeros(self.nnzb + 1, dtype=np.int64)
        np.cumsum(self.block_sizes, out=s[1:])
        return s

    def summary(self) -> dict:
        return {"name": self.name, "n": self.n, "N": self.N, "nnzb": self.nnzb,
                "nnz": self.nnz, **self.meta}


# --------------------------------------------------------------------------
# graph assembly
# --------------------------------------------------------------------------

def _graph_from_pairs(n: int, pi: np.ndarray, pj: np.ndarray, pd: np.ndarray):
    """Symmetric CSR block pattern from unordered pairs ``pi < pj`` plus self."""
    pi = np.asarray(pi, dtype=np.int64)
    pj = np.asarray(pj, dtype=np.int64)
    ar = np.arange(n, dtype=np.int64)
    rows = np.concatenate([ar, pi, pj])
    cols = np.concatenate([ar, pj, pi])
    dist = np.concatenate([np.zeros(n), pd, pd])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate pair in neighbour list")
    rows, cols, dist = rows[order], cols[order], dist[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), dist


def _tri_index(b: int) -> np.ndarray:
    """(b*b,) map from a full row-major b x b position to its upper-triangle slot."""
    p, q = np.divmod(np.arange(b * b), b)
    lo, hi = np.minimum(p, q), np.maximum(p, q)
    return lo * b - lo * (lo - 1) // 2 + (hi - lo)


def _symmetric_values(rng, b, row_ptr, col_idx, dist, decay, chunk=200_000):
    """Symmetric block values ``U[-1,1] * exp(-r/decay)``, graph order.

    Draw order: one ``uniform(-1, 1)`` stream whose consecutive segments
    belong to the upper blocks ``i <= j`` in ascending ``(i, j)``; a block with
    ``i < j`` takes ``b_i*b_j`` numbers (row-major), a self block takes
    ``b_i(b_i+1)/2`` numbers (its upper triangle row by row).  Lower blocks are
    the transposes of their mirror images.
    """
    n = b.shape[0]
    nnzb = col_idx.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    cols = col_idx.astype(np.int64)
    bi = b[rows].astype(np.int64)
    bj = b[cols].astype(np.int64)
    sizes = bi * bj
    gbase = np.zeros(nnzb + 1, dtype=np.int64)
    np.cumsum(sizes, out=gbase[1:])

    upper = rows <= cols
    seg_len = np.where(rows == cols, bi * (bi + 1) // 2, sizes)
    seg_len = np.where(upper, seg_len, 0)
    seg = np.zeros(nnzb + 1, dtype=np.int64)
    np.cumsum(seg_len, out=seg[1:])
    U = rng.uniform(-1.0, 1.0, size=int(seg[-1]))

    # index of the mirror block (j, i) of every block (i, j)
    key = rows * n + cols
    mirror = np.searchsorted(key, cols * n + rows)
    w = np.exp(-dist / decay)

    values = np.empty(int(gbase[-1]), dtype=np.float64)
    shapes = np.unique(np.stack([bi, bj], axis=1), axis=0)
    for sbi, sbj in shapes:
        sbi, sbj = int(sbi), int(sbj)
        sel_shape = (bi == sbi) & (bj == sbj)
        ar = np.arange(sbi * sbj, dtype=np.int64)
        # element (p, q) of a lower block is element (q, p) of its mirror
        p, q = np.divmod(ar, sbj)
        transposed = q * sbi + p
        for kind in ("upper", "lower", "self"):
            if kind == "upper":
                sel = sel_shape & (rows < cols)
            elif kind == "lower":
                sel = sel_shape & (rows > cols)
            else:
                sel = sel_shape & (rows == cols)
            ks = np.nonzero(sel)[0]
            for c0 in range(0, ks.size, chunk):
                kk = ks[c0:c0 + chunk]
                dst = gbase[kk][:, None] + ar[None, :]
                if kind == "upper":
                    src = seg[kk][:, None] + ar[None, :]
                elif kind == "lower":
                    src = seg[mirror[kk]][:, None] + transposed[None, :]
                else:
                    src = seg[kk][:, None] + _tri_index(sbi)[None, :]
                values[dst] = U[src] * w[kk][:, None]
    return values


# --------------------------------------------------------------------------
# geometries
# --------------------------------------------------------------------------

def random_cube(n_atoms: int, density: float, species, r_cut: float, decay: float,
                seed: int, name: str = "random_cube", box: float | None = None) -> Operator:
    """Atoms uniform in a periodic cube; block (i, j) present when the
    minimum-image distance is strictly below ``r_cut`` (self always present).

    ``species`` is a list of ``(block_size, count)``; counts are exact and are
    assigned to atoms by a seeded permutation.
    """
    rng = np.random.default_rng(seed)
    L = (n_atoms / density) ** (1.0 / 3.0) if box is None else float(box)
    if not r_cut <= L / 2:
        raise ValueError("r_cut must be below half the box for unique minimum images")
    pos = rng.uniform(0.0, L, size=(n_atoms, 3))
    bvals = np.array([s[0] for s in species], dtype=np.int32)
    counts = [int(s[1]) for s in species]
    if sum(counts) != n_atoms:
        raise ValueError("species counts must sum to n_atoms")
    spec = rng.permutation(np.repeat(np.arange(len(species)), counts))
    b = bvals[spec].astype(np.int32)

    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(r_cut, output_type="ndarray")
    pairs = pairs.reshape(-1, 2).astype(np.int64)
    d = pos[pairs[:, 1]] - pos[pairs[:, 0]]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(axis=1))
    keep = r < r_cut
    pi, pj, r = pairs[keep, 0], pairs[keep, 1], r[keep]
    lo, hi = np.minimum(pi, pj), np.maximum(pi, pj)
    row_ptr, col_idx, dist = _graph_from_pairs(n_atoms, lo, hi, r)
    values = _symmetric_values(rng, b, row_ptr, col_idx, dist, decay)
    return Operator(name, b, row_ptr, col_idx, values, dist,
                    {"box": L, "r_cut": r_cut, "decay": decay, "seed": seed,
                     "_rng": rng, "pos": pos})


_SC_FIRST = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
_SC_SECOND = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]


def sc_lattice(m: int, bsize: int, seed: int, decay: float = 1.0,
               name: str = "sc_lattice") -> Operator:
    """Periodic ``m^3`` simple-cubic lattice (lattice constant 1), uniform
    block size; self + 6 first + 12 second neighbours (19 blocks per row).
    Atom index ``x + m*y + m*m*z``."""
    if m < 3:
        raise ValueError("m >= 3 keeps all 18 neighbours distinct")
    rng = np.random.default_rng(seed)
    idx = np.arange(m ** 3, dtype=np.int64)
    x, y, z = idx % m, (idx // m) % m, idx // (m * m)
    pi, pj, pd = [], [], []
    for offs, r in ((_SC_FIRST, 1.0), (_SC_SECOND, np.sqrt(2.0))):
        for dx, dy, dz in offs:
            j = (x + dx) % m + m * ((y + dy) % m) + m * m * ((z + dz) % m)
            pi.append(np.minimum(idx, j))
            pj.append(np.maximum(idx, j))
            pd.append(np.full(idx.shape, r))
    pi, pj, pd = np.concatenate(pi), np.concatenate(pj), np.concatenate(pd)
    b = np.full(m ** 3, bsize, dtype=np.int32)
    row_ptr, col_idx, dist = _graph_from_pairs(m ** 3, pi, pj, pd)
    values = _symmetric_values(rng, b, row_ptr, col_idx, dist, decay)
    return Operator(name, b, row_ptr, col_idx, values, dist,
                    {"m": m, "decay": decay, "seed": seed, "_rng": rng})


# zincblende nearest-neighbour directions in units of a/4 (cation -> anion)
_ZB_NN = np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)], dtype=np.int64)
_FCC = np.array([(0, 0, 0), (0, 2, 2), (2, 0, 2), (2, 2, 0)], dtype=np.int64)


def zincblende_sphere(radius: float, a: float, b_cat: int, b_an: int, r_cut: float,
                      seed: int, b_h: int = 1, h_bond: float = 1.5, decay: float = 1.0,
                      name: str = "zincblende_sphere") -> Operator:
    """Binary zincblende cluster inside a sphere centred on a cation.

    Cations on fcc sites, anions displaced by ``(a/4)(1,1,1)``; every atom with
    ``|r| <= radius`` is kept.  Cation/anion pairs couple when closer than
    ``r_cut``.  Each missing nearest-neighbour bond gets one passivating atom
    of block size ``b_h`` placed ``h_bond`` along the bond; it couples only to
    its host and itself.  Atoms are ordered by lattice position (z, y, x) and
    each passivating atom follows its host.
    """
    rng = np.random.default_rng(seed)
    u = a / 4.0                      # integer coordinates are in units of a/4
    M = int(np.ceil(radius / a)) + 2
    cells = np.stack(np.meshgrid(*[np.arange(-M, M + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    cat = (cells[:, None, :] * 4 + _FCC[None, :, :]).reshape(-1, 3)
    an = cat + 1
    lim = (radius / u) ** 2

    def inside(c):
        return (c * c).sum(axis=-1) <= lim

    cat = cat[inside(cat)]
    an = an[inside(an)]
    coords = np.concatenate([cat, an])
    kind = np.concatenate([np.zeros(len(cat), np.int8), np.ones(len(an), np.int8)])
    order = np.lexsort((coords[:, 0], coords[:, 1], coords[:, 2]))
    coords, kind = coords[order], kind[order]
    nh = len(coords)

    # missing bonds -> passivating atoms
    sign = np.where(kind == 0, 1, -1)[:, None, None]
    nbr = coords[:, None, :] + sign * _ZB_NN[None, :, :]          # (nh, 4, 3)
    missing = ~inside(nbr)
    host_of_h = np.repeat(np.arange(nh), 4).reshape(nh, 4)[missing]
    dirs = (sign * _ZB_NN[None, :, :])[missing].astype(np.float64)
    h_pos = coords[host_of_h] * u + h_bond * dirs / np.sqrt(3.0)

    # final order: every host followed by its passivating atoms
    n_h = host_of_h.size
    n = nh + n_h
    h_count = np.bincount(host_of_h, minlength=nh)
    new_host = np.arange(nh) + np.concatenate([[0], np.cumsum(h_count)[:-1]])
    # within a host, passivating atoms keep their bond order
    rank_in_host = np.arange(n_h) - np.concatenate([[0], np.cumsum(h_count)[:-1]])[host_of_h]
    new_h = new_host[host_of_h] + 1 + rank_in_host
    pos = np.empty((n, 3))
    pos[new_host] = coords * u
    pos[new_h] = h_pos
    b = np.empty(n, dtype=np.int32)
    b[new_host] = np.where(kind == 0, b_cat, b_an)
    b[new_h] = b_h

    tree = cKDTree(coords * u)
    pairs = tree.query_pairs(r_cut, output_type="ndarray").reshape(-1, 2).astype(np.int64)
    r = np.linalg.norm((coords[pairs[:, 1]] - coords[pairs[:, 0]]) * u, axis=1)
    keep = r < r_cut
    pairs, r = pairs[keep], r[keep]
    hi_ = np.concatenate([new_host[pairs[:, 0]], new_host[host_of_h]])
    hj_ = np.concatenate([new_host[pairs[:, 1]], new_h])
    hr = np.concatenate([r, np.full(n_h, h_bond)])
    lo, hi = np.minimum(hi_, hj_), np.maximum(hi_, hj_)
    row_ptr, col_idx, dist = _graph_from_pairs(n, lo, hi, hr)
    values = _symmetric_values(rng, b, row_ptr, col_idx, dist, decay)
    return Operator(name, b, row_ptr, col_idx, values, dist,
                    {"radius": radius, "a": a, "r_cut": r_cut, "n_cation": int((kind == 0).sum()),
                     "n_anion": int((kind == 1).sum()), "n_passivating": int(n_h),
                     "decay": decay, "seed": seed, "_rng": rng})


def random_pattern(seed: int, n: int, bset=(1, 2, 3, 4, 9, 13), density: float = 0.2,
                   empty_rows: int = 0, unsorted: bool = False, symmetric: bool = False,
                   with_self: bool = True, name: str = "random_pattern") -> Operator:
    """Non-geometric random block pattern for edge cases.

    ``empty_rows`` rows are left without blocks (self blocks removed too);
    ``unsorted`` shuffles the column order inside every row; values are
    ``U[-1, 1]`` (symmetric when requested).
    """
    rng = np.random.default_rng(seed)
    b = rng.choice(np.asarray(bset, dtype=np.int32), size=n).astype(np.int32)
    mask = rng.random((n, n)) < density
    if symmetric:
        mask = np.triu(mask) | np.triu(mask, 1).T
    if with_self:
        np.fill_diagonal(mask, True)
    if empty_rows:
        er = rng.choice(n, size=min(empty_rows, n), replace=False)
        mask[er, :] = False
        if symmetric:
            mask[:, er] = False
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    col_idx = cols.astype(np.int32)
    dist = np.zeros(col_idx.shape[0])
    if symmetric:
        values = _symmetric_values(rng, b, row_ptr, col_idx, dist, decay=1.0)
    else:
        sizes = b[rows].astype(np.int64) * b[cols].astype(np.int64)
        values = rng.uniform(-1.0, 1.0, size=int(sizes.sum()))
    op = Operator(name, b, row_ptr, col_idx, values, dist, {"seed": seed, "_rng": rng})
    if unsorted:
        op = shuffle_columns(op, rng)
    return op


def shuffle_columns(op: Operator, rng) -> Operator:
    """Permute the block order inside every row (values move with their blocks)."""
    base = op.block_base
    perm_blocks = np.empty(op.nnzb, dtype=np.int64)
    for i in range(op.n):
        s, e = int(op.row_ptr[i]), int(op.row_ptr[i + 1])
        perm_blocks[s:e] = s + rng.permutation(e - s)
    new_vals = np.concatenate([op.values[base[k]:base[k + 1]] for k in perm_blocks]) \
        if op.nnzb else op.values.copy()
    return Operator(op.name, op.b, op.row_ptr, op.col_idx[perm_blocks].copy(), new_vals,
                    op.dist[perm_blocks].copy(), op.meta)


def multivector(op: Operator, nrhs: int, rng=None, seed: int | None = None) -> np.ndarray:
    """Row-major ``N x nrhs`` FP64 multi-vector with N(0, 1) entries, drawn
    from the operator's own stream (after its values) unless a seed is given."""
    if rng is None:
        rng = op.meta["_rng"] if seed is None else np.random.default_rng(seed)
    return rng.standard_normal((op.N, nrhs))


def inf_norm_scale(op: Operator, margin: float = 1.01) -> float:
    """``margin * max_r sum_c |a_rc|``: a Gershgorin bound used to map the
    spectrum into [-1, 1] before a Chebyshev expansion (input preparation)."""
    rows = op.block_rows
    bi = op.b[rows].astype(np.int64)
    bj = op.b[op.col_idx].astype(np.int64)
    base = op.block_base
    off = op.off
    rowsum = np.zeros(op.N)
    for sbi, sbj in np.unique(np.stack([bi, bj], 1), axis=0):
        ks = np.nonzero((bi == sbi) & (bj == sbj))[0]
        blk = np.abs(op.values[base[ks][:, None] + np.arange(sbi * sbj)[None, :]])
        rs = blk.reshape(-1, sbi, sbj).sum(axis=2)                    # (count, bi)
        np.add.at(rowsum, (off[rows[ks]][:, None] + np.arange(sbi)[None, :]).ravel(), rs.ravel())
    return float(margin * rowsum.max())


def scaled(op: Operator, s: float, name: str | None = None) -> Operator:
    """The same pattern with every value divided by ``s``."""
    return Operator(name or op.name, op.b, op.row_ptr, op.col_idx, op.values / s, op.dist,
                    dict(op.meta, scale=s))
