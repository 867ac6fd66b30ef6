"""C-ABI behaviour that needs no GPU: exports, validation, planner maps.

Validation happens on the host before any HIP call, so every error status
below is produced here on a machine without a device.
"""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2609_04397_amd import _lib
from workloads import random_pattern, sc_lattice, make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vbcsr.h")


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vbcsr_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (vbcsr_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    assert set(names) == set(_lib.SIGNATURES), "ctypes table and header disagree"


def _plan(lib, b, rp, ci, nval, fwd=None, tr=None, max_shapes=256, order="atom"):
    b = np.ascontiguousarray(b, np.int32)
    rp = np.ascontiguousarray(rp, np.int64)
    ci = np.ascontiguousarray(ci, np.int32)
    ns = ctypes.c_int32()
    shapes = np.zeros(3 * max_shapes, np.int32)
    pv = ctypes.c_int64()
    rc = lib.vbcsr_plan_host(b.size, b.ctypes.data, rp.ctypes.data, ci.ctypes.data if ci.size else None,
                             nval, ctypes.byref(ns), shapes.ctypes.data, max_shapes,
                             fwd.ctypes.data if fwd is not None else None,
                             tr.ctypes.data if tr is not None else None, ctypes.byref(pv),
                             ctypes.byref(_lib.PlanOpts(0, 0, 0, _lib.ORDER[order])))
    return rc, ns.value, shapes[:3 * ns.value].reshape(-1, 3), pv.value


def test_planner_shape_classes_match_recount(lib):
    op = random_pattern(3, 60, bset=(1, 4, 9, 13), density=0.15, empty_rows=4, unsorted=True)
    rc, ns, shapes, pv = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz)
    assert rc == 0
    bi = op.b[op.block_rows]
    bj = op.b[op.col_idx]
    u, c = np.unique(np.stack([bi, bj], 1), axis=0, return_counts=True)
    assert np.array_equal(shapes[:, :2], u) and np.array_equal(shapes[:, 2], c)
    # every panel padded to a multiple of 4 values
    assert op.nnz <= pv < op.nnz + 4 * op.n


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_page_maps_are_bijections(lib, seed):
    op = random_pattern(seed, 50, bset=(1, 2, 5, 9, 13), density=0.2, empty_rows=3, unsorted=True)
    fwd = np.zeros(op.nnzb, np.int64)
    tr = np.zeros(op.nnzb, np.int64)
    rc, _, _, pv = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz, fwd, tr)
    assert rc == 0
    sizes = op.block_sizes
    for pos in (fwd, tr):
        order = np.argsort(pos)
        starts = pos[order]
        ends = starts + sizes[order]
        assert starts[0] == 0
        if pos is fwd:  # page_values counts the forward pages
            assert ends[-1] <= pv < ends[-1] + 4
        gaps = starts[1:] - ends[:-1]
        # blocks tile the pages except for < 4 values of padding after a
        # panel, so that every panel starts on a multiple of 4
        assert np.all((gaps >= 0) & (gaps < 4))
        assert np.all(starts[1:][gaps > 0] % 4 == 0)


def test_forward_pages_group_rows_and_shapes(lib):
    """Within the forward pages, the blocks of one block row are contiguous and
    ordered by (b_j, j); rows follow atom order."""
    op = random_pattern(11, 40, bset=(1, 4, 9), density=0.3, unsorted=True)
    fwd = np.zeros(op.nnzb, np.int64)
    rc, *_ = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz, fwd)
    assert rc == 0
    rows = op.block_rows
    key = np.lexsort((op.col_idx, op.b[op.col_idx], rows))
    assert np.all(np.diff(fwd[key]) > 0)


def test_transposed_pages_group_columns(lib):
    op = random_pattern(12, 40, bset=(1, 4, 9), density=0.3, unsorted=True)
    tr = np.zeros(op.nnzb, np.int64)
    rc, *_ = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz, None, tr)
    assert rc == 0
    rows = op.block_rows
    key = np.lexsort((rows, op.b[rows], op.col_idx))
    assert np.all(np.diff(tr[key]) > 0)


def test_uniform_lattice_single_shape(lib):
    op = sc_lattice(4, 13, seed=2)
    rc, ns, shapes, _ = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz)
    assert rc == 0 and ns == 1 and tuple(shapes[0]) == (13, 13, 19 * 64)


def _case(lib, b, rp, ci, nval):
    rc, *_ = _plan(lib, b, rp, ci, nval)
    return rc


def test_validation_errors(lib):
    b = np.array([2, 1, 3], np.int32)
    rp = np.array([0, 2, 3, 5], np.int64)
    ci = np.array([0, 2, 1, 0, 2], np.int32)
    nval = 2 * 2 + 2 * 3 + 1 * 1 + 3 * 2 + 3 * 3
    assert _case(lib, b, rp, ci, nval) == _lib.VBCSR_OK
    assert _case(lib, b, rp, ci, nval + 1) == _lib.VBCSR_ESHAPE
    assert _case(lib, b, np.array([1, 2, 3, 5]), ci, nval) == _lib.VBCSR_EINVAL      # row_ptr[0] != 0
    assert _case(lib, b, np.array([0, 3, 2, 5]), ci, nval) == _lib.VBCSR_EINVAL      # decreasing
    assert _case(lib, b, rp, np.array([0, 3, 1, 0, 2]), nval) == _lib.VBCSR_EINVAL   # col out of range
    assert _case(lib, b, rp, np.array([0, -1, 1, 0, 2]), nval) == _lib.VBCSR_EINVAL
    assert _case(lib, b, rp, np.array([0, 0, 1, 0, 2]), 2 * 2 * 2 + 1 + 15) == _lib.VBCSR_EDUP
    assert _case(lib, np.array([2, 0, 3], np.int32), rp, ci, nval) == _lib.VBCSR_EINVAL
    assert _case(lib, np.array([2, 65, 3], np.int32), rp, ci, nval) == _lib.VBCSR_EUNSUPPORTED
    msg = lib.vbcsr_last_error().decode()
    assert "exceeds" in msg


def test_panel_size_limit(lib):
    """One block row (or block column) holding 2^28 values is refused: the
    kernels address a panel with 32-bit byte offsets."""
    n = 1 << 16
    b = np.full(n, 64, np.int32)
    nval = 64 * 64 * n
    # every block in row 0
    rp = np.full(n + 1, n, np.int64)
    rp[0] = 0
    ci = np.arange(n, dtype=np.int32)
    assert _case(lib, b, rp, ci, nval) == _lib.VBCSR_EUNSUPPORTED
    assert "block row 0" in lib.vbcsr_last_error().decode()
    # every block in column 0
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.zeros(n, np.int32)
    assert _case(lib, b, rp, ci, nval) == _lib.VBCSR_EUNSUPPORTED
    assert "block column 0" in lib.vbcsr_last_error().decode()
    # one block fewer in the row is accepted by the validation
    b2 = b.copy()
    b2[-1] = 63
    rp = np.full(n + 1, n, np.int64)
    rp[0] = 0
    ci = np.arange(n, dtype=np.int32)
    rc = _case(lib, b2, rp, ci, 64 * 64 * (n - 1) + 64 * 63)
    assert rc == _lib.VBCSR_OK


def _processing_positions(op, fwd):
    """Processing position of every atom (rank of its panel's start)."""
    start = np.full(op.n, np.iinfo(np.int64).max)
    np.minimum.at(start, op.block_rows, fwd)
    pos = np.empty(op.n, np.int64)
    pos[np.argsort(start, kind="stable")] = np.arange(op.n)
    return pos


def test_row_order_rcm_cluster_and_auto(lib):
    """RCM is a permutation that shortens the processing distance of coupled
    atoms of a randomly ordered structure; the clustered order is a
    permutation whose clusters of 256 consecutive atoms are connected; AUTO
    is the clustered order; every order keeps each row's blocks contiguous."""
    from workloads.core import random_cube
    op = random_cube(3000, 0.05, [(1, 600), (4, 1200), (9, 1200)], r_cut=5.0, decay=2.0, seed=7)
    dist, pos_of = {}, {}
    for order in ("atom", "rcm", "cluster", "auto"):
        fwd = np.zeros(op.nnzb, np.int64)
        tr = np.zeros(op.nnzb, np.int64)
        rc, _, _, pv = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz, fwd, tr, order=order)
        assert rc == 0
        pos = _processing_positions(op, fwd)
        assert np.array_equal(np.sort(pos), np.arange(op.n))
        pos_of[order] = pos
        dist[order] = np.abs(pos[op.block_rows] - pos[op.col_idx]).mean()
        # blocks of one row stay contiguous and ordered by (b_j, j) in any order
        key = np.lexsort((op.col_idx, op.b[op.col_idx], pos[op.block_rows]))
        assert np.all(np.diff(fwd[key]) > 0)
    assert dist["rcm"] <= 0.5 * dist["atom"]
    assert np.array_equal(pos_of["auto"], pos_of["cluster"])
    assert np.array_equal(_cluster_reference(op.n, op.row_ptr, op.col_idx, 256),
                          np.argsort(pos_of["cluster"]))


def _cluster_reference(n, rp, ci, S):
    """The clustered order from its definition: clusters of up to S atoms
    (listed ascending), each grown breadth-first over untaken atoms (neighbours: the row's
    columns in stored order, then the column's rows ascending), seeded at the
    first queued but untaken atom of the previous cluster, else at the
    lowest untaken atom."""
    rows = np.repeat(np.arange(n), np.diff(rp))
    col_rows = [[] for _ in range(n)]
    for i, j in zip(rows, ci):
        col_rows[j].append(i)
    taken = np.zeros(n, bool)
    order, seed = [], None
    while len(order) < n:
        if seed is None or taken[seed]:
            seed = int(np.argmin(taken))
        cluster, queue, queued = [], [seed], {seed}
        head = 0
        while head < len(queue) and len(cluster) < S:
            v = queue[head]
            head += 1
            cluster.append(v)
            if len(cluster) == S:
                break
            for u in list(ci[rp[v]:rp[v + 1]]) + col_rows[v]:
                if not taken[u] and u not in queued and u not in cluster:
                    queued.add(u)
                    queue.append(u)
        for v in cluster:
            taken[v] = True
        order += sorted(cluster)
        rest = [u for u in queue[head:] if not taken[u]]
        seed = rest[0] if rest else None
    return np.array(order)


def test_row_order_rejects_unknown(lib):
    op = random_pattern(3, 10, bset=(2, 3), density=0.3)
    ns = ctypes.c_int32()
    shapes = np.zeros(3 * 16, np.int32)
    pv = ctypes.c_int64()
    rc = lib.vbcsr_plan_host(op.n, op.b.ctypes.data, op.row_ptr.ctypes.data, op.col_idx.ctypes.data,
                             op.nnz, ctypes.byref(ns), shapes.ctypes.data, 16, None, None,
                             ctypes.byref(pv), ctypes.byref(_lib.PlanOpts(0, 0, 0, 7)))
    assert rc == _lib.VBCSR_EINVAL


def test_empty_graph_is_valid(lib):
    rc, ns, _, pv = _plan(lib, np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32), 0)
    assert rc == 0 and ns == 0 and pv == 0
    rc, ns, _, pv = _plan(lib, np.array([3, 4], np.int32), np.zeros(3, np.int64), np.zeros(0, np.int32), 0)
    assert rc == 0 and ns == 0 and pv == 0


def test_null_handle_and_bad_arguments(lib):
    assert lib.vbcsr_spmm(None, None, 1, None, 1, 1, 1.0, 0.0, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_spmm_t(None, None, 1, None, 1, 1, 1.0, 0.0, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_sddmm(None, None, 1, None, 1, 1, None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_set_values(None, None, 0, 0, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_info(None, None, None, None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_get_structure(None, None, None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_get_values(None, None, 0, None) == _lib.VBCSR_EINVAL
    out = ctypes.c_void_p(1)
    assert lib.vbcsr_spgemm(ctypes.byref(out), None, None, 0.0, None, None, None) == _lib.VBCSR_EINVAL
    assert out.value is None
    assert lib.vbcsr_spgemm(None, None, None, 0.0, None, None, None) == _lib.VBCSR_EINVAL
    # page-layout calls
    n = ctypes.c_int64(-1)
    assert lib.vbcsr_page_size(None, ctypes.byref(n)) == _lib.VBCSR_EINVAL and n.value == -1
    assert lib.vbcsr_get_pages(None, None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_use_pages(None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_refresh_transposed(None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_sddmm_pages(None, None, 1, None, 1, 1, None, None) == _lib.VBCSR_EINVAL
    lib.vbcsr_destroy(None)
    h = ctypes.c_void_p()
    b = np.array([1], np.int32)
    rp = np.array([0, 1], np.int64)
    ci = np.array([0], np.int32)
    assert lib.vbcsr_create(None, 1, b.ctypes.data, rp.ctypes.data, ci.ctypes.data, None, 1, 0,
                            None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_create(ctypes.byref(h), 1, b.ctypes.data, rp.ctypes.data, ci.ctypes.data,
                            None, 1, 7, None, None) == _lib.VBCSR_EINVAL
    opts = _lib.PlanOpts(3, 0, 0)
    assert lib.vbcsr_create(ctypes.byref(h), 1, b.ctypes.data, rp.ctypes.data, ci.ctypes.data,
                            None, 1, 0, ctypes.byref(opts), None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_create(ctypes.byref(h), 1, b.ctypes.data, rp.ctypes.data, ci.ctypes.data,
                            None, 2, 0, None, None) == _lib.VBCSR_ESHAPE
    assert h.value is None


def test_injected_allocation_failure_reports_enomem():
    """VBCSR_FAIL_ALLOC_AFTER=0 fails the first device allocation before any
    HIP call, so the out-of-memory path is exercised without a device."""
    code = r"""
import ctypes, numpy as np
from paper_2609_04397_amd import _lib
lib = _lib.load()
b = np.array([2, 3], np.int32); rp = np.array([0, 2, 3], np.int64); ci = np.array([0, 1, 1], np.int32)
h = ctypes.c_void_p()
rc = lib.vbcsr_create(ctypes.byref(h), 2, b.ctypes.data, rp.ctypes.data, ci.ctypes.data, None,
                      4 + 6 + 9, 0, None, None)
print(rc, h.value, lib.vbcsr_last_error().decode())
"""
    env = dict(os.environ, VBCSR_FAIL_ALLOC_AFTER="0")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    rc, hv, msg = out.stdout.split(" ", 2)
    assert int(rc) == _lib.VBCSR_ENOMEM and hv == "None" and "injected" in msg


def test_c3_shape_classes_full_size_small():
    """The zincblende stand-in has the nine (b_i, b_j) classes of cation (13),
    anion (9) and passivating (1) atoms."""
    op, _ = make_config("C3", scale=0.003, nrhs=1)
    lib = _lib.load()
    rc, ns, shapes, _ = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz)
    assert rc == 0 and ns == 9
    assert {(int(a), int(c)) for a, c, _ in shapes} == {(x, y) for x in (1, 9, 13) for y in (1, 9, 13)}


def test_large_graph_threaded_planner(lib):
    """A graph above the planner's threading threshold (12,000 atoms): page
    maps tile the pages, rows are grouped by (b_j, j), columns by (b_i, i),
    shape classes recount, and of two bad rows the first one is reported."""
    from workloads.configs import make_operator
    op = make_operator("C5", 0.12)
    assert op.n >= 8192
    fwd = np.zeros(op.nnzb, np.int64)
    tr = np.zeros(op.nnzb, np.int64)
    for order in ("atom", "rcm"):
        rc, ns, shapes, pv = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz, fwd, tr, order=order)
        assert rc == 0
        sizes = op.block_sizes
        for pos in (fwd, tr):
            o = np.argsort(pos)
            gaps = pos[o][1:] - (pos[o] + sizes[o])[:-1]
            assert pos[o][0] == 0 and np.all((gaps >= 0) & (gaps < 4))
    rows = op.block_rows
    key = np.lexsort((op.col_idx, op.b[op.col_idx], rows))
    rc, *_ = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz, fwd, tr, order="atom")
    assert np.all(np.diff(fwd[key]) > 0)
    keyt = np.lexsort((rows, op.b[rows], op.col_idx))
    assert np.all(np.diff(tr[keyt]) > 0)
    u, c = np.unique(np.stack([op.b[rows], op.b[op.col_idx]], 1), axis=0, return_counts=True)
    rc, ns, shapes, pv = _plan(lib, op.b, op.row_ptr, op.col_idx, op.nnz)
    assert np.array_equal(shapes[:, :2], u) and np.array_equal(shapes[:, 2], c)
    # two bad rows far apart: a duplicate in a late row, an out-of-range
    # column in an earlier one; the earlier row is reported
    ci = op.col_idx.copy()
    late, early = op.n - 5, 7000
    s_late = int(op.row_ptr[late])
    ci[s_late + 1] = ci[s_late]
    rc = _case(lib, op.b, op.row_ptr, ci, op.nnz)
    assert rc == _lib.VBCSR_EDUP
    assert "duplicate block (%d," % late in lib.vbcsr_last_error().decode()
    ci[int(op.row_ptr[early])] = op.n + 3
    rc = _case(lib, op.b, op.row_ptr, ci, op.nnz)
    assert rc == _lib.VBCSR_EINVAL
    assert ("in row %d" % early) in lib.vbcsr_last_error().decode()


def _rcm_reference(n, rp, ci):
    """Reverse Cuthill-McKee written out from its definition: neighbours of
    an atom are the other atoms of its row's and its column's blocks (a pair
    present both ways counts twice, also in the degree), breadth-first search
    from the unvisited atom of least (degree, index), neighbours visited in
    (degree, index) order, the sequence reversed."""
    rows = np.repeat(np.arange(n), np.diff(rp))
    off = rows != ci
    deg = np.bincount(rows[off], minlength=n) + np.bincount(ci[off], minlength=n)
    nbr = [[] for _ in range(n)]
    for i, j in zip(rows[off].tolist(), ci[off].tolist()):
        nbr[i].append(j)
        nbr[j].append(i)
    for lst in nbr:
        lst.sort(key=lambda x: (deg[x], x))
    seen = np.zeros(n, bool)
    order = []
    for s0 in sorted(range(n), key=lambda x: (deg[x], x)):
        if seen[s0]:
            continue
        seen[s0] = True
        head = len(order)
        order.append(s0)
        while head < len(order):
            v = order[head]
            head += 1
            for u in nbr[v]:
                if not seen[u]:
                    seen[u] = True
                    order.append(u)
    return order[::-1]


def test_rcm_order_matches_definition(lib):
    """Above the threading threshold (9,000 atoms), on a non-symmetric graph
    with unsorted columns, empty rows and some diagonal blocks: the panels of
    the forward pages follow the reverse Cuthill-McKee order of the
    definition, and a rerun gives the same layout."""
    rng = np.random.default_rng(42)
    n = 9000
    cnt = rng.integers(0, 12, n)
    cnt[rng.choice(n, 40, replace=False)] = 0
    rows = []
    for i in range(n):
        c = rng.choice(n, cnt[i], replace=False) if cnt[i] else np.zeros(0, np.int64)
        if cnt[i] and rng.random() < 0.3 and i not in c:
            c[0] = i
        rows.append(rng.permutation(c))
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    ci = np.concatenate(rows).astype(np.int32)
    b = rng.choice([1, 4, 9, 13], n).astype(np.int32)
    nval = int(np.sum(b[np.repeat(np.arange(n), np.diff(rp))].astype(np.int64) * b[ci]))
    fwd = np.zeros(len(ci), np.int64)
    tr = np.zeros(len(ci), np.int64)
    rc, *_ = _plan(lib, b, rp, ci, nval, fwd, tr, order="rcm")
    assert rc == 0
    ref = _rcm_reference(n, rp, ci)
    # panel start of every non-empty row = its smallest forward offset
    blk_rows = np.repeat(np.arange(n), np.diff(rp))
    start = np.full(n, np.iinfo(np.int64).max)
    np.minimum.at(start, blk_rows, fwd)
    got = [i for i in np.argsort(start, kind="stable") if cnt[i] > 0]
    assert got == [i for i in ref if cnt[i] > 0]
    fwd2, tr2 = np.zeros_like(fwd), np.zeros_like(tr)
    _plan(lib, b, rp, ci, nval, fwd2, tr2, order="rcm")
    assert np.array_equal(fwd, fwd2) and np.array_equal(tr, tr2)


_OOM_CHILD = r"""
import ctypes, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2609_04397_amd import _lib
sys.path.insert(0, sys.argv[1] + "/tests")
from test_abi_host import _plan
lib = _lib.load()
rng = np.random.default_rng(0)
n, per = 20000, 60
rp = np.arange(0, n * per + 1, per, dtype=np.int64)
ci = np.concatenate([np.sort(rng.choice(n, per, replace=False)) for _ in range(n)]).astype(np.int32)
b = np.full(n, 4, np.int32)
nval = 16 * n * per
fwd = np.zeros(n * per, np.int64)
tr = np.zeros(n * per, np.int64)
def vm_bytes():
    for line in open("/proc/self/status"):
        if line.startswith("VmSize:"):
            return int(line.split()[1]) * 1024
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
if hard != resource.RLIM_INFINITY:
    print("skip")
    sys.exit(0)
resource.setrlimit(resource.RLIMIT_AS, (vm_bytes() + (32 << 20), hard))
rc, *_ = _plan(lib, b, rp, ci, nval, fwd, tr, order="rcm")
msg = lib.vbcsr_last_error().decode()
resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
rc2, *_ = _plan(lib, b, rp, ci, nval, fwd, tr, order="rcm")
print(rc, rc2, msg)
"""


def test_host_allocation_failure_is_a_status(lib):
    """With the address space capped just above what the process holds, the
    threaded planner cannot allocate its tables: the entry point returns
    VBCSR_ENOMEM with a message naming it (no exception crosses the C ABI),
    and succeeds again once the cap is lifted."""
    r = subprocess.run([sys.executable, "-c", _OOM_CHILD, ROOT], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    if r.stdout.strip() == "skip":
        pytest.skip("the address-space limit of this process cannot be raised back")
    rc, rc2, msg = r.stdout.strip().split(" ", 2)
    assert int(rc) == _lib.VBCSR_ENOMEM and "vbcsr_plan_host" in msg, r.stdout
    assert int(rc2) == 0


_LOG_CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
from paper_2609_04397_amd import _lib
from test_abi_host import _plan
from workloads import make_config
op, _ = make_config("C5", scale=0.05, nrhs=1)
rc, ns, shapes, pv = _plan(_lib.load(), op.b, op.row_ptr, op.col_idx, op.nnz, order="cluster")
print(rc, ns, int(pv))
"""


def test_planner_log_statistics():
    """VBCSR_LOG prints the planner's statistics on stderr: sizes, the shape
    classes with their counts, the layout's padding and the balance of the
    panels; without it the planner prints nothing."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, VBCSR_LOG="1")
    r = subprocess.run([sys.executable, "-c", _LOG_CHILD, root], capture_output=True, text=True,
                       env=env, timeout=120)
    assert r.returncode == 0, r.stderr
    rc, ns, pv = map(int, r.stdout.split())
    assert rc == 0 and ns == 9
    lines = [l for l in r.stderr.splitlines() if l.startswith("vbcsr plan:")]
    assert len(lines) == 4
    assert "5000 atoms" in lines[0] and "order clustered" in lines[0]
    classes = lines[1].split(":", 2)[2].split()
    assert len(classes) == 9 and sum(int(c.split(":")[1]) for c in classes[1:]) > 0
    assert "pages %d values" % pv in lines[2]
    env.pop("VBCSR_LOG")
    r = subprocess.run([sys.executable, "-c", _LOG_CHILD, root], capture_output=True, text=True,
                       env=env, timeout=120)
    assert r.returncode == 0 and "vbcsr plan" not in r.stderr
