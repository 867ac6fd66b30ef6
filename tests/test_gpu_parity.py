"""Parity of the HIP products with the FP64 CPU oracle (through the C ABI).

Small inputs span several panels, every block size class the kernels
distinguish (b = 1, sizes below and above 16, up to 64), empty rows,
unsorted column order and ragged right-hand-side tiles.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, check, rounded, TOL, DT
from metrics import rel_f, comp
from workloads import random_pattern, make_config, sc_lattice

pytestmark = pytest.mark.gpu


from paper_2609_04397_amd.matrix import Matrix


PATTERNS = {
    "mixed": dict(seed=1, n=40, bset=(1, 4, 9, 13), density=0.2, empty_rows=3, unsorted=True),
    "wide": dict(seed=2, n=24, bset=(2, 5, 16, 17, 20, 33), density=0.3, empty_rows=1),
    "big": dict(seed=3, n=10, bset=(64, 31, 48), density=0.5),
    "scalar": dict(seed=4, n=300, bset=(1,), density=0.03, empty_rows=10, unsorted=True),
    # blocks of exactly 16 columns (the widest that leave the block-sampled
    # product's output window whole) next to 7-wide ones
    "sixteen": dict(seed=6, n=36, bset=(7, 16), density=0.3, empty_rows=2, unsorted=True),
}


@pytest.fixture(scope="module", params=sorted(PATTERNS))
def pattern(request):
    return request.param, random_pattern(**PATTERNS[request.param])


@pytest.mark.parametrize("path,nrhs", [("vec", 1), ("vec", 2), ("vec", 3), ("vec", 8), ("vec", 11),
                                       ("mfma", 1), ("mfma", 16), ("mfma", 33), ("mfma", 64),
                                       ("mfma", 100), ("mfma", 128)])
def test_fp64_forward_and_transpose(pattern, path, nrhs):
    name, op = pattern
    print("case", name, path, nrhs, flush=True)
    A = Matrix.from_operator(op, prec="fp64", path=path)
    rng = np.random.default_rng(nrhs)
    X = rng.standard_normal((op.N, nrhs))
    Y0 = rng.standard_normal((op.N, nrhs))
    for transpose in (False, True):
        ref = (oracle.spmm_t if transpose else oracle.spmm)(op, X, alpha=1.5, beta=-0.5, Y=Y0)
        Yd = dev(Y0, "fp64")
        A.spmm(dev(X, "fp64"), Yd, alpha=1.5, beta=-0.5, transpose=transpose)
        scale = 1.5 * oracle.abs_product(op, X, transpose_op=transpose) + 0.5 * np.abs(Y0)
        check(host(Yd), ref, "fp64", scale, "%s %s nrhs=%d T=%s" % (name, path, nrhs, transpose))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("nrhs", [1, 8, 16, 32, 40, 64, 100, 128])
def test_reduced_precision_forward(pattern, prec, nrhs):
    name, op = pattern
    print("case", name, prec, nrhs, flush=True)
    A = Matrix.from_operator(op, prec=prec)
    X = np.random.default_rng(5).standard_normal((op.N, nrhs))
    Xr = rounded(X, prec)
    for transpose in (False, True):
        ref = (oracle.spmm_t if transpose else oracle.spmm)(op, Xr)
        got = host(A.spmm(dev(X, prec), transpose=transpose))
        check(got, ref, prec, label="%s %s nrhs=%d T=%s" % (name, prec, nrhs, transpose))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nrhs", [1, 7, 32, 64, 100])
def test_sddmm(pattern, prec, nrhs):
    name, op = pattern
    print("case sddmm", name, prec, nrhs, flush=True)
    A = Matrix.from_operator(op, prec=prec)
    rng = np.random.default_rng(9)
    dY = rounded(rng.standard_normal((op.N, nrhs)), prec)
    X = rounded(rng.standard_normal((op.N, nrhs)), prec)
    ref = oracle.sddmm(op, dY, X)
    got = host(A.sddmm(dev(dY, prec), dev(X, prec)))
    scale = oracle.sddmm(op, np.abs(dY), np.abs(X))
    check(got, ref, prec, scale if prec == "fp64" else None, "sddmm %s %s" % (name, prec))


def test_beta_zero_ignores_nan_and_empty_rows():
    op = random_pattern(7, 30, bset=(3, 9), density=0.2, empty_rows=6)
    A = Matrix.from_operator(op)
    X = np.random.default_rng(1).standard_normal((op.N, 4))
    for path in ("vec", "mfma"):
        A2 = Matrix.from_operator(op, path=path)
        Y = torch.full((op.N, 4), float("nan"), dtype=torch.float64, device="cuda")
        A2.spmm(dev(X, "fp64"), Y, beta=0.0)
        y = host(Y)
        assert np.all(np.isfinite(y))
        check(y, oracle.spmm(op, X), "fp64", oracle.abs_product(op, X))
    # empty rows: Y_i = beta * Y_i
    Y0 = np.random.default_rng(2).standard_normal((op.N, 4))
    Yd = dev(Y0, "fp64")
    A.spmm(dev(X, "fp64"), Yd, alpha=0.0, beta=2.0)
    assert np.array_equal(host(Yd), 2.0 * Y0)


def test_strided_vectors():
    op = random_pattern(8, 25, bset=(4, 9), density=0.25)
    A = Matrix.from_operator(op)
    Xbig = np.random.default_rng(3).standard_normal((op.N, 10))
    Xd = dev(Xbig, "fp64")[:, 2:7]          # ld = 10, nrhs = 5
    Yd = torch.zeros((op.N, 12), dtype=torch.float64, device="cuda")
    Yv = Yd[:, 1:6]
    from paper_2609_04397_amd import _lib
    import ctypes
    lib = _lib.load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.vbcsr_spmm(A._h, ctypes.c_void_p(Xd.data_ptr()), 10, ctypes.c_void_p(Yv.data_ptr()),
                              12, 5, 1.0, 0.0, s))
    y = host(Yd)
    check(y[:, 1:6], oracle.spmm(op, Xbig[:, 2:7]), "fp64", oracle.abs_product(op, Xbig[:, 2:7]))
    assert np.all(y[:, :1] == 0) and np.all(y[:, 6:] == 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_x_rows_beyond_2gib(prec):
    """X whose rows span more than 2^31 bytes (large leading dimension): the
    matrix-core kernels then read it through 64-bit pointers instead of one
    buffer descriptor; the vector kernel always does."""
    op = random_pattern(15, 60, bset=(4, 9, 13), density=0.2, empty_rows=1)
    s = 8 if prec == "fp64" else 4
    ld = ((1 << 31) // (s * op.N) + 64) // 4 * 4
    assert op.N * ld * s > (1 << 31)
    print("case big-ld", prec, op.N, ld, flush=True)
    X = np.random.default_rng(5).standard_normal((op.N, 40))
    big = torch.zeros((op.N, ld), dtype=DT[prec], device="cuda")
    big[:, :40] = dev(X, prec)
    for path, nrhs in (("mfma", 32), ("mfma", 40), ("vec", 3)):
        A = Matrix.from_operator(op, prec=prec, path=path)
        Xr = rounded(X[:, :nrhs], prec)
        for transpose in (False, True):
            ref = (oracle.spmm_t if transpose else oracle.spmm)(op, Xr)
            got = host(A.spmm(big[:, :nrhs], transpose=transpose))
            scale = oracle.abs_product(op, Xr, transpose_op=transpose) if prec == "fp64" else None
            check(got, ref, prec, scale, "big ld %s %s nrhs=%d T=%s" % (prec, path, nrhs, transpose))
        A.close()
    del big
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,path,nrhs", [("fp64", "vec", 1), ("fp64", "vec", 2), ("fp64", "vec", 4),
                                            ("fp64", "vec", 8), ("fp32", "vec", 1), ("fp32", "vec", 2),
                                            ("fp64", "mfma", 16), ("fp32", "mfma", 32),
                                            ("bf16x3", "auto", 64)])
def test_nonfinite_values_stay_in_their_rows(prec, path, nrhs):
    """Inf in the blocks of a few block rows reaches exactly the outputs those
    blocks feed; neighbouring panels (odd lengths, so their last value loads
    end next to an Inf panel) stay finite and match the oracle."""
    op = random_pattern(21, 30, bset=(1, 3, 5, 13), density=0.25, empty_rows=2)
    bad = np.array([3, 10, 17])
    rows = op.block_rows
    vmask = np.repeat(np.isin(rows, bad), np.diff(op.block_base))
    vals = op.values.copy()
    vals[vmask] = np.inf
    clean = op.values.copy()
    clean[vmask] = 0.0
    from workloads.core import Operator
    op0 = Operator(op.name, op.b, op.row_ptr, op.col_idx, clean, op.dist)
    A = Matrix.from_operator(op, prec=prec, values=vals, path=path)
    X = np.random.default_rng(9).standard_normal((op.N, nrhs))
    Xr = rounded(X, prec)
    off = op.off
    fwd_bad = np.isin(np.arange(op.n), bad)
    adj_bad = np.zeros(op.n, bool)
    adj_bad[op.col_idx[np.isin(rows, bad)]] = True
    for transpose, atom_bad in ((False, fwd_bad), (True, adj_bad)):
        print("case nonfinite", prec, path, nrhs, transpose, flush=True)
        got = host(A.spmm(dev(X, prec), transpose=transpose))
        good = np.repeat(~atom_bad, np.diff(off))
        ref = (oracle.spmm_t if transpose else oracle.spmm)(op0, Xr)
        assert np.all(np.isfinite(got[good]))
        # an output fed by an Inf block is not finite
        fed = np.repeat(atom_bad & (np.bincount(rows if not transpose else op.col_idx,
                                                minlength=op.n) > 0), np.diff(off))
        assert not np.isfinite(got[fed]).any()
        check(got[good], ref[good], prec, label="nonfinite %s %s %d T=%s" % (prec, path, nrhs, transpose))
    A.close()


@pytest.mark.parametrize("order", ["rcm", "cluster"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_row_order_does_not_change_results(prec, order):
    """Processing the panels in RCM or clustered order instead of atom order
    leaves every product bit for bit the same (one wave still sums each
    output row in the same panel order) and matches the oracle; moments agree
    to rounding."""
    op = random_pattern(5, 600, bset=(1, 4, 9, 13), density=0.012, empty_rows=3, unsorted=True)
    rng = np.random.default_rng(12)
    A1 = Matrix.from_operator(op, prec=prec, row_order="atom")
    A2 = Matrix.from_operator(op, prec=prec, row_order=order)
    for nrhs in (1, 2, 8, 32, 64):
        print("case order", prec, nrhs, flush=True)
        X = dev(rng.standard_normal((op.N, nrhs)), prec)
        for transpose in (False, True):
            y1 = host(A1.spmm(X, transpose=transpose))
            y2 = host(A2.spmm(X, transpose=transpose))
            assert np.array_equal(y1, y2)
        if prec != "bf16x3":
            G = dev(rng.standard_normal((op.N, nrhs)), prec)
            assert np.array_equal(host(A1.sddmm(G, X)), host(A2.sddmm(G, X)))
    ref = oracle.spmm(op, rounded(host(X), prec))
    check(host(A2.spmm(X)), ref, prec)
    from workloads.core import inf_norm_scale, scaled
    ops = scaled(op, inf_norm_scale(op))
    R = rng.standard_normal((op.N, 5))
    B1 = Matrix.from_operator(ops, prec=prec, row_order="atom")
    B2 = Matrix.from_operator(ops, prec=prec, row_order=order)
    m1 = B1.cheb_moments(dev(R, prec), 16)
    m2 = B2.cheb_moments(dev(R, prec), 16)
    assert np.max(np.abs(m1 - m2)) <= 1e-13 * np.max(np.abs(m1[0]))


def test_argument_errors_on_device():
    from paper_2609_04397_amd import _lib, VbcsrError
    import ctypes
    op = random_pattern(9, 10, bset=(2, 3), density=0.3)
    A = Matrix.from_operator(op)
    lib = _lib.load()
    X = torch.zeros((op.N, 4), dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(X.data_ptr())
    assert lib.vbcsr_spmm(A._h, p, 4, p, 4, 4, 1.0, 0.0, s) == _lib.VBCSR_EINVAL   # overlap
    Y = torch.zeros_like(X)
    q = ctypes.c_void_p(Y.data_ptr())
    assert lib.vbcsr_spmm(A._h, p, 3, q, 4, 4, 1.0, 0.0, s) == _lib.VBCSR_EINVAL   # ldx < nrhs
    assert lib.vbcsr_spmm(A._h, p, 4, q, 4, 0, 1.0, 0.0, s) == _lib.VBCSR_EINVAL   # nrhs = 0
    assert lib.vbcsr_spmm(A._h, None, 4, q, 4, 4, 1.0, 0.0, s) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_sddmm(A._h, p, 4, q, 4, 4, None, s) == _lib.VBCSR_EINVAL
    with pytest.raises(TypeError):
        A.spmm(X.float())


def test_empty_operator():
    A = Matrix(np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32))
    X = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    assert A.spmm(X).shape == (0, 3)
    assert A.sddmm(X, X).numel() == 0
    assert A.info()["N"] == 0
    B = Matrix(np.array([2, 3], np.int32), np.zeros(3, np.int64), np.zeros(0, np.int32))
    Y0 = torch.ones((5, 2), dtype=torch.float64, device="cuda")
    B.spmm(torch.ones((5, 2), dtype=torch.float64, device="cuda"), Y0, beta=3.0)
    assert np.array_equal(host(Y0), np.full((5, 2), 3.0))


def test_set_values_host_and_device():
    op = random_pattern(10, 20, bset=(1, 4, 9), density=0.3)
    A = Matrix.from_operator(op)
    X = np.random.default_rng(4).standard_normal((op.N, 3))
    v2 = np.random.default_rng(5).uniform(-1, 1, op.nnz)
    A.set_values(v2)
    check(host(A.spmm(dev(X, "fp64"))), oracle.spmm(op, X, values=v2), "fp64",
          oracle.abs_product(op, X, values=v2))
    v3 = np.random.default_rng(6).uniform(-1, 1, op.nnz)
    A.set_values(dev(v3, "fp64"))
    check(host(A.spmm(dev(X, "fp64"), transpose=True)), oracle.spmm_t(op, X, values=v3), "fp64",
          oracle.abs_product(op, X, values=v3, transpose_op=True))
    # float values into an FP64 handle are widened exactly
    v4 = v3.astype(np.float32)
    A.set_values(torch.from_numpy(v4).cuda())
    check(host(A.spmm(dev(X, "fp64"))), oracle.spmm(op, X, values=v4.astype(np.float64)), "fp64",
          oracle.abs_product(op, X, values=v4.astype(np.float64)))


def test_bitwise_reproducible():
    op, vec = make_config("C1", scale=0.3, nrhs=16)
    for prec in ("fp64", "fp32", "bf16x3"):
        A = Matrix.from_operator(op, prec=prec)
        X = dev(vec["X"], prec)
        a = host(A.spmm(X))
        b = host(A.spmm(X))
        assert np.array_equal(a, b)
        assert np.array_equal(host(A.spmm(X, transpose=True)), host(A.spmm(X, transpose=True)))
        assert np.array_equal(host(A.sddmm(X, X)), host(A.sddmm(X, X)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vec_tiles_agree_with_oracle(prec):
    """Every pass width of the vector kernel, full and ragged last passes,
    and X rows that do / do not start on 16-byte boundaries (the staging of
    whole row pieces applies only to the former)."""
    op, vec = make_config("C1", scale=0.2, nrhs=12)
    X = vec["X"]
    Xr = rounded(X, prec)
    for nrhs in (8, 12):
        ref = oracle.spmm(op, Xr[:, :nrhs])
        scale = oracle.abs_product(op, Xr[:, :nrhs]) if prec == "fp64" else None
        for tile in (1, 2, 4, 8):
            print("case vec tile", prec, nrhs, tile, flush=True)
            A = Matrix.from_operator(op, prec=prec, path="vec", nrhs_tile=tile)
            check(host(A.spmm(dev(X[:, :nrhs], prec))), ref, prec, scale, "tile %d nrhs %d" % (tile, nrhs))
            for ld, off in ((16, 0), (17, 1), (18, 2)):
                big = torch.zeros((op.N, ld), dtype=DT[prec], device="cuda")
                big[:, off:off + nrhs] = dev(X[:, :nrhs], prec)
                got = host(A.spmm(big[:, off:off + nrhs]))
                check(got, ref, prec, scale, "tile %d nrhs %d ld %d off %d" % (tile, nrhs, ld, off))
            A.close()
