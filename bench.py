#!/usr/bin/env python
"""Benchmark of the variable-block sparse hot path on one MI355X.

Headline workload (``value``): the multispecies zincblende nanoparticle --
a sphere of radius 104 A cut from a zincblende lattice (a = 5.87 A) with
13-orbital cations, 9-orbital anions and 1-orbital passivating atoms on the
dangling bonds, couplings through the third neighbour shell (199,911 atoms,
N = 2,062,795 scalar rows, 5,284,875 blocks in 9 shape classes, 632,664,771
FP64 values, 5.06 GB).  One *step* is one pass over the FP64 hot path on
this operator:

  spmm_fp64_n64    Y = A X                   nrhs 64 (the workload's width)
  spmm_t_fp64_n64  dX = A^T G                nrhs 64 (adjoint)
  sddmm_fp64_n64   dA = G X^T on the blocks  nrhs 64
  spmv_fp64        y = A x                   nrhs 1
  spmm_fp64_n8     Y = A X                   nrhs 8
  spmm_t_fp64_n8   dX = A^T G                nrhs 8
  cheb_fp64_n64    T <- 2 A' T_k - T with its FP64 moment, A' = A / (1.01 ||A||_inf)

Timed alongside, each in a loop of its own with the same protocol:

  precision  the same operator in FP32 and BF16x3 at nrhs 64 (forward);
  fwd_bwd    the differentiation form on the 100,000-atom three-species
             operator (b = 1/4/9, nrhs 32): forward + adjoint + block-sampled
             product as three raw calls and through the autograd function
             (values in graph order, and in the forward-page layout), FP32
             and plain FP64, and their ratio;
  c2_step    the 32^3 simple-cubic lattice (b = 13): SpMV, SpMM/SpMM^T/SDDMM
             at nrhs 32 and one Chebyshev step in FP64, FP32 and BF16x3 at
             nrhs 64 on the scaled operator;
  spgemm     the thresholded block product A A of the 11,520-atom operator
             with b in 9..20 (G1) at eps 0 and 1: whole call (host clock,
             median of 3 after 1) and its phases (the same records as
             --spgemm, without the oracle).

Timing: W untimed warm-up steps, then K steps bracketed by device
synchronisation; every call is also bracketed by HIP events on the stream
it is launched on (torch's current stream, which the library is handed),
which gives each kernel's average duration.

Output: one JSON line.  ``value`` is the headline step's algorithmic HBM
throughput (sum of algorithmic bytes / step time), ``roofline`` describes
its kernel with the largest time share, ``cpu_baseline`` times the FP64 CPU
oracle on a bounded sample of the same step (sampled block rows), and every
row carries ``err_vs_oracle``: its error on those sampled rows against the
oracle, computed after the timed loops.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
METRIC = "VBCSR SpMM GFLOP/s & HBM GB/s (% roofline); fwd+bwd ms vs plain FP64"


def algorithmic_bytes(op, nrhs, s_v, s_x, kind):
    """Bytes a kernel must move (no padding, each operand once).

    product:   values + 4 B per block index + 8 B per row pointer
               + X read + Y write (+ Y read when beta != 0)
    cheb:      product with beta = -1 plus the R read of the fused moment
    sddmm:     dY and X read + dA written + indices
    """
    idx = 4 * op.nnzb + 8 * (op.n + 1)
    vec = s_x * op.N * nrhs
    if kind == "product":
        return s_v * op.nnz + idx + 2 * vec
    if kind == "cheb":
        return s_v * op.nnz + idx + 4 * vec
    if kind == "sddmm":
        return s_v * op.nnz + idx + 2 * vec
    raise ValueError(kind)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sections", default="c3,precision,fwd_bwd,c2,spgemm",
                    help="comma list of timed sections (c3 is the headline)")
    ap.add_argument("--only", default="", help="comma list of rows to run (profiling)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (CPU baseline and err_vs_oracle)")
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for traffic counters)")
    ap.add_argument("--sweep", default="",
                    help="write an nrhs sweep over the workloads (JSON lines) to this file")
    ap.add_argument("--spgemm", action="store_true",
                    help="only run the block product records (G1, A A) and print them")
    ap.add_argument("--kpm", action="store_true",
                    help="only run the KPM density-of-states records and print them")
    ap.add_argument("--orders", action="store_true",
                    help="time the products of C3 and C5 in each processing order and exit")
    ap.add_argument("--kspace", action="store_true",
                    help="only run the reciprocal-space operator records and print them")
    ap.add_argument("--ceilings", action="store_true",
                    help="time plain 1 GiB fill, sum and copy kernels (write-only, read-only "
                         "and read + write rates of this device) and exit")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# timed sections
# ---------------------------------------------------------------------------

class Row:
    """One timed call: ``fn`` launches it; ``capture`` (after the timed loop)
    returns the sampled host output and what the oracle needs to check it."""

    def __init__(self, name, fn, nbytes, flops, nrhs, prec, capture=None):
        self.name, self.fn, self.nbytes, self.flops = name, fn, int(nbytes), float(flops)
        self.nrhs, self.prec, self.capture = nrhs, prec, capture


def peak_key(prec):
    return {"fp64": "fp64", "fp32": "fp32", "bf16x3": "bf16"}[prec]


def time_rows(rows, steps, warmup, only=()):
    """Warm-up, then ``steps`` timed passes over ``rows`` (each call between
    two HIP events on the current stream); returns (per-row dicts, ms/step)."""
    import torch
    if only:
        rows = [r for r in rows if r.name in only]
    if not rows:
        return [], 0.0
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        for r in rows:
            r.fn()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in rows] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(steps):
        for i, r in enumerate(rows):
            ev[st][i][0].record(stream)
            r.fn()
            ev[st][i][1].record(stream)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    out = []
    for i, r in enumerate(rows):
        t = np.array([ev[st][i][0].elapsed_time(ev[st][i][1]) for st in range(steps)])
        avg = float(t.mean())
        gbs = r.nbytes / (avg * 1e-3) / 1e9
        tf = r.flops / (avg * 1e-3) / 1e12
        roof = max(r.nbytes / (HBM_PEAK_GBS * 1e9), r.flops / (PEAK_TFLOPS[peak_key(r.prec)] * 1e12))
        out.append({"kernel": r.name, "prec": r.prec, "nrhs": r.nrhs, "avg_ms": round(avg, 5),
                    "median_ms": round(float(np.median(t)), 5), "min_ms": round(float(t.min()), 5),
                    "alg_bytes": r.nbytes, "gbs": round(gbs, 1), "tflops": round(tf, 3),
                    "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                    "roofline_frac": round(roof * 1e3 / avg, 4), "err_vs_oracle": None})
    return out, ms_step


def sample_atoms(op, k, seed, extra=()):
    """Block rows checked against the oracle: the first and last atom, ``k``
    random ones and ``extra``; returns (atoms, their scalar rows)."""
    rng = np.random.default_rng(seed)
    atoms = np.unique(np.concatenate([[0, op.n - 1], rng.choice(op.n, size=min(k, op.n),
                                                                replace=False),
                                      np.asarray(extra, dtype=np.int64)]).astype(np.int64))
    off = op.off
    srows = np.concatenate([np.arange(off[a], off[a + 1]) for a in atoms])
    return atoms, srows


def sampled_value_index(op, atoms):
    """Positions (graph order) of the values of the blocks in rows ``atoms``."""
    keep = np.isin(op.block_rows, atoms)
    base = op.block_base
    ks = np.nonzero(keep)[0]
    sizes = base[ks + 1] - base[ks]
    start = np.repeat(base[ks] - np.concatenate([[0], np.cumsum(sizes)[:-1]]), sizes)
    return keep, start + np.arange(int(sizes.sum()), dtype=np.int64)


def product_rows(prefix, op, M, prec, vecs, nrhs_list, with_t, with_sddmm, atoms, srows,
                 sddmm_nrhs=None):
    """Forward (and adjoint, SDDMM) rows of one handle; every output is
    captured on the sampled rows for the oracle leg."""
    import torch
    s_v = 8 if prec == "fp64" else 4
    s_x = 8 if prec == "fp64" else 4
    dt = torch.float64 if prec == "fp64" else torch.float32
    dev = torch.device("cuda", 0)
    sd = torch.from_numpy(srows).to(dev)
    rows = []
    for nrhs in nrhs_list:
        X = vecs["X"][:, :nrhs]
        G = vecs["G"][:, :nrhs]
        xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev, dt)
        gd = torch.from_numpy(np.ascontiguousarray(G)).to(dev, dt)
        y = torch.empty_like(xd)
        dx = torch.empty_like(xd)
        tag = "spmv" if nrhs == 1 else "spmm"
        nm = "%s%s_%s%s" % (prefix, tag, prec, "" if nrhs == 1 else "_n%d" % nrhs)
        fl = 2.0 * op.nnz * nrhs
        nb = algorithmic_bytes(op, nrhs, s_v, s_x, "product")

        def cap_f(y=y, xd=xd, X=X):
            M.spmm(xd, y)
            return {"kind": "fwd", "op": op, "X": X, "prec": prec, "atoms": atoms, "srows": srows,
                    "got": y.index_select(0, sd).double().cpu().numpy()}
        rows.append(Row(nm, lambda y=y, xd=xd: M.spmm(xd, y), nb, fl, nrhs, prec, cap_f))
        if with_t:
            def cap_t(dx=dx, gd=gd, G=G):
                M.spmm_t(gd, dx)
                return {"kind": "adj", "op": op, "X": G, "prec": prec, "atoms": atoms,
                        "srows": srows, "got": dx.index_select(0, sd).double().cpu().numpy()}
            rows.append(Row(nm.replace(tag + "_", tag + "_t_", 1),
                            lambda dx=dx, gd=gd: M.spmm_t(gd, dx), nb, fl, nrhs, prec, cap_t))
        if with_sddmm and nrhs == (sddmm_nrhs or nrhs_list[0]):
            dA = torch.empty(op.nnz, dtype=dt, device=dev)
            keep, vidx = sampled_value_index(op, atoms)
            vd = torch.from_numpy(vidx).to(dev)

            def cap_s(dA=dA, gd=gd, xd=xd, X=X, G=G, vd=vd, keep=keep):
                M.sddmm(gd, xd, dA)
                return {"kind": "sddmm", "op": op, "X": X, "G": G, "prec": prec, "keep": keep,
                        "got": dA.index_select(0, vd).double().cpu().numpy()}
            rows.append(Row("%ssddmm_%s_n%d" % (prefix, prec, nrhs),
                            lambda dA=dA, gd=gd, xd=xd: M.sddmm(gd, xd, dA),
                            algorithmic_bytes(op, nrhs, s_v, s_x, "sddmm"), fl, nrhs, prec, cap_s))
    return rows


def cheb_row(name, opc, M, prec, nrhs, seed, atoms, srows):
    """One Chebyshev step ``T <- 2 A' T_k - T`` with its fused FP64 moment on
    the scaled operator ``opc``.  The step overwrites its own input, so the
    capture runs it once more on fresh copies."""
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((opc.N, nrhs))
    Tk = rng.uniform(-1, 1, (opc.N, nrhs))
    Tp = rng.uniform(-1, 1, (opc.N, nrhs))
    Rd, Tkd, Tpd = (torch.from_numpy(a).to(dev, dt) for a in (R, Tk, Tp))
    ws = torch.empty(M.cheb_workspace_bytes(nrhs, 0), dtype=torch.uint8, device=dev)
    mu = torch.zeros(nrhs, dtype=torch.float64, device=dev)
    sd = torch.from_numpy(srows).to(dev)
    s_v = 8 if prec == "fp64" else 4

    def cap():
        T = torch.from_numpy(Tp).to(dev, dt)
        M.cheb_step(Tkd, T, Rd, mu, ws)
        return {"kind": "cheb", "op": opc, "X": Tk, "Y": Tp, "prec": prec, "atoms": atoms,
                "srows": srows, "got": T.index_select(0, sd).double().cpu().numpy()}
    return Row(name, lambda: M.cheb_step(Tkd, Tpd, Rd, mu, ws),
               algorithmic_bytes(opc, nrhs, s_v, s_v, "cheb"), 2.0 * opc.nnz * nrhs, nrhs, prec, cap)


def describe(op):
    return {"n_atoms": op.n, "N": op.N, "nnzb": op.nnzb, "n_values": op.nnz}


def run_c3(args, checks, only):
    """The headline: the FP64 hot path on the zincblende nanoparticle."""
    import torch
    from paper_2609_04397_amd import Matrix
    from workloads import make_config
    from workloads.core import inf_norm_scale, scaled

    t0 = time.time()
    op, vec = make_config("C3", nrhs=64)
    vec["G"] = np.random.default_rng(33).standard_normal((op.N, 64))
    s = inf_norm_scale(op)
    opc = scaled(op, s, name="C3 scaled")
    gen_s = time.time() - t0
    # 1/8 of the block rows (and some passivating atoms with their hosts):
    # the rows err_vs_oracle checks and the CPU baseline's sample
    h = np.nonzero(op.b == 1)[0][:40]
    atoms, srows = sample_atoms(op, op.n // 8, 3, extra=np.concatenate([h, h - 1]))
    t0 = time.time()
    A = Matrix.from_operator(op, prec="fp64")
    C = Matrix.from_operator(opc, prec="fp64")
    torch.cuda.synchronize()
    create_s = time.time() - t0
    rows = product_rows("", op, A, "fp64", vec, (64,), True, True, atoms, srows)
    rows += product_rows("", op, A, "fp64", vec, (1, 8), True, False, atoms, srows)
    rows.append(cheb_row("cheb_fp64_n64", opc, C, "fp64", 64, 34, atoms, srows))
    res, ms = time_rows(rows, args.steps, args.warmup, only)
    caps = {r.name: r.capture for r in rows if not only or r.name in only}
    for name, cap in caps.items():
        checks.append((name, cap()))
    A.close()
    C.close()
    torch.cuda.synchronize()
    info = {"workload": "C3: zincblende nanoparticle, sphere R = 104 A of a zincblende "
                        "lattice a = 5.87 A, cations b = 13, anions b = 9, passivating "
                        "b = 1 atoms on dangling bonds, couplings through the 3rd shell, "
                        "U[-1,1]*exp(-r) symmetric blocks, X/G/R ~ N(0,1), FP64",
            **describe(op), "n_shape_classes": 9, "step": [r["kernel"] for r in res],
            "setup_s": {"generate": round(gen_s, 2), "create_2_handles": round(create_s, 2)}}
    return res, ms, info, op


def run_precision(args, checks, only, op=None):
    """FP32 and BF16x3 forms of the headline operator (nrhs 64, forward)."""
    import torch
    from paper_2609_04397_amd import Matrix
    from workloads import make_config
    if op is None:
        op, _ = make_config("C3", nrhs=1)
    vec = {"X": np.random.default_rng(35).standard_normal((op.N, 64))}
    vec["G"] = vec["X"]
    atoms, srows = sample_atoms(op, 300, 5)
    out = []
    for prec in ("fp32", "bf16x3"):
        M = Matrix.from_operator(op, prec=prec)
        rows = product_rows("", op, M, prec, vec, (64,), False, False, atoms, srows)
        res, _ = time_rows(rows, args.steps, args.warmup, only)
        for r in rows:
            if not only or r.name in only:
                checks.append((r.name, r.capture()))
        out += res
        M.close()
    return out


def run_fwd_bwd(args, checks, only):
    """Differentiation form on the 100,000-atom operator: forward, adjoint and
    block-sampled product at nrhs 32, as three raw calls and through the
    autograd function (loss sum(Y o G), so dY = G), FP32 against plain FP64."""
    import torch
    from paper_2609_04397_amd import Matrix, spmm, spmm_pages
    from workloads import make_config
    op, vec = make_config("C5")
    dev = torch.device("cuda", 0)
    atoms, srows = sample_atoms(op, 400, 6)
    out = {"workload": "C5: 100,000 atoms uniform in a periodic cube (0.05 / A^3), "
                       "b = 1/4/9 (20k/40k/40k), cutoff 5 A, values U[-1,1]*exp(-r/2) "
                       "(FP32-rounded), nrhs 32, loss sum(Y o G)", **describe(op), "rows": []}
    for prec in ("fp32", "fp64"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        M = Matrix.from_operator(op, prec=prec)
        rows = product_rows("c5_", op, M, prec, vec, (32,), True, True, atoms, srows)
        V = torch.from_numpy(op.values).to(dev, dt).requires_grad_(True)
        X = torch.from_numpy(vec["X"]).to(dev, dt).requires_grad_(True)
        G = torch.from_numpy(vec["G"]).to(dev, dt)

        def autograd_step(V=V, X=X, G=G, M=M):
            Y = spmm(V, X, M)
            return torch.autograd.grad(Y, (V, X), G)
        raw_bytes, raw_flops = sum(r.nbytes for r in rows), sum(r.flops for r in rows)
        rows.append(Row("c5_autograd_fwd_bwd_%s" % prec, autograd_step, raw_bytes, raw_flops, 32,
                        prec))
        # the same step with the parameter in the forward-page layout: no
        # packing in the forward, the transposed pages rebuilt for dX
        Mp = Matrix.from_operator(op, prec=prec)
        Pg = Mp.get_pages().requires_grad_(True)

        def pages_step(P=Pg, X=X, G=G, M=Mp):
            Y = spmm_pages(P, X, M)
            return torch.autograd.grad(Y, (P, X), G)
        rows.append(Row("c5_autograd_pages_fwd_bwd_%s" % prec, pages_step, raw_bytes, raw_flops,
                        32, prec))
        res, _ = time_rows(rows, args.steps, args.warmup, only)
        for r in rows:
            if r.capture is not None and (not only or r.name in only):
                checks.append((r.name, r.capture()))
        out["rows"] += res
        raw = [r for r in res if not r["kernel"].startswith("c5_autograd")]
        if len(raw) == 3:
            out["%s_ms" % prec] = round(sum(r["avg_ms"] for r in raw), 4)
        for key, name in (("autograd", "c5_autograd_fwd_bwd_"),
                          ("autograd_pages", "c5_autograd_pages_fwd_bwd_")):
            ag = [r for r in res if r["kernel"] == name + prec]
            if ag:
                out["%s_%s_ms" % (key, prec)] = ag[0]["avg_ms"]
                if len(raw) == 3:
                    out["%s_over_raw_%s" % (key, prec)] = round(ag[0]["avg_ms"] / out["%s_ms" % prec], 3)
        M.close()
        Mp.close()
        del V, X, G, Pg
    if "fp32_ms" in out and "fp64_ms" in out:
        out["ratio_fp32_over_fp64"] = round(out["fp32_ms"] / out["fp64_ms"], 4)
    return out


def run_c2(args, checks, only):
    """The 32^3 lattice step of the previous headline: SpMV, nrhs-32
    forward/adjoint/SDDMM (FP64) and one Chebyshev step per precision form on
    the scaled operator (nrhs 64)."""
    import torch
    from paper_2609_04397_amd import Matrix
    from workloads import make_config
    from workloads.core import inf_norm_scale, scaled
    op, vec = make_config("C2", nrhs=32)
    vec["G"] = np.random.default_rng(22).standard_normal((op.N, 32))
    opc = scaled(op, inf_norm_scale(op), name="C4")
    atoms, srows = sample_atoms(op, 400, 7)
    A = Matrix.from_operator(op, prec="fp64")
    rows = product_rows("c2_", op, A, "fp64", vec, (32,), True, True, atoms, srows)
    rows += product_rows("c2_", op, A, "fp64", vec, (1,), False, False, atoms, srows)
    hs = [A]
    for prec in ("fp64", "fp32", "bf16x3"):
        M = Matrix.from_operator(opc, prec=prec)
        hs.append(M)
        rows.append(cheb_row("c2_cheb_%s_n64" % prec, opc, M, prec, 64, 44, atoms, srows))
    res, ms = time_rows(rows, args.steps, args.warmup, only)
    for r in rows:
        if not only or r.name in only:
            checks.append((r.name, r.capture()))
    for M in hs:
        M.close()
    return {"workload": "C2/C4: periodic 32^3 simple-cubic lattice, b = 13, self + 6 + 12 "
                        "neighbours, U[-1,1]*exp(-r) symmetric blocks; Chebyshev rows on "
                        "A / (1.01 ||A||_inf)", **describe(op), "ms_per_step": round(ms, 4),
            "rows": res}


def main():
    args = parse()
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU only: this library has no multi-GPU path "
                 "(requested --gpus %d)" % args.gpus)
    if args.spgemm or args.kpm or args.kspace or args.orders or args.ceilings:
        recs = (spgemm_records(with_cpu=not args.no_cpu) if args.spgemm else []) + \
            (kpm_records(with_cpu=not args.no_cpu) if args.kpm else []) + \
            (kspace_records() if args.kspace else []) + \
            (order_records() if args.orders else []) + \
            ([bandwidth_ceilings()] if args.ceilings else [])
        for rec in recs:
            print(json.dumps(rec), flush=True)
        return
    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sections = set(args.sections.split(","))
    only = set(args.only.split(",")) if args.only else set()
    checks = []
    out = {"metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded generators; the paper's inputs are not public)"}
    c3op = None
    if "c3" in sections:
        print("bench: c3 section", file=sys.stderr, flush=True)
        res, ms, info, c3op = run_c3(args, checks, only)
        nbytes = sum(r["alg_bytes"] for r in res)
        flops = sum(2.0 * info["n_values"] * r["nrhs"] for r in res)
        out["value"] = round(nbytes / (ms * 1e-3) / 1e9, 1) if res else None
        out["ms_per_step"] = round(ms, 4)
        out["config"] = info
        out["gflops"] = round(flops / (ms * 1e-3) / 1e9, 1) if res else None
        out["kernel_ms_sum"] = round(sum(r["avg_ms"] for r in res), 4)
        out["rows"] = res
        if res:
            out["roofline"] = roofline(res, "c3")
    if "precision" in sections:
        print("bench: precision section", file=sys.stderr, flush=True)
        out["precision"] = {"workload": "C3 (as the headline), nrhs 64, forward",
                            "rows": run_precision(args, checks, only, c3op)}
    c3op = None
    if "fwd_bwd" in sections:
        print("bench: fwd_bwd section", file=sys.stderr, flush=True)
        out["fwd_bwd"] = run_fwd_bwd(args, checks, only)
    if "c2" in sections:
        print("bench: c2 section", file=sys.stderr, flush=True)
        out["c2_step"] = run_c2(args, checks, only)
    if "spgemm" in sections:
        print("bench: spgemm section", file=sys.stderr, flush=True)
        out["spgemm"] = spgemm_records(with_cpu=False)
    if args.calib:
        out["copy_calib"] = copy_calibration()
    out["device"] = device_info()
    if not args.no_cpu and checks:
        print("bench: oracle leg", file=sys.stderr, flush=True)
        base, errs = oracle_leg(checks, out.get("rows", []))
        if base is not None:
            out["cpu_baseline"] = base
        for blk in [out.get("rows", []), out.get("precision", {}).get("rows", []),
                    out.get("fwd_bwd", {}).get("rows", []), out.get("c2_step", {}).get("rows", [])]:
            for r in blk:
                if r["kernel"] in errs:
                    r["err_vs_oracle"] = errs[r["kernel"]]
    if args.sweep:
        run_sweep(args.sweep)
    print(json.dumps(out), flush=True)


def roofline(rows, workload):
    """Roofline object of the row with the largest time share: HBM-bound when
    its algorithmic bytes at 8 TB/s take at least as long as its flops at the
    dtype's matrix/vector peak, else compute-bound."""
    dom = max(rows, key=lambda r: r["avg_ms"])
    pk = PEAK_TFLOPS[peak_key(dom["prec"])]
    t_mem = dom["alg_bytes"] / (HBM_PEAK_GBS * 1e9)
    t_flop = dom["tflops"] * 1e12 * dom["avg_ms"] * 1e-3 / (pk * 1e12)
    if t_mem >= t_flop:
        roof = {"bound": "hbm", "achieved": dom["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "mfma", "achieved": dom["tflops"], "peak": pk, "unit": "TFLOP/s",
                "frac": round(dom["tflops"] / pk, 4)}
    roof["kernel"] = dom["kernel"]
    roof["hbm_frac"] = dom["hbm_frac"]
    roof["traffic"] = traffic_record(dom["kernel"], workload)
    return roof


def copy_calibration():
    import torch
    dev = torch.device("cuda", 0)
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    return {"bytes_read": 1 << 30, "bytes_written": 1 << 30,
            "gbs": round(2 * (1 << 30) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)}


def bandwidth_ceilings(reps=20):
    """Rates of plain streaming kernels over 1 GiB (torch's fill, sum and
    copy), medians of ``reps`` HIP-event timings after 3 untimed calls: the
    write-only, read-only and read + write bandwidth this device reaches,
    beside the 8 TB/s datasheet peak the roofline fractions use."""
    import torch
    dev = torch.device("cuda", 0)
    n = 1 << 27
    src = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    acc = torch.empty((), dtype=torch.float64, device=dev)
    out = {"workload": "plain 1 GiB FP64 streams (torch fill_, sum, copy_)", "device": device_info()}
    for name, fn, nbytes in (("fill_write_only", lambda: dst.fill_(2.0), n * 8),
                             ("sum_read_only", lambda: torch.sum(src, dim=0, out=acc), n * 8),
                             ("copy_read_write", lambda: dst.copy_(src), 2 * n * 8)):
        ms = _time_call(fn, warm=3, reps=reps)
        out[name] = {"ms": round(ms, 4), "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac_of_8tbs": round(nbytes / (ms * 1e-3) / 8e12, 4)}
    return out


def device_info():
    """What the runtime and rocminfo report for GPU 0 (compute units, clock,
    memory), beside the datasheet figures the roofline uses (256 CUs at up to
    2.4 GHz, 288 GB HBM3E at 8 TB/s)."""
    import subprocess
    import torch
    p = torch.cuda.get_device_properties(0)
    info = {"name": p.name, "arch": getattr(p, "gcnArchName", None),
            "compute_units": p.multi_processor_count,
            "memory_gib": round(p.total_memory / 2 ** 30, 1)}
    try:
        txt = subprocess.run(["rocminfo"], capture_output=True, text=True, timeout=30).stdout
        for agent in txt.split("Agent ")[1:]:
            if "gfx" in agent and "Compute Unit" in agent:
                for line in agent.splitlines():
                    line = line.strip()
                    if line.startswith("Max Clock Freq. (MHz):"):
                        info["rocminfo_max_clock_mhz"] = int(line.split(":")[1].split()[0])
                    elif line.startswith("Compute Unit:"):
                        info["rocminfo_compute_units"] = int(line.split(":")[1].split()[0])
                    elif line.startswith("Marketing Name:"):
                        info["rocminfo_name"] = line.split(":", 1)[1].strip()
                break
    except Exception as e:  # rocminfo missing or slow: report what the runtime gave
        info["rocminfo_error"] = str(e)[:80]
    return info


def _time_call(fn, warm=3, reps=7):
    """Median of ``reps`` HIP-event timings after ``warm`` untimed calls."""
    import torch
    for _ in range(warm):
        fn()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def run_sweep(path):
    """nrhs sweep of the forward/adjoint products over the workloads, and the
    fwd+bwd form of the 100k-atom FP32 operator against plain FP64.  One JSON
    object per line in ``path``; the paper's timing protocol (median of 7
    after 3 warm-ups)."""
    import torch
    from paper_2609_04397_amd import Matrix
    from workloads import make_config

    dev = torch.device("cuda", 0)
    out = open(path, "w")

    def emit(rec):
        out.write(json.dumps(rec) + "\n")
        out.flush()
        print("sweep", rec["workload"], rec["op"], rec["prec"], rec["nrhs"], rec["ms"],
              rec.get("hbm_frac"), flush=True)

    def rate(op, prec, nrhs, ms, kind="product"):
        s_v = {"fp64": 8, "fp32": 4, "bf16x3": 4}[prec]
        s_x = 8 if prec == "fp64" else 4
        nbytes = algorithmic_bytes(op, nrhs, s_v, s_x, kind)
        flops = 2.0 * op.nnz * nrhs
        peak = PEAK_TFLOPS["fp64" if prec == "fp64" else ("fp32" if prec == "fp32" else "bf16")]
        roof = max(nbytes / (HBM_PEAK_GBS * 1e9), flops / (peak * 1e12)) * 1e3
        return {"ms": round(ms, 5), "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
                "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "roofline_frac": round(roof / ms, 4), "alg_bytes": int(nbytes)}

    # C1 (17.5 MB) stays in the 256 MB MALL between calls: also time it cold
    # (a 1 GiB scratch write before every call) and as a 1000-launch average
    op1, _ = make_config("C1", nrhs=1)
    A1 = Matrix.from_operator(op1)
    X1c = torch.randn((op1.N, 16), dtype=torch.float64, device=dev)
    Y1c = torch.empty_like(X1c)
    scratch = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    cold = []
    for _ in range(7):
        scratch.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        A1.spmm(X1c, Y1c)
        e1.record()
        e1.synchronize()
        cold.append(e0.elapsed_time(e1))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(1000):
        A1.spmm(X1c, Y1c)
    e1.record()
    e1.synchronize()
    size1 = {"workload": "C1", "n_atoms": op1.n, "N": op1.N, "nnzb": op1.nnzb, "n_values": op1.nnz}
    emit(dict(size1, op="spmm cold", prec="fp64", nrhs=16, **rate(op1, "fp64", 16, float(np.median(cold)))))
    emit(dict(size1, op="spmm 1000-launch mean", prec="fp64", nrhs=16,
              **rate(op1, "fp64", 16, e0.elapsed_time(e1) / 1000)))
    del scratch, A1, X1c, Y1c
    plan = [("C1", [("fp64", (1, 2, 4, 8, 16), True)]),
            ("C2", [("fp64", (1, 2, 4, 8, 16, 32, 64), True), ("fp32", (1, 8, 64), False),
                    ("bf16x3", (64,), False)]),
            ("C3", [("fp64", (1, 2, 4, 8, 64), True)]),
            # the paper's fixed-block (b = 8) and variable-block (b in 9..20)
            # kernel-efficiency domains, ~500 MiB each, SpMV and nrhs 16
            ("P8", [("fp64", (1, 16), True)]),
            ("G1", [("fp64", (1, 16), True)])]
    for name, forms in plan:
        op, _ = make_config(name, nrhs=1)
        size = {"workload": name, "n_atoms": op.n, "N": op.N, "nnzb": op.nnzb, "n_values": op.nnz}
        for prec, nrhss, with_t in forms:
            A = Matrix.from_operator(op, prec=prec)
            dt = torch.float64 if prec == "fp64" else torch.float32
            for nrhs in nrhss:
                X = torch.randn((op.N, nrhs), dtype=dt, device=dev)
                Y = torch.empty_like(X)
                ms = _time_call(lambda: A.spmm(X, Y))
                emit(dict(size, op="spmm", prec=prec, nrhs=nrhs, **rate(op, prec, nrhs, ms),
                          cache_resident=bool(op.nnz * (8 if prec == "fp64" else 4) < 256e6)))
                if with_t and nrhs in (1, 8, 16, 32, 64):
                    ms = _time_call(lambda: A.spmm_t(X, Y))
                    emit(dict(size, op="spmm_t", prec=prec, nrhs=nrhs, **rate(op, prec, nrhs, ms),
                              cache_resident=bool(op.nnz * 8 < 256e6)))
                del X, Y
            A.close()
        del op
    # differentiation form: forward + adjoint + block-sampled product
    op, vec = make_config("C5")
    size = {"workload": "C5", "n_atoms": op.n, "N": op.N, "nnzb": op.nnzb, "n_values": op.nnz}
    fb = {}
    for prec in ("fp32", "fp64"):
        A = Matrix.from_operator(op, prec=prec)
        dt = torch.float64 if prec == "fp64" else torch.float32
        X = torch.from_numpy(vec["X"]).to(dev, dt)
        G = torch.from_numpy(vec["G"]).to(dev, dt)
        Y, dX = torch.empty_like(X), torch.empty_like(X)
        dA = torch.empty(op.nnz, dtype=dt, device=dev)
        t_f = _time_call(lambda: A.spmm(X, Y))
        t_t = _time_call(lambda: A.spmm_t(G, dX))
        t_s = _time_call(lambda: A.sddmm(G, X, dA))
        t_all = _time_call(lambda: (A.spmm(X, Y), A.spmm_t(G, dX), A.sddmm(G, X, dA)))
        fb[prec] = t_all
        emit(dict(size, op="spmm", prec=prec, nrhs=32, **rate(op, prec, 32, t_f)))
        emit(dict(size, op="spmm_t", prec=prec, nrhs=32, **rate(op, prec, 32, t_t)))
        emit(dict(size, op="sddmm", prec=prec, nrhs=32, **rate(op, prec, 32, t_s, "sddmm")))
        emit(dict(size, op="fwd+bwd", prec=prec, nrhs=32, ms=round(t_all, 5),
                  fwd_ms=round(t_f, 5)))
        A.close()
    emit(dict(size, op="fwd+bwd ratio fp32/fp64", prec="fp32", nrhs=32,
              ms=round(fb["fp32"], 5), ratio=round(fb["fp32"] / fb["fp64"], 4)))
    del op, vec
    # the whole degree-64 recurrence of the precision form: plain (64 products)
    # and with moment doubling (32 products + 32 column dot products)
    op4, vec4 = make_config("C4", nrhs=64)
    size = {"workload": "C4", "n_atoms": op4.n, "N": op4.N, "nnzb": op4.nnzb, "n_values": op4.nnz}
    for prec in ("fp64", "fp32", "bf16x3"):
        A = Matrix.from_operator(op4, prec=prec)
        dt = torch.float64 if prec == "fp64" else torch.float32
        R = torch.from_numpy(vec4["R"]).to(dev, dt)
        ws = torch.empty(A.cheb_workspace_bytes(64, 64), dtype=torch.uint8, device=dev)
        t_plain = _time_call(lambda: A.cheb_moments(R, 64, workspace=ws), warm=1, reps=3)
        t_dbl = _time_call(lambda: A.cheb_moments(R, 64, workspace=ws, doubled=True), warm=1, reps=3)
        emit(dict(size, op="cheb degree 64", prec=prec, nrhs=64, ms=round(t_plain, 4),
                  doubled_ms=round(t_dbl, 4), speedup=round(t_plain / t_dbl, 3)))
        A.close()
    del op4, vec4
    for rec in spgemm_records(with_cpu=True):
        emit(rec)
    for rec in kpm_records(with_cpu=True):
        emit(rec)
    for rec in kspace_records():
        emit(rec)
    out.close()


def order_records():
    """The planner's processing orders side by side: FP64 products and
    block-sampled products of the zincblende particle (C3, atoms in lattice
    generation order) and of the 100,000-atom structure (C5, atoms in random
    order), with the panels in atom order, reverse Cuthill-McKee order and
    clustered order (median of 7 after 3)."""
    import torch
    from paper_2609_04397_amd import Matrix
    from workloads import make_config

    dev = torch.device("cuda", 0)
    recs = []
    for name, cases in (("C3", ((1, "spmm"), (8, "spmm"), (64, "spmm"), (64, "sddmm"))),
                        ("C5", ((1, "spmm"), (32, "spmm"), (32, "sddmm")))):
        op, _ = make_config(name, nrhs=1)
        for order in ("atom", "rcm", "cluster"):
            A = Matrix.from_operator(op, row_order=order)
            for nrhs, kind in cases:
                X = torch.randn((op.N, nrhs), dtype=torch.float64, device=dev)
                if kind == "spmm":
                    Y = torch.empty_like(X)
                    ms = _time_call(lambda: A.spmm(X, Y))
                else:
                    dA = torch.empty(op.nnz, dtype=torch.float64, device=dev)
                    ms = _time_call(lambda: A.sddmm(X, X, dA))
                rec = {"workload": name, "op": kind, "prec": "fp64", "order": order, "nrhs": nrhs,
                       "ms": round(ms, 4)}
                print("orders", json.dumps(rec), file=sys.stderr, flush=True)
                recs.append(rec)
                del X
            A.close()
        del op
    return recs


def kspace_records():
    """Reciprocal-space form of the 100k-atom cube (C5 as a periodic cell:
    every block carries its minimum-image shift, 21 images): sampling O(k)
    (R+tau convention) and complex products with O(k) and O(k)^H, FP64.
    Algorithmic bytes: sampling reads the real values (8 B each) and writes
    both complex pages (2 x 16 B per value); a product reads the complex
    pages once (16 B per value), 4 B per panel column index, X once and
    writes Y (16 B per complex element)."""
    import torch
    from paper_2609_04397_amd.kspace import KMatrix
    from workloads.configs import make_operator
    from workloads.periodic import from_cube

    Z = from_cube(make_operator("C5"))
    KM = KMatrix.from_images(Z)
    size = {"workload": "C5 periodic", "n_atoms": Z.n, "N": Z.N, "nnzb": Z.nnzb,
            "n_values": Z.nnz, "n_images": int(Z.shifts.shape[0])}
    k = np.array([0.2, -0.1, 0.35])
    ms = _time_call(lambda: KM.sample(k, "R+tau"))
    nb = 8 * Z.nnz + 2 * 16 * KM.n_values_k
    recs = [dict(size, op="kspace sample", prec="fp64", nrhs=None, ms=round(ms, 4),
                 gbs=round(nb / ms / 1e6, 1), hbm_frac=round(nb / ms / 1e6 / HBM_PEAK_GBS, 4),
                 alg_bytes=int(nb))]
    dev = torch.device("cuda", 0)
    cols = int(sum(int(Z.b[j]) for j in KM.structure()[1]))
    for nrhs in (1, 4, 16):
        X = torch.randn(Z.N, nrhs, dtype=torch.complex128, device=dev)
        Y = torch.empty_like(X)
        for adj in (False, True):
            ms = _time_call(lambda: KM.spmm(X, Y, adjoint=adj))
            nb = 16 * KM.n_values_k + 4 * cols + 2 * 16 * Z.N * nrhs
            recs.append(dict(size, op="kspace spmm_h" if adj else "kspace spmm", prec="fp64",
                             nrhs=nrhs, ms=round(ms, 4), gbs=round(nb / ms / 1e6, 1),
                             hbm_frac=round(nb / ms / 1e6 / HBM_PEAK_GBS, 4), alg_bytes=int(nb)))
    KM.close()
    return recs


def kpm_records(with_cpu=True):
    """Density of states from 147,456 Chebyshev moments (the paper's count)
    on 300,000 points of the scaled axis, Jackson damping.  The kernel takes
    one FMA and one add per moment and point (Clenshaw), so its ceiling is
    the FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz / 2
    instructions = 19.66e12 point-moments per second.  The oracle (direct
    cos(k arccos x) sums, numpy) is timed on 64 of the points."""
    import torch
    from paper_2609_04397_amd import kpm

    M, P = 147456, 300000
    lam = np.random.default_rng(5).uniform(-0.9, 0.9, 64)
    mu = np.empty(M)
    t0, t1 = np.ones_like(lam), lam.copy()
    mu[0], mu[1] = 1.0, t1.mean()
    for k in range(2, M):
        t0, t1 = t1, 2 * lam * t1 - t0
        mu[k] = t1.mean()
    dev = torch.device("cuda", 0)
    mud = torch.from_numpy(mu).to(dev)
    x = torch.linspace(-0.99, 0.99, P, dtype=torch.float64, device=dev)
    work = torch.empty(M, dtype=torch.float64, device=dev)
    ms = _time_call(lambda: kpm.dos(mud, x, "jackson", work=work))
    rate = (M - 1) * P / (ms * 1e-3)
    peak = 256 * 4 * 16 * 2.4e9 / 2
    recs = [{"workload": "KPM DOS", "op": "kpm_dos jackson", "prec": "fp64", "nrhs": None,
             "n_moments": M, "n_points": P, "ms": round(ms, 4),
             "point_moments_per_s": round(rate, 1), "alu_frac": round(rate / peak, 4),
             "alu_peak_point_moments_per_s": peak}]
    if with_cpu:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from oracle import kpm as okpm
        xs = np.linspace(-0.99, 0.99, 64)
        t = time.perf_counter()
        okpm.dos(mu, xs)
        dt = time.perf_counter() - t
        recs.append({"workload": "KPM DOS", "op": "kpm_dos oracle (numpy, 64 points)",
                     "prec": "fp64", "nrhs": None, "n_moments": M, "n_points": 64,
                     "ms": round(dt * 1e3, 2), "point_moments_per_s": round(M * 64 / dt, 1)})
    return recs


def spgemm_records(with_cpu=True):
    """Thresholded block product A A of the G1 operator (11,520 atoms, b in
    9..20, 502 MiB of FP64 values) at eps = 0 and eps = 1 (which drops about
    60 % of the product's blocks): whole-call time, its phases, and the
    numeric kernel's FP64 matrix-core rate.  The CPU oracle (one thread) is
    timed on 200 sampled block rows for comparison."""
    import torch
    from paper_2609_04397_amd import Matrix
    from workloads.configs import make_operator

    op = make_operator("G1")
    size = {"workload": "G1", "n_atoms": op.n, "N": op.N, "nnzb": op.nnzb, "n_values": op.nnz}
    A = Matrix.from_operator(op)
    recs = []
    for eps in (0.0, 1.0):
        runs = []
        for _ in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C, st = A.spgemm(A, eps)
            torch.cuda.synchronize()
            runs.append(((time.perf_counter() - t0) * 1e3, st))
            C.close()
        runs = runs[1:]  # first call warms up
        tot = float(np.median([r[0] for r in runs]))
        st = sorted(runs, key=lambda r: r[1]["ms_numeric"])[len(runs) // 2][1]
        tf = st["flops"] / (st["ms_numeric"] * 1e-3) / 1e12
        rec = dict(size, op="spgemm A A", prec="fp64", nrhs=None, eps=eps, ms=round(tot, 3),
                   numeric_ms=round(st["ms_numeric"], 4),
                   phases_ms={k[3:]: round(st[k], 3) for k in st if k.startswith("ms_")},
                   candidates=st["candidates"], kept_symbolic=st["kept_symbolic"],
                   nnzb_C=st["nnzb"], products=st["products"], gflop=round(st["flops"] / 1e9, 3),
                   numeric_tflops=round(tf, 3), mfma_frac=round(tf / PEAK_TFLOPS["fp64"], 4))
        recs.append(rec)
    A.close()
    if with_cpu:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import oracle
        rows = np.random.default_rng(0).choice(op.n, 200, replace=False)
        fl = 0.0
        for i in rows:
            ks = op.col_idx[op.row_ptr[i]:op.row_ptr[i + 1]]
            for k in ks:
                js = op.col_idx[op.row_ptr[k]:op.row_ptr[k + 1]]
                fl += 2.0 * op.b[i] * op.b[k] * float(op.b[js].sum())
        t0 = time.perf_counter()
        oracle.spgemm(op, op, 0.0, rows=rows)
        dt = time.perf_counter() - t0
        recs.append(dict(size, op="spgemm A A oracle (1 thread, 200 rows)", prec="fp64", nrhs=None,
                         eps=0.0, ms=round(dt * 1e3, 2), gflop=round(fl / 1e9, 4),
                         gflops=round(fl / dt / 1e9, 3),
                         full_product_s_est=round(dt * op.n / 200, 2)))
    return recs


def restrict(op, keep_blocks):
    """The operator with only the blocks ``keep_blocks`` (graph order kept),
    over the same atoms: its product equals the full product on every row
    whose blocks are all kept."""
    from workloads.core import Operator
    keep = np.asarray(keep_blocks, dtype=bool)
    counts = np.bincount(op.block_rows[keep], minlength=op.n)
    rp = np.zeros(op.n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    vmask = np.repeat(keep, np.diff(op.block_base))
    return Operator(op.name + "-sampled", op.b, rp, op.col_idx[keep], op.values[vmask],
                    op.dist[keep])


def oracle_leg(checks, headline_rows, budget_s=12.0):
    """The FP64 CPU oracle on the sampled block rows of every timed row.

    Returns (cpu_baseline, errors).  ``cpu_baseline`` times the oracle's
    products on the headline rows' samples (the scalar-CSR expansion of the
    sampled operator is set-up, excluded like the device planner), repeated
    until about ``budget_s`` seconds of CPU work, median per row; each
    sample's algorithmic bytes are the row's bytes scaled by the fraction of
    the operator's values the sample holds.  ``errors`` holds, per row, the
    error of the device output on the sampled rows: rel_F and componentwise
    (FP64), rel_F against the oracle on the FP64 inputs and on the inputs
    rounded to FP32 (FP32, BF16x3)."""
    import oracle

    def rounded(a, prec):
        return a if prec == "fp64" else np.asarray(a, np.float64).astype(np.float32).astype(np.float64)

    def rel_f(y, ref):
        d = np.linalg.norm(ref)
        return float(np.linalg.norm(y - ref) / d) if d > 0 else float(np.linalg.norm(y))

    def comp(y, ref, scale):
        d = np.abs(y - ref)
        z = scale == 0
        if np.any(d[z] != 0):
            return float("inf")
        return float((d / np.where(z, 1.0, scale)).max()) if d.size else 0.0

    prepared = []
    cache = {}
    for name, c in checks:
        op = c["op"]
        key = (id(op), "col" if c["kind"] == "adj" else "row",
               id(c["keep"]) if c["kind"] == "sddmm" else id(c["atoms"]))
        if key not in cache:
            if c["kind"] == "sddmm":
                cache[key] = restrict(op, c["keep"])
            elif c["kind"] == "adj":
                cache[key] = restrict(op, np.isin(op.col_idx, c["atoms"]))
            else:
                cache[key] = restrict(op, np.isin(op.block_rows, c["atoms"]))
        prepared.append((name, c, cache[key]))

    def run(c, sub, values=None, rnd="fp64"):
        """One oracle product of the check's kind on its sample."""
        X = rounded(c["X"], rnd)
        if c["kind"] == "sddmm":
            return oracle.sddmm(sub if values is None else _with(sub, values), rounded(c["G"], rnd), X)
        A = oracle.expand_op(sub, values)
        if c["kind"] == "adj":
            A = oracle.transpose(A)
        if c["kind"] == "cheb":
            Y = oracle.csr_spmm(A, X, alpha=2.0, beta=-1.0, Y=rounded(c["Y"], rnd))
        else:
            Y = oracle.csr_spmm(A, X)
        return Y[c["srows"]]

    def _with(sub, values):
        from workloads.core import Operator
        return Operator(sub.name, sub.b, sub.row_ptr, sub.col_idx, values, sub.dist)

    errors = {}
    for name, c, sub in prepared:
        got = c["got"]
        ref = run(c, sub)
        e = {"rows_checked": int(len(c["srows"])) if "srows" in c else None,
             "rel_F": rel_f(got, ref)}
        if c["prec"] == "fp64":
            if c["kind"] == "sddmm":
                scale = oracle.sddmm(sub, np.abs(c["G"]), np.abs(c["X"]))
                e["values_checked"] = int(got.size)
            else:
                A = oracle.expand_op(sub).abs()
                if c["kind"] == "adj":
                    A = oracle.transpose(A)
                scale = oracle.csr_spmm(A, np.abs(c["X"]))[c["srows"]]
                if c["kind"] == "cheb":
                    scale = 2.0 * scale + np.abs(c["Y"][c["srows"]])
            e["comp"] = comp(got, ref, scale)
        else:
            e["rel_F_rounded_inputs"] = rel_f(got, run(c, sub, rounded(sub.values, "fp32"), "fp32"))
        errors[name] = {k: (float("%.3e" % v) if isinstance(v, float) else v) for k, v in e.items()}

    # the CPU baseline: the headline rows' samples, timed
    head = {r["kernel"]: r for r in headline_rows}
    timed = [(n, c, s) for n, c, s in prepared if n in head]
    if not timed:
        return None, errors
    exp = {}
    for n, c, s in timed:
        if c["kind"] != "sddmm":
            A = oracle.expand_op(s)
            exp[n] = oracle.transpose(A) if c["kind"] == "adj" else A
    per = {n: [] for n, _, _ in timed}
    reps = 0
    t_all = time.perf_counter()
    while True:
        for n, c, s in timed:
            X = c["X"]
            t0 = time.perf_counter()
            if c["kind"] == "sddmm":
                oracle.sddmm(s, c["G"], X)
            elif c["kind"] == "cheb":
                oracle.csr_spmm(exp[n], X, alpha=2.0, beta=-1.0, Y=c["Y"])
            else:
                oracle.csr_spmm(exp[n], X)
            per[n].append(time.perf_counter() - t0)
        reps += 1
        if reps >= 3 and (time.perf_counter() - t_all >= budget_s or reps >= 7):
            break
    cpu_s = time.perf_counter() - t_all
    med = {n: float(np.median(v)) for n, v in per.items()}
    nbytes = {n: head[n]["alg_bytes"] * s.nnz / c["op"].nnz for n, c, s in timed}
    tot_b, tot_s = sum(nbytes.values()), sum(med.values())
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    frac = {n: round(s.nnz / c["op"].nnz, 5) for n, c, s in timed}
    base = {"value": round(tot_b / tot_s / 1e9, 3), "unit": "GB/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": "every row of the headline step on the FP64 scalar-CSR oracle, restricted "
                      "to the sampled block rows (adjoint: block columns) that err_vs_oracle "
                      "checks, %.2f-%.2f %% of the values; median of %d repetitions, %.1f s of CPU "
                      "work; algorithmic bytes scaled by the sampled fraction of the values; "
                      "scalar-CSR expansion excluded" % (100 * min(frac.values()),
                                                         100 * max(frac.values()), reps, cpu_s),
            "per_row_s": {n: round(v, 4) for n, v in med.items()},
            "sampled_value_fraction": frac, "cpu_model": cpu_model,
            "host_threads": os.cpu_count()}
    return base, errors


def traffic_record(kernel, workload):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    of ``workload``, or None when the sources changed since the counters
    were taken."""
    import re
    path = os.path.join(ROOT, "profiles", "pmc_traffic_%s.md" % workload)
    if not os.path.exists(path):
        return None
    m = re.search(r"<!-- traffic: (\{.*\}) -->", open(path).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("sha") != kernel_source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return int(k["fetch_bytes"] + k["write_bytes"])


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "abi.cpp", "planner.cpp", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2609_04397_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
