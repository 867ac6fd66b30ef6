#!/usr/bin/env python
"""Benchmark of the variable-block sparse hot path on one MI355X.

Workload: the periodic 32x32x32 simple-cubic lattice with 13 orbitals per
atom (self + 6 + 12 neighbours, 19 blocks per row; 32,768 atoms, N =
425,984 scalar rows, 622,592 blocks, 105,218,048 values), synthetic seeded
values, FP64 unless stated.  One *step* is one pass over every product of the
hot path on this operator:

  spmv_fp64        Y = A x                   nrhs 1   (FP64)
  spmm_fp64        Y = A X                   nrhs 32  (FP64)
  spmm_t_fp64      dX = A^T G                nrhs 32  (FP64, adjoint)
  sddmm_fp64       dA = G X^T on the blocks  nrhs 32  (FP64)
  cheb_fp64        T <- 2 A' T_k - T, moment nrhs 64  (FP64, A' = A / 1.01||A||_inf)
  cheb_fp32        the same step, FP32 pages and vectors, FP64 moments
  cheb_bf16x3      the same step, BF16x3 matrix-core product, FP64 moments

The forward/adjoint/SDDMM triple is the differentiation form (fwd + bwd).
Timing: W untimed warm-up steps, then K steps bracketed by device
synchronisation; every call is also bracketed by HIP events on the stream
it is launched on, which gives each kernel's average duration.

Output: one JSON line (rank 0).  ``value`` is the step's algorithmic HBM
throughput (sum of algorithmic bytes / step time), ``roofline`` describes the
kernel with the largest time share, ``cpu_baseline`` times the FP64 CPU
oracle on a bounded sample of the same step.
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
    ap.add_argument("--lattice", type=int, default=32, help="lattice edge (32 = full workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="", help="comma list of kernels to run (profiling)")
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for traffic counters)")
    ap.add_argument("--sweep", default="",
                    help="write an nrhs sweep over the workloads (JSON lines) to this file")
    ap.add_argument("--spgemm", action="store_true",
                    help="only run the block product records (G1, A A) and print them")
    ap.add_argument("--kpm", action="store_true",
                    help="only run the KPM density-of-states records and print them")
    ap.add_argument("--kspace", action="store_true",
                    help="only run the reciprocal-space operator records and print them")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU only: this build has no multi-GPU path "
                 "(requested --gpus %d)" % args.gpus)
    if args.spgemm or args.kpm or args.kspace:
        recs = (spgemm_records(with_cpu=not args.no_cpu) if args.spgemm else []) + \
            (kpm_records(with_cpu=not args.no_cpu) if args.kpm else []) + \
            (kspace_records() if args.kspace else [])
        for rec in recs:
            print(json.dumps(rec), flush=True)
        return
    import torch
    from paper_2609_04397_amd import Matrix
    from workloads.core import sc_lattice, inf_norm_scale, scaled

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    op = sc_lattice(args.lattice, 13, seed=2, decay=1.0, name="C2")
    rng = op.meta["_rng"]
    X32 = rng.standard_normal((op.N, 32))
    X1 = np.ascontiguousarray(X32[:, :1])
    G32 = np.random.default_rng(22).standard_normal((op.N, 32))
    s = inf_norm_scale(op)
    opc = scaled(op, s, name="C4")
    R64 = np.random.default_rng(4).standard_normal((op.N, 64))
    gen_s = time.time() - t0

    t0 = time.time()
    A64 = Matrix.from_operator(op, prec="fp64")
    C64 = Matrix.from_operator(opc, prec="fp64")
    C32 = Matrix.from_operator(opc, prec="fp32")
    Cbf = Matrix.from_operator(opc, prec="bf16x3")
    torch.cuda.synchronize()
    create_s = time.time() - t0

    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float64)
    d32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    x1, x32, g32 = d64(X1), d64(X32), d64(G32)
    y1 = torch.empty_like(x1)
    y32 = torch.empty_like(x32)
    dx32 = torch.empty_like(x32)
    dA = torch.empty(op.nnz, dtype=torch.float64, device=dev)
    vecs = {}
    for name, M, conv in (("fp64", C64, d64), ("fp32", C32, d32), ("bf16x3", Cbf, d32)):
        R = conv(R64)
        Tk = conv(np.random.default_rng(5).uniform(-1, 1, (op.N, 64)))
        Tp = conv(np.random.default_rng(6).uniform(-1, 1, (op.N, 64)))
        ws = torch.empty(M.cheb_workspace_bytes(64, 0), dtype=torch.uint8, device=dev)
        mu = torch.zeros(64, dtype=torch.float64, device=dev)
        vecs[name] = (M, R, Tk, Tp, ws, mu)

    def cheb(name):
        M, R, Tk, Tp, ws, mu = vecs[name]
        return lambda: M.cheb_step(Tk, Tp, R, mu, ws)

    kernels = [
        ("spmv_fp64", lambda: A64.spmm(x1, y1), algorithmic_bytes(op, 1, 8, 8, "product"), 1, "fp64"),
        ("spmm_fp64", lambda: A64.spmm(x32, y32), algorithmic_bytes(op, 32, 8, 8, "product"), 32, "fp64"),
        ("spmm_t_fp64", lambda: A64.spmm_t(g32, dx32), algorithmic_bytes(op, 32, 8, 8, "product"), 32, "fp64"),
        ("sddmm_fp64", lambda: A64.sddmm(g32, x32, dA), algorithmic_bytes(op, 32, 8, 8, "sddmm"), 32, "fp64"),
        ("cheb_fp64", cheb("fp64"), algorithmic_bytes(op, 64, 8, 8, "cheb"), 64, "fp64"),
        ("cheb_fp32", cheb("fp32"), algorithmic_bytes(op, 64, 4, 4, "cheb"), 64, "fp32"),
        ("cheb_bf16x3", cheb("bf16x3"), algorithmic_bytes(op, 64, 4, 4, "cheb"), 64, "bf16"),
    ]
    if args.only:
        keep = set(args.only.split(","))
        kernels = [k for k in kernels if k[0] in keep]

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        for k in kernels:
            k[1]()
    torch.cuda.synchronize()

    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in kernels] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for st in range(args.steps):
        for i, k in enumerate(kernels):
            ev[st][i][0].record(stream)
            k[1]()
            ev[st][i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_step = wall * 1e3 / args.steps

    rows = []
    total_bytes = 0
    total_flops = 0
    for i, (name, _, nbytes, nrhs, dt) in enumerate(kernels):
        times = np.array([ev[st][i][0].elapsed_time(ev[st][i][1]) for st in range(args.steps)])
        avg_ms = float(times.mean())
        flops = 2.0 * op.nnz * nrhs
        total_bytes += nbytes
        total_flops += flops
        gbs = nbytes / (avg_ms * 1e-3) / 1e9
        tf = flops / (avg_ms * 1e-3) / 1e12
        roof_ms = max(nbytes / (HBM_PEAK_GBS * 1e9), flops / (PEAK_TFLOPS[dt] * 1e12)) * 1e3
        rows.append({"kernel": name, "nrhs": nrhs, "avg_ms": round(avg_ms, 5),
                     "median_ms": round(float(np.median(times)), 5),
                     "min_ms": round(float(times.min()), 5),
                     "alg_bytes": int(nbytes), "gbs": round(gbs, 1), "tflops": round(tf, 3),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "roofline_frac": round(roof_ms / avg_ms, 4)})

    dom = max(rows, key=lambda r: r["avg_ms"])
    dom_dt = [k[4] for k in kernels if k[0] == dom["kernel"]][0]
    hbm_bound = dom["alg_bytes"] / (HBM_PEAK_GBS * 1e9) >= 2.0 * op.nnz * dom["nrhs"] / (PEAK_TFLOPS[dom_dt] * 1e12)
    if hbm_bound:
        roof = {"bound": "hbm", "achieved": dom["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "mfma", "achieved": dom["tflops"], "peak": PEAK_TFLOPS[dom_dt],
                "unit": "TFLOP/s", "frac": round(dom["tflops"] / PEAK_TFLOPS[dom_dt], 4)}
    roof["kernel"] = dom["kernel"]
    roof["traffic"] = traffic_record(dom["kernel"])

    kernel_ms = sum(r["avg_ms"] for r in rows)
    value = total_bytes / (ms_step * 1e-3) / 1e9
    fwd = [r for r in rows if r["kernel"] == "spmm_fp64"]
    fb = [r for r in rows if r["kernel"] in ("spmm_fp64", "spmm_t_fp64", "sddmm_fp64")]
    out = {
        "metric": "VBCSR SpMM GFLOP/s & HBM GB/s (% roofline); fwd+bwd ms vs plain FP64",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sc-lattice %d^3, b=13, 19 blocks/row (self+6+12), "
                               "U[-1,1]*exp(-r) symmetric blocks, X/G/R ~ N(0,1)" % args.lattice,
                   "n_atoms": op.n, "N": op.N, "nnzb": op.nnzb, "n_values": op.nnz,
                   "step": [k[0] for k in kernels]},
        "gflops": round(total_flops / (ms_step * 1e-3) / 1e9, 1),
        "kernel_ms_sum": round(kernel_ms, 4),
        "rows": rows,
        "roofline": roof,
        "fwd_bwd_fp64_ms": round(sum(r["avg_ms"] for r in fb), 4) if len(fb) == 3 else None,
        "fwd_bwd_over_fwd": round(sum(r["avg_ms"] for r in fb) / fwd[0]["avg_ms"], 3)
        if len(fb) == 3 else None,
        "setup_s": {"generate": round(gen_s, 2), "create_4_handles": round(create_s, 2)},
        "device": device_info(),
    }
    if args.calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        out["copy_calib"] = {"bytes_read": 1 << 30, "bytes_written": 1 << 30,
                             "gbs": round(2 * (1 << 30) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)}
    if args.sweep:
        run_sweep(args.sweep)
    if not args.no_cpu and len(kernels) == 7:
        out["cpu_baseline"] = cpu_baseline(op, opc, X1, X32, G32, R64, total_bytes)
    print(json.dumps(out))


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


def cpu_baseline(op, opc, X1, X32, G32, R64, step_bytes, budget_s=12.0):
    """The FP64 oracle (all host cores) on every product of the step, full
    size, repeated until about ``budget_s`` seconds of CPU work are timed;
    the oracle's scalar-CSR expansion and transpose are set-up, excluded like
    the device planner.  Every precision form runs as the FP64 oracle."""
    import oracle

    A = oracle.expand_op(op)
    At = oracle.transpose(A)
    Ac = oracle.expand_op(opc)
    T = np.random.default_rng(5).uniform(-1, 1, (op.N, 64))
    Tp = np.random.default_rng(6).uniform(-1, 1, (op.N, 64))
    names = ["spmv_fp64", "spmm_fp64", "spmm_t_fp64", "sddmm_fp64", "cheb_fp64", "cheb_fp32",
             "cheb_bf16x3"]
    per = {k: [] for k in names}
    reps = 0
    t_all = time.perf_counter()
    while True:
        t = {}
        t0 = time.perf_counter()
        oracle.csr_spmm(A, X1)
        t["spmv_fp64"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.csr_spmm(A, X32)
        t["spmm_fp64"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.csr_spmm(At, G32)
        t["spmm_t_fp64"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.sddmm(op, G32, X32)
        t["sddmm_fp64"] = time.perf_counter() - t0
        for k in ("cheb_fp64", "cheb_fp32", "cheb_bf16x3"):
            t0 = time.perf_counter()
            Y = oracle.csr_spmm(Ac, T, alpha=2.0, beta=-1.0, Y=Tp)
            (R64 * Y).sum(axis=0)
            t[k] = time.perf_counter() - t0
        reps += 1
        for k in names:
            per[k].append(t[k])
        if time.perf_counter() - t_all >= budget_s or reps >= 7:
            break
    med = {k: float(np.median(v)) for k, v in per.items()}
    step_s = sum(med.values())
    cores = oracle.max_threads()
    # the same oracle on one thread (bitwise the same results), on the SpMV
    # and the nrhs-32 SpMM only: the whole step would take ~20 s there
    oracle.set_threads(1)
    try:
        t1 = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.csr_spmm(A, X1)
            oracle.csr_spmm(A, X32)
            t1.append(time.perf_counter() - t0)
    finally:
        oracle.set_threads(cores)
    one = float(np.median(t1))
    one_bytes = algorithmic_bytes(op, 1, 8, 8, "product") + algorithmic_bytes(op, 32, 8, 8, "product")
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(step_bytes / step_s / 1e9, 3), "unit": "GB/s",
            "cores": cores, "kind": "oracle",
            "sample": "the whole step (7 products, full size) on the FP64 scalar-CSR oracle, "
                      "median of %d repetitions (%.1f s of CPU work); expansion/transpose "
                      "excluded; FP32/BF16x3 forms run as FP64" % (reps, time.perf_counter() - t_all),
            "step_s": round(step_s, 4),
            "per_kernel_s": {k: round(v, 4) for k, v in med.items()},
            "single_thread": {"value": round(one_bytes / one / 1e9, 3), "unit": "GB/s",
                              "sample": "spmv_fp64 + spmm_fp64 (nrhs 32), median of 3",
                              "s": round(one, 4)},
            "cpu_model": cpu_model, "host_threads": os.cpu_count()}


def traffic_record(kernel):
    """HBM bytes per launch of ``kernel`` from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "pmc_traffic.md")
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
