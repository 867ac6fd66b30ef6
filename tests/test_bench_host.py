"""Host-side checks of the benchmark harness (no GPU): the one-GPU refusal,
the algorithmic byte model against a brute-force count over the blocks, the
roofline object's choice of bound, the rule that a counter-based traffic
figure is reported only for the kernel sources it was taken on, and that
every profile summary's command runs files of the repository."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from workloads import random_pattern

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line for a configuration it did not run


@pytest.mark.parametrize("seed", [1, 2])
def test_algorithmic_bytes_against_a_block_count(bench, seed):
    op = random_pattern(seed=seed, n=23, bset=(1, 4, 9, 13), density=0.3, empty_rows=2, unsorted=True)
    # brute force over the stored blocks: values, one 4-byte column index per
    # block, one 8-byte pointer per block row (+1), the vectors
    nvals = 0
    for i in range(op.n):
        for k in range(op.row_ptr[i], op.row_ptr[i + 1]):
            nvals += int(op.b[i]) * int(op.b[op.col_idx[k]])
    nblocks = int(op.row_ptr[-1])
    N = int(np.sum(op.b))
    for s_v, s_x in ((8, 8), (4, 4)):
        for nrhs in (1, 8, 64):
            vec = s_x * N * nrhs
            base = s_v * nvals + 4 * nblocks + 8 * (op.n + 1)
            assert bench.algorithmic_bytes(op, nrhs, s_v, s_x, "product") == base + 2 * vec
            # the fused moment reads R and the recurrence reads T_{k-1}
            assert bench.algorithmic_bytes(op, nrhs, s_v, s_x, "cheb") == base + 4 * vec
            # dY and X read, dA written (as many values as the operator holds)
            assert bench.algorithmic_bytes(op, nrhs, s_v, s_x, "sddmm") == base + 2 * vec
    with pytest.raises(ValueError):
        bench.algorithmic_bytes(op, 1, 8, 8, "other")


def _row(name, prec, ms, nbytes, flops):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": name, "prec": prec, "avg_ms": ms, "alg_bytes": nbytes, "gbs": gbs,
            "tflops": flops / (ms * 1e-3) / 1e12, "hbm_frac": gbs / 8000.0}


def test_roofline_takes_the_longest_row_and_its_bound(bench):
    # 1 GB in 0.25 ms (4 TB/s) with few flops: bandwidth-bound
    mem = _row("mem", "fp64", 0.25, 1e9, 1e9)
    # 0.5 GB with 60 GFLOP in 1 ms: 60 GFLOP take 0.76 ms at 78.6 TFLOP/s,
    # its bytes 0.0625 ms at 8 TB/s, so the matrix peak bounds it
    mm = _row("mm", "fp64", 1.0, 5e8, 6e10)
    roof = bench.roofline([mem, mm], "no_such_workload")
    assert roof["kernel"] == "mm" and roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s"
    assert roof["peak"] == 78.6
    assert roof["frac"] == pytest.approx(60.0 / 78.6, abs=1e-4)
    assert roof["traffic"] is None   # no counter summary for this workload
    mem2 = _row("mem2", "fp32", 2.0, 8e9, 1e9)
    roof = bench.roofline([mem, mm, mem2], "no_such_workload")
    assert roof["kernel"] == "mem2" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    assert roof["frac"] == pytest.approx(4000.0 / 8000.0, abs=1e-4)


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(bench, tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"sha": bench.kernel_source_sha(),
           "kernels": {"k": {"fetch_bytes": 1000, "write_bytes": 24}}}
    (prof / "pmc_traffic_w.md").write_text("summary\n<!-- traffic: %s -->\n" % json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # kernel_source_sha reads the sources under ROOT: keep the real ones
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: rec["sha"])
    assert bench.traffic_record("k", "w") == 1024
    assert bench.traffic_record("other", "w") is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench.traffic_record("k", "w") is None


def test_committed_counter_summaries_name_their_sources(bench):
    """Each committed traffic summary carries the source hash it was taken
    on; bench.py reports its figure only while that hash is current."""
    for w in ("c3", "c5"):
        path = os.path.join(ROOT, "profiles", "pmc_traffic_%s.md" % w)
        assert os.path.exists(path), path
        text = open(path).read()
        start = text.index("<!-- traffic: ") + len("<!-- traffic: ")
        rec = json.loads(text[start:text.index(" -->", start)])
        assert len(rec["sha"]) == 16 and rec["kernels"]
        for k in rec["kernels"].values():
            assert k["fetch_bytes"] > 0 and k["write_bytes"] > 0


def test_profile_commands_run_committed_files_only():
    """Every profile summary gives the command that made it; the scripts
    those commands run are files of the repository, never working files."""
    import re
    import glob
    prof = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert prof
    for path in prof:
        text = open(path).read()
        blocks = re.findall(r"```\n(.*?)```", text, re.S)
        cmds = [l for b in blocks for l in b.splitlines() if "rocprofv3" in l]
        assert cmds, "%s gives no rocprofv3 command" % os.path.basename(path)
        for c in cmds:
            assert "_work" not in c, c
            prog = c.split(" -- ", 1)[1].split()
            scripts = [t for t in prog if t.endswith((".py", ".sh"))]
            assert scripts, c
            for t in scripts:
                rel = t.replace("$REPO/", "")
                assert os.path.isfile(os.path.join(ROOT, rel)), (os.path.basename(path), t)
