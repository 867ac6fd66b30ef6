"""Helpers for the GPU parity tests: every product goes through the C ABI
(paper_2609_04397_amd.Matrix) and is compared with the CPU oracle."""
import numpy as np
import torch

import oracle
from metrics import rel_f, comp

TOL = {  # relative Frobenius / componentwise bounds against the FP64 oracle
    "fp64": (1e-12, 1e-12),
    # FP32 storage and accumulation: input rounding 2^-24 plus sqrt(n) growth
    "fp32": (1e-5, None),
    # BF16x3: each product keeps hi*hi + hi*lo + lo*hi of a 16-bit split,
    # relative error <= 3 * 2^-18 ~ 1.1e-5 per term, plus FP32 accumulation
    "bf16x3": (5e-5, None),
}
DT = {"fp64": torch.float64, "fp32": torch.float32, "bf16x3": torch.float32}


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=DT[prec])


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rounded(a, prec):
    """The FP64 value of what the device sees for a given precision."""
    return a if prec == "fp64" else a.astype(np.float32).astype(np.float64)


def check(got, ref, prec, scale=None, label=""):
    rf_tol, comp_tol = TOL[prec]
    r = rel_f(got, ref)
    assert r <= rf_tol, "%s rel_F %.3e > %.1e" % (label, r, rf_tol)
    if comp_tol is not None and scale is not None:
        c = comp(got, ref, scale)
        assert c <= comp_tol, "%s comp %.3e > %.1e" % (label, c, comp_tol)
    return r
