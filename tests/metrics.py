"""Error metrics shared by the tests (the paper defines none).

rel_F  = ||Y - Y_ref||_F / ||Y_ref||_F
comp   = max |Y - Y_ref| / (|A||X|), the componentwise dot-product bound
         gamma_n * sum |a x|; entries whose scale is zero must match exactly.
"""
import numpy as np


def rel_f(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(y - ref)
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return float(num / den)


def comp(y, ref, scale):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    d = np.abs(y - ref)
    zero = scale == 0.0
    if np.any(d[zero] != 0.0):
        return np.inf
    s = np.where(zero, 1.0, scale)
    return float((d / s).max()) if d.size else 0.0


def load_golden(path):
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = [float(t) for t in v.split()]
    return out
