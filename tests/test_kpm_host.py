"""Host entry points of the KPM reconstruction (threshold, gap) against the
oracle: no device needed."""
import numpy as np
import pytest

from oracle import kpm as okpm
from paper_2609_04397_amd import _lib, kpm


@pytest.mark.parametrize("M,N", [(1, 1), (512, 2000), (147456, 1063609)])
def test_threshold_matches_oracle(M, N):
    assert kpm.threshold(M, N, 0.1) == pytest.approx(0.1 * okpm.single_state_peak(M, N), rel=1e-15)


def test_gap_matches_oracle_on_random_densities():
    rng = np.random.default_rng(0)
    for trial in range(200):
        n = int(rng.integers(0, 60))
        x = np.sort(rng.uniform(-1, 1, n))
        x = np.unique(x)
        rho = rng.uniform(0, 1, x.size) * (rng.random(x.size) < 0.6)
        thr = float(rng.uniform(0.05, 0.6))
        assert kpm.gap(x, rho, thr) == okpm.gap(x, rho, thr)


def test_gap_errors_and_edges():
    x = np.array([0.0, 0.1, 0.2, 0.3])
    assert kpm.gap(x, np.array([1.0, 0.0, 0.0, 1.0]), 0.5) == (0.0, 0.3)
    assert kpm.gap(x, np.array([0.0, 1.0, 1.0, 0.0]), 0.5) is None   # runs at the ends do not count
    assert kpm.gap(x[:0], x[:0], 0.5) is None
    with pytest.raises(_lib.VbcsrError):
        kpm.gap(np.array([0.0, 0.0, 1.0]), np.ones(3), 0.5)
    with pytest.raises(_lib.VbcsrError):
        kpm.threshold(0, 10, 0.1)
    lib = _lib.load()
    assert lib.vbcsr_kpm_dos(None, 4, 1, None, 0, None, None, None) == _lib.VBCSR_EINVAL
    assert lib.vbcsr_kpm_dos(None, 0, 1, None, 0, None, None, None) == _lib.VBCSR_EINVAL
