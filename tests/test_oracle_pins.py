"""The FP64 oracle against what the paper and mathematics fix (CPU only)."""
import pytest

import oracle
from tests import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_threads_do_not_change_results(orc):
    import numpy as np
    import workload
    w = workload.config(workload.MEDIUM, B=64)
    a = orc.loglike_w(w, threads=1)
    b = orc.loglike_w(w, threads=4)
    assert np.array_equal(a, b)


def test_workload_truth_is_near_best_fit(orc):
    """The simulated data sit within the noise of the region model at the
    truth: chi-square per element is close to sigma^2 (the sub-pixel
    mismatch of the sky simulation is far below the 25 mK noise)."""
    import numpy as np
    import workload
    w = workload.config(workload.SMALL, B=8)
    th = w.truth[None, :]
    ll = orc.loglike_w(w, th)[0]
    n = w.F * w.T
    s2 = w.truth[-1] ** 2
    chi2 = -2.0 * s2 * (ll + 0.5 * n * np.log(2 * np.pi * s2))
    assert 0.7 < chi2 / (n * s2) < 1.3, chi2 / (n * s2)
