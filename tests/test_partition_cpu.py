"""The library's partition (fgl_partition, host code of libfgl) against the
oracle's Algorithms 1 and 2: bit-identical edges on the same weights (CPU,
no device call)."""
import numpy as np
import pytest

from oracle import regions
from workload.sky import make_sky
from tests.regions_pins import GOLDEN


def test_worked_examples():
    from paper_2603_13196_amd import fgl
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        head, b, w, e = [x.strip() for x in line.split("|")]
        meth, k = head.split()
        got = fgl.fgl_partition(np.array(b.split(), float), np.array(w.split(), float), int(k), meth)
        assert np.array_equal(got, np.array(e.split(), float)), (line, got)


@pytest.mark.parametrize("method", ["hierarchical", "recursive"])
@pytest.mark.parametrize("scheme", regions.SCHEMES)
def test_equals_oracle_on_sky_importance(method, scheme):
    from paper_2603_13196_amd import fgl
    s = make_sky(24, 48, np.linspace(50.0, 200.0, 7), 6, seed=17)
    I = regions.importance(s, scheme)
    for n in (1, 2, 3, 5, 8, 13, 24):
        want = regions.partition(s.beta, I, n, method)
        got = fgl.fgl_partition(s.beta, I, n, method)
        assert np.array_equal(got, want), (n, got, want)


def test_ties_and_degenerate():
    from paper_2603_13196_amd import fgl
    rng = np.random.Generator(np.random.PCG64(3))
    b = np.round(rng.normal(2.8, 0.1, 400), 2)          # many equal indices
    w = rng.integers(0, 3, 400).astype(float)           # zero weights too
    for method in ("hierarchical", "recursive"):
        for n in range(1, 20):
            assert np.array_equal(fgl.fgl_partition(b, w, n, method),
                                  regions.partition(b, w, n, method)), (method, n)
    one = fgl.fgl_partition([2.7], [1.0], 3, "recursive")
    assert np.array_equal(one, regions.partition(np.array([2.7]), np.array([1.0]), 3, "recursive"))


def test_argument_errors():
    from paper_2603_13196_amd import fgl
    for args in (([], [], 2, "recursive"), ([1.0], [0.0], 2, "recursive"),
                 ([1.0, np.nan], [1, 1], 2, "recursive"), ([1.0], [-1.0], 1, "recursive"),
                 ([1.0], [1.0], 0, "recursive"), ([1.0], [1.0], 2, 7)):
        with pytest.raises(fgl.FGLError) as e:
            fgl.fgl_partition(*args)
        assert e.value.code == fgl.FGL_EINVAL
