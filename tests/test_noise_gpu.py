"""GPU parity of the residual-likelihood reference distribution (accuracy
criterion, Sec. 5) against the FP64 oracle, through the C-ABI.

Tolerance.  The device sums -2 ln u1 per word pair (the squared radius of a
Box-Muller pair) through a running product of u1 values and one logarithm
per thread; the oracle squares and adds both normals.  Each u1 factor and
each term carries a relative rounding of a few 2^-53, so S = sum z^2 (about
n) differs by well under 1e-13 S, and lnL by at most that times
sigma_noise^2 / (2 sigma_like^2) S <= |lnL| + (n/2) |ln(2 pi sigma_like^2)|.
The bar is |dlnL| <= 1e-12 (|lnL| + n).
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import noise as nz

pytestmark = pytest.mark.gpu

FT = 301 * 96             # residuals per data set of the 301-channel, 96-bin grid


def _fgl():
    from paper_2603_13196_amd import fgl
    return fgl


def _bar(ref, n):
    return 1e-12 * (np.abs(ref) + n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 1021, 1022, 1023, 1024,
                               4 * 256 * 3 + 1, FT, FT + 3])
def test_noise_loglike_matches_oracle(n):
    R, s_n, s_l, seed = 5, 0.025, 0.025, 2603
    print(f"noise parity n={n} R={R} seed={seed}", flush=True)
    got = _fgl().fgl_noise_loglike(n, R, s_n, s_l, seed)
    ref = nz.noise_loglike(n, R, s_n, s_l, seed)
    assert np.all(np.abs(got - ref) <= _bar(ref, n)), np.max(np.abs(got - ref))


@pytest.mark.parametrize("s_n,s_l,seed", [(0.025, 0.03, 0), (0.1, 0.001, 2**64 - 1),
                                          (0.0, 0.025, 17)])
def test_noise_loglike_sigmas_and_seeds(s_n, s_l, seed):
    n, R = 4099, 3
    print(f"noise sigmas s_n={s_n} s_l={s_l} seed={seed}", flush=True)
    got = _fgl().fgl_noise_loglike(n, R, s_n, s_l, seed)
    ref = nz.noise_loglike(n, R, s_n, s_l, seed)
    assert np.all(np.abs(got - ref) <= _bar(ref, n)), np.max(np.abs(got - ref))
    if s_n == 0.0:
        np.testing.assert_allclose(got, -0.5 * n * math.log(2 * math.pi * s_l * s_l),
                                   rtol=1e-15)


def test_noise_loglike_full_size_sampled_and_distribution():
    R, s_n, seed = 4096, 0.025, 11
    print(f"noise full size n={FT} R={R}", flush=True)
    got, ms = _fgl().fgl_noise_loglike(FT, R, s_n, s_n, seed, timed=True)
    assert ms > 0.0
    for r in (0, 1, 2047, 4095):
        ref = nz.noise_loglike(FT, 1, s_n, s_n, seed, first=r)[0]
        assert abs(got[r] - ref) <= _bar(ref, FT), (r, got[r] - ref)
    norm = 0.5 * FT * math.log(2 * math.pi * s_n * s_n)
    chi2 = -2.0 * (got + norm)
    assert stats.kstest(chi2, stats.chi2(FT).cdf).pvalue > 1e-3
    assert len(np.unique(got)) == R
    # the same call again gives the same values
    assert np.array_equal(got, _fgl().fgl_noise_loglike(FT, R, s_n, s_n, seed))


def test_noise_loglike_largest_sizes():
    # the most data sets a call takes (2^23, three residuals each: a full
    # pair and a cut one), and the longest data set (2^31 residuals)
    fgl = _fgl()
    R, n, s_n, seed = 2**23, 3, 0.025, 21
    print(f"noise largest R={R} n={n}", flush=True)
    got = fgl.fgl_noise_loglike(n, R, s_n, s_n, seed)
    assert got.shape == (R,) and np.all(np.isfinite(got))
    for r in (0, 1, 2**22, R - 1):
        ref = nz.noise_loglike(n, 1, s_n, s_n, seed, first=r)[0]
        assert abs(got[r] - ref) <= _bar(ref, n), (r, got[r] - ref)
    norm = 0.5 * n * math.log(2 * math.pi * s_n * s_n)
    sub = got[np.random.default_rng(0).choice(R, 200_000, replace=False)]
    assert stats.kstest(-2.0 * (sub + norm), stats.chi2(n).cdf).pvalue > 1e-3
    n = 2**31
    print(f"noise largest n={n}", flush=True)
    one = fgl.fgl_noise_loglike(n, 1, 1.0, 1.0, 5)[0]
    S = -2.0 * (one + 0.5 * n * math.log(2 * math.pi))
    assert abs(S - n) < 6.0 * math.sqrt(2.0 * n), (S, n)


def test_noise_realisation_does_not_depend_on_the_batch():
    # realisation r is fixed by (seed, r): a smaller batch is a bitwise prefix
    fgl = _fgl()
    big = fgl.fgl_noise_loglike(1001, 300, 0.025, 0.02, 77)
    for R in (1, 7, 256, 299):
        assert np.array_equal(fgl.fgl_noise_loglike(1001, R, 0.025, 0.02, 77), big[:R]), R


def test_noise_quantile_is_exact():
    ref = _fgl().fgl_noise_loglike(1000, 2000, 0.025, 0.025, 5)
    srt = np.sort(ref)
    lbar = np.concatenate([[srt[0] - 1.0, srt[-1] + 1.0], srt[[0, 1, 999, 1998, 1999]],
                           np.linspace(srt[0], srt[-1], 37)])
    q = _fgl().fgl_noise_quantile(ref, lbar)
    assert np.array_equal(q, nz.quantile(ref, lbar))
    # ties and a reference of one value
    assert np.array_equal(_fgl().fgl_noise_quantile([1.0, 1.0, 2.0, 3.0], [1.0, 0.5, 2.5, 3.0]),
                          [0.5, 0.0, 0.75, 1.0])
    assert np.array_equal(_fgl().fgl_noise_quantile([4.0], [3.0, 4.0]), [0.0, 1.0])
