"""Pins of the residual-likelihood oracle (accuracy criterion, Sec. 5).

- The generator against numpy's own Philox4x64-10 bit generator (an
  implementation of the same published generator, written independently).
- The normals against the standard normal law (Kolmogorov-Smirnov), and the
  reference lnL against the chi-squared law with n degrees of freedom that
  the sum of n squared standard normals follows.
- lnL_noise against the oracle's full likelihood (Eq. likelihood) evaluated at
  the parameters that generated data = model + noise: the definition of the
  reference distribution, through an independent code path.
- The quantile q against brute-force special cases.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workload
from oracle import noise as nz


@pytest.mark.parametrize("key,ctr", [
    ((1, 2), (5, 0, 0, 0)),
    ((0, 0), (1, 0, 0, 0)),
    ((2**64 - 1, 0x123), (2**64 - 16, 7, 9, 2**64 - 1)),
    ((0x0123456789ABCDEF, 2**63), (2**40 + 3, 2**63 + 5, 0, 12345)),
])
def test_philox_matches_numpy_bit_generator(key, ctr):
    # numpy's Philox increments its counter before each block, so start it
    # one below the block wanted
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array([ctr[0] - 1, *ctr[1:]], dtype=np.uint64))
    ref = g.random_raw(8)
    c2 = (ctr[0] + 1, *ctr[1:])
    got = nz.philox4x64(np.array([ctr, c2], dtype=np.uint64), key).reshape(-1)
    assert np.array_equal(got, ref)


def test_normals_are_standard_normal():
    z = np.concatenate([nz.normals(50_001, r, 7) for r in range(4)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    # pairs from one (u1, u2) are uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5.0 / math.sqrt(z.size / 2)


def test_normals_layout():
    # a prefix of a realisation does not depend on its length; realisations
    # and seeds differ
    a = nz.normals(13, 3, 11)
    for n in (1, 2, 3, 4, 5, 8, 12):
        assert np.array_equal(nz.normals(n, 3, 11), a[:n])
    assert not np.array_equal(nz.normals(13, 4, 11), a)
    assert not np.array_equal(nz.normals(13, 3, 12), a)
    # word pairs: normals 2j and 2j+1 share rho
    z = nz.normals(4000, 0, 5)
    rho2 = z[0::2] ** 2 + z[1::2] ** 2
    ctr = np.zeros((1000, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1000, dtype=np.uint64)
    x = nz.philox4x64(ctr, (5, 0)).reshape(-1, 2)
    u1 = ((x[:, 0] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    np.testing.assert_allclose(rho2, -2.0 * np.log(u1), rtol=1e-13)


def test_noise_loglike_is_chi_squared():
    n, R, s_n, s_l = 60, 600, 0.025, 0.03
    lnl = nz.noise_loglike(n, R, s_n, s_l, seed=3)
    norm = 0.5 * n * math.log(2.0 * math.pi * s_l * s_l)
    chi2 = -2.0 * (lnl + norm) * s_l * s_l / (s_n * s_n)
    assert stats.kstest(chi2, stats.chi2(n).cdf).pvalue > 1e-3
    assert abs(chi2.mean() - n) < 5.0 * math.sqrt(2.0 * n / R)


@pytest.mark.parametrize("T", [1, 4])
def test_noise_loglike_is_the_likelihood_of_model_plus_noise(T):
    w = workload.make(4, workload.freq_grid(50.0, 200.0, 1.0), T, 2,
                      workload.SEED_BASE + 41)
    orc = oracle.load()
    F = w.freqs.size
    n, R, s_n, s_l, seed = F * T, 5, 0.025, 0.02, 99
    m = orc.model(w.K, w.freqs, w.nu_ref, w.t_cmb, w.truth)
    row = w.truth.copy()
    row[-1] = s_l
    ref = np.array([orc.loglike(w.K, w.freqs, m + s_n * nz.normals(n, r, seed).reshape(F, T),
                                w.nu_ref, w.t_cmb, row[None, :])[0] for r in range(R)])
    got = nz.noise_loglike(n, R, s_n, s_l, seed)
    np.testing.assert_allclose(got, ref, rtol=1e-9)


def test_quantile_special_cases():
    rng = np.random.default_rng(1)
    ref = rng.normal(size=1000)
    srt = np.sort(ref)
    assert nz.quantile(ref, [srt[0] - 1.0])[0] == 0.0
    assert nz.quantile(ref, [srt[-1]])[0] == 1.0
    k = np.array([0, 9, 499, 998])
    np.testing.assert_array_equal(nz.quantile(ref, srt[k]), (k + 1) / 1000.0)
    # ties count as "at or below"
    np.testing.assert_array_equal(nz.quantile([1.0, 1.0, 2.0, 3.0], [1.0, 0.5, 2.5]),
                                  [0.5, 0.0, 0.75])
