"""Pins of the residual-likelihood oracle (accuracy criterion, Sec. 5).

- The generator against the known-answer blocks published with
  Philox4x32-10 (Salmon et al., SC 2011, and the Random123 release that
  accompanies it), and the counter layout of both streams of the normals
  through that pinned generator.
- The normals against the standard normal law (Kolmogorov-Smirnov), and the
  reference lnL against the chi-squared law with n degrees of freedom that
  the sum of n squared standard normals follows.
- lnL_noise against the oracle's full likelihood (Eq. likelihood) evaluated at
  the parameters that generated data = model + noise: the definition of the
  reference distribution, through an independent code path.
- The quantile q against brute-force special cases.

Every pin takes the oracle module as an argument, so that copies of it with
a planted mistake can be run through the same pins.
"""
import math
import types

import numpy as np
import pytest
from scipy import stats

import oracle
import workload
from oracle import noise as nz

# Philox4x32-10 known answers: (key, counter, block)
PHILOX_KAT = [
    ((0x00000000, 0x00000000), (0x00000000, 0x00000000, 0x00000000, 0x00000000),
     (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0xA4093822, 0x299F31D0), (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def pin_philox(m):
    ctr = np.array([c for _, c, _ in PHILOX_KAT], dtype=np.uint32)
    for i, (key, c, want) in enumerate(PHILOX_KAT):
        got = m.philox4x32(np.array([c, c], dtype=np.uint32), key)
        assert got.dtype == np.uint32
        assert [int(x) for x in got[0]] == list(want), key
        assert np.array_equal(got[0], got[1])
    # a batch of counters is the blocks one by one
    key = PHILOX_KAT[2][0]
    batch = m.philox4x32(ctr, key)
    for i in range(len(ctr)):
        assert np.array_equal(batch[i], m.philox4x32(ctr[i:i + 1], key)[0])


def pin_layout(m):
    # under key (seed low word, seed high word), block b of stream s is
    # Philox of counter (b, r, s, 0x6e6f6973); normals 2j and 2j+1 are the
    # Box-Muller pair of u1 = (w + 1) 2^-32 and u2 = v 2^-32, w and v word j
    # of the two streams (the counters are built here, the generator is the
    # pinned one)
    r, seed, nblk = 3, (1 << 40) + 11, 300

    def words(stream):
        ctr = np.zeros((nblk, 4), dtype=np.uint32)
        ctr[:, 0] = np.arange(nblk)
        ctr[:, 1] = r
        ctr[:, 2] = stream
        ctr[:, 3] = 0x6E6F6973
        return m.philox4x32(ctr, (seed & 0xFFFFFFFF, seed >> 32)).reshape(-1)

    u1 = (words(0).astype(np.float64) + 1.0) * 2.0 ** -32
    u2 = words(1).astype(np.float64) * 2.0 ** -32
    z = m.normals(8 * nblk, r, seed)
    np.testing.assert_allclose(z[0::2] ** 2 + z[1::2] ** 2, -2.0 * np.log(u1), rtol=1e-12)
    ang = np.mod(np.arctan2(z[1::2], z[0::2]), 2.0 * math.pi)
    d = np.abs(ang - 2.0 * math.pi * u2)
    assert np.all(np.minimum(d, 2.0 * math.pi - d) < 1e-9)
    # a prefix of a realisation does not depend on its length; realisations
    # and seeds (either word) differ
    a = m.normals(13, 3, 11)
    for n in (1, 2, 3, 4, 5, 8, 9, 12):
        assert np.array_equal(m.normals(n, 3, 11), a[:n])
    assert not np.array_equal(m.normals(13, 4, 11), a)
    assert not np.array_equal(m.normals(13, 3, 12), a)
    assert not np.array_equal(m.normals(13, 3, 11 + (1 << 32)), a)


def pin_normals(m):
    z = np.concatenate([m.normals(50_001, r, 7) for r in range(4)])
    assert np.all(np.isfinite(z))
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    # the two normals of a pair are uncorrelated, and so are their squares
    k = 5.0 / math.sqrt(z.size / 2)
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < k
    assert abs(np.corrcoef(z[0::2] ** 2, z[1::2] ** 2)[0, 1]) < k


def pin_chi2(m):
    n, R, s_n, s_l = 60, 600, 0.025, 0.03
    lnl = m.noise_loglike(n, R, s_n, s_l, seed=3)
    norm = 0.5 * n * math.log(2.0 * math.pi * s_l * s_l)
    chi2 = -2.0 * (lnl + norm) * s_l * s_l / (s_n * s_n)
    assert stats.kstest(chi2, stats.chi2(n).cdf).pvalue > 1e-3
    assert abs(chi2.mean() - n) < 5.0 * math.sqrt(2.0 * n / R)


def pin_likelihood(m, T=4):
    w = workload.make(4, workload.freq_grid(50.0, 200.0, 1.0), T, 2,
                      workload.SEED_BASE + 41)
    orc = oracle.load()
    F = w.freqs.size
    n, R, s_n, s_l, seed = F * T, 5, 0.025, 0.02, 99
    mod = orc.model(w.K, w.freqs, w.nu_ref, w.t_cmb, w.truth)
    row = w.truth.copy()
    row[-1] = s_l
    ref = np.array([orc.loglike(w.K, w.freqs, mod + s_n * m.normals(n, r, seed).reshape(F, T),
                                w.nu_ref, w.t_cmb, row[None, :])[0] for r in range(R)])
    got = m.noise_loglike(n, R, s_n, s_l, seed)
    np.testing.assert_allclose(got, ref, rtol=1e-9)


def pin_quantile(m):
    rng = np.random.default_rng(1)
    ref = rng.normal(size=1000)
    srt = np.sort(ref)
    assert m.quantile(ref, [srt[0] - 1.0])[0] == 0.0
    assert m.quantile(ref, [srt[-1]])[0] == 1.0
    k = np.array([0, 9, 499, 998])
    np.testing.assert_array_equal(m.quantile(ref, srt[k]), (k + 1) / 1000.0)
    # ties count as "at or below"
    np.testing.assert_array_equal(m.quantile([1.0, 1.0, 2.0, 3.0], [1.0, 0.5, 2.5]),
                                  [0.5, 0.0, 0.75])


PINS = [pin_philox, pin_layout, pin_normals, pin_chi2, pin_likelihood, pin_quantile]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(nz)


def test_likelihood_identity_time_integrated():
    pin_likelihood(nz, T=1)


# Plausible mistakes, each planted into a copy of the oracle's source.
MUTANTS = {
    "philox multiplier": ("PHILOX_M0 = 0xD2511F53", "PHILOX_M0 = 0xD2511F55"),
    "Weyl increment": ("PHILOX_W1 = 0xBB67AE85", "PHILOX_W1 = 0xBB67AE87"),
    "key bumped before the first round": ("        if rnd:\n", "        if True:\n"),
    "nine rounds": ("PHILOX_ROUNDS = 10", "PHILOX_ROUNDS = 9"),
    "round outputs swapped": ("(hi1 ^ c1 ^ np.uint32(k0), lo1,", "(lo1, hi1 ^ c1 ^ np.uint32(k0),"),
    "realisation in the wrong counter word": ("ctr[:, 1] = np.uint32(r)", "ctr[:, 2] = np.uint32(r)"),
    "no tag word": ("ctr[:, 3] = np.uint32(NOISE_TAG)", "ctr[:, 3] = np.uint32(0)"),
    "seed high word dropped": ("(seed >> 32) & MASK32)", "0)"),
    "one stream for u1 and u2": ("ctr[:, 2] = np.uint32(1)", "ctr[:, 2] = np.uint32(0)"),
    "cosine for both normals": ("rho * np.sin(ang)", "rho * np.cos(ang)"),
    "u2 from the u1 words": ("u2 = v.astype", "u2 = w.astype"),
    "u1 scale": ("+ 1.0) * scale", "+ 1.0) * scale * 2.0"),
    "normalisation without the half": ("norm = 0.5 * n * math.log", "norm = n * math.log"),
    "quadratic term without the 2": ("/ (2.0 * sigma_like * sigma_like)", "/ (sigma_like * sigma_like)"),
    "noise scaled by sigma_like": ("e = sigma_noise * normals", "e = sigma_like * normals"),
    "strict quantile": ("ref <= x", "ref < x"),
}


def _mutant(old, new):
    src = open(nz.__file__).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("noise_mutant")
    exec(compile(src.replace(old, new), "noise_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_every_planted_mistake_is_caught(name):
    mod = _mutant(*MUTANTS[name])
    caught = []
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except (AssertionError, ValueError, FloatingPointError):
            caught.append(pin.__name__)
    assert caught, f"no pin catches: {name}"
