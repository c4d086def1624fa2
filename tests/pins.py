"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` takes an oracle object (``oracle.Oracle``) and raises
AssertionError when the oracle disagrees.  They are used twice: on the real
oracle (tests/test_oracle_pins.py) and on copies of it with a planted mistake
(tests/test_oracle_mutants.py), where at least one pin must fail.

None of these compares the oracle with a retyping of its own formula in the
same precision: the references are 50-digit mpmath evaluations of the
paper's equations, exact floating-point identities, scipy's Gaussian
log-density, and structural properties of the model (region permutation
symmetry and the strict nesting of Sec. 4).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np
from scipy import stats

NO_21CM = 1
mp.mp.dps = 50


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _rand_problem(rng, N, F, T, lo=50.0, hi=200.0):
    K = rng.lognormal(math.log(10.0), 0.7, size=(N, F, T)).astype(np.float32)
    freqs = np.sort(rng.uniform(lo, hi, size=F))
    return K, freqs


def _rand_theta(rng, N, B=1):
    th = np.empty((B, N + 4))
    th[:, :N] = rng.uniform(2.0, 3.5, size=(B, N))
    th[:, N] = rng.uniform(-0.5, 0.0, size=B)
    th[:, N + 1] = rng.uniform(50, 200, size=B)
    th[:, N + 2] = rng.uniform(5, 40, size=B)
    th[:, N + 3] = np.exp(rng.uniform(math.log(1e-3), math.log(0.1), size=B))
    return th


def mp_model(K, freqs, nu_ref, t_cmb, th, no21=False):
    """50-digit evaluation of Eqs. fast_forward_model and t21model."""
    N, F, T = K.shape
    beta = [mp.mpf(float(b)) for b in th[:N]]
    out = [[None] * T for _ in range(F)]
    for f in range(F):
        nu = mp.mpf(float(freqs[f]))
        x = nu / mp.mpf(float(nu_ref))
        p = [mp.power(x, -b) for b in beta]
        s21 = mp.mpf(0)
        if not no21:
            A, nu0, w = (mp.mpf(float(v)) for v in th[N:N + 3])
            s21 = A * mp.exp(-(nu - nu0) ** 2 / (2 * w * w))
        for t in range(T):
            acc = mp.mpf(0)
            for i in range(N):
                acc += mp.mpf(float(K[i, f, t])) * p[i]
            out[f][t] = acc + mp.mpf(float(t_cmb)) + s21
    return out


def mp_loglike(K, freqs, D, nu_ref, t_cmb, th, no21=False):
    """50-digit evaluation of Eq. likelihood."""
    N, F, T = K.shape
    m = mp_model(K, freqs, nu_ref, t_cmb, th, no21)
    sig = mp.mpf(float(th[-1]))
    chi2 = mp.mpf(0)
    for f in range(F):
        for t in range(T):
            r = mp.mpf(float(D[f, t])) - m[f][t]
            chi2 += r * r
    n = F * T
    return -chi2 / (2 * sig * sig) - mp.mpf(n) / 2 * mp.log(2 * mp.pi * sig * sig)


def _relerr(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


# ---------------------------------------------------------------------------

def pin_brute_force(orc, seeds=range(6)):
    """Tiny random problems (N<=3, F<=4, T<=3) against 50-digit mpmath:
    relative error of lnL <= 1e-13 and of every model value <= 1e-14."""
    for s in seeds:
        rng = _rng(100 + s)
        N, F, T = int(rng.integers(1, 4)), int(rng.integers(1, 5)), int(rng.integers(1, 4))
        K, freqs = _rand_problem(rng, N, F, T)
        th = _rand_theta(rng, N, 3)
        D = rng.normal(30.0, 10.0, size=(F, T))
        got = orc.loglike(K, freqs, D, 230.0, 2.725, th)
        for b in range(3):
            ref = mp_loglike(K, freqs, D, 230.0, 2.725, th[b])
            assert _relerr(got[b], ref) <= 1e-13, (s, b, got[b], float(ref))
            m = orc.model(K, freqs, 230.0, 2.725, th[b])
            mref = mp_model(K, freqs, 230.0, 2.725, th[b])
            for f in range(F):
                for t in range(T):
                    assert _relerr(m[f, t], mref[f][t]) <= 1e-14, (s, f, t)


def pin_n1_closed_form(orc):
    """N = 1: M = c (nu/nu_ref)^(-beta) + T_CMB + A exp(-(nu-nu0)^2/(2w^2)),
    checked value by value against mpmath on a 151-channel band, T = 2."""
    rng = _rng(7)
    freqs = np.linspace(50.0, 200.0, 151)
    c = np.float32(123.25)
    K = np.full((1, 151, 2), c, dtype=np.float32)
    K[0, :, 1] = np.float32(0.5)
    th = np.array([2.71, -0.2, 95.0, 12.5, 0.03])
    m = orc.model(K, freqs, 230.0, 2.725, th)
    for f in range(0, 151, 10):
        nu = mp.mpf(float(freqs[f]))
        for t, cc in ((0, c), (1, np.float32(0.5))):
            ref = (mp.mpf(float(cc)) * mp.power(nu / 230, -mp.mpf("2.71")) + mp.mpf("2.725")
                   + mp.mpf("-0.2") * mp.exp(-(nu - 95) ** 2 / (2 * mp.mpf("12.5") ** 2)))
            assert _relerr(m[f, t], ref) <= 1e-14, (f, t)


def pin_unit_power(orc):
    """beta = 0, or nu = nu_ref: every power is exactly one, so the
    foreground is the plain region sum of K (exactly summed with fsum, then
    rounded) and M = sum_i K + T_CMB."""
    rng = _rng(11)
    N, F, T = 5, 7, 3
    K, freqs = _rand_problem(rng, N, F, T)
    th = np.zeros(N + 1)
    th[-1] = 0.1
    m = orc.model(K, freqs, 230.0, 2.725, th, flags=NO_21CM)
    for f in range(F):
        for t in range(T):
            s = math.fsum([float(K[i, f, t]) for i in range(N)])
            assert abs(m[f, t] - (s + 2.725)) <= 4e-16 * (s + 2.725) * N, (f, t)
    th2 = np.concatenate([rng.uniform(2, 3.5, N), [0.1]])
    m2 = orc.model(K, np.full(F, 230.0), 230.0, 2.725, th2, flags=NO_21CM)
    for f in range(F):
        for t in range(T):
            s = math.fsum([float(K[i, f, t]) for i in range(N)])
            assert abs(m2[f, t] - (s + 2.725)) <= 4e-16 * (s + 2.725) * N


def pin_t21_profile(orc):
    """K = 0: M = T_CMB + A exp(-(nu-nu0)^2/(2 w^2)) (Eq. t21model): at
    nu = nu0 the profile is A; at nu0 +- w it is A e^(-1/2); at nu0 +- 2w it
    is A e^(-2); the sign of A is kept."""
    freqs = np.array([60.0, 70.0, 80.0, 90.0, 100.0])
    K = np.zeros((2, 5, 1), dtype=np.float32)
    th = np.array([2.5, 3.0, -0.25, 80.0, 10.0, 0.05])
    m = orc.model(K, freqs, 230.0, 2.725, th)[:, 0] - 2.725
    want = -0.25 * np.exp(-0.5 * np.array([4.0, 1.0, 0.0, 1.0, 4.0]))
    assert np.allclose(m, want, rtol=1e-14, atol=1e-16), (m, want)


def pin_linearity(orc):
    """The foreground is linear in K: with T_CMB = 0 and no 21-cm term,
    doubling K doubles M exactly (every operation scales by two), and
    M(K1 + K2) = M(K1) + M(K2) to rounding for K1, K2 whose FP32 sum is
    exact."""
    rng = _rng(13)
    N, F, T = 4, 9, 5
    K, freqs = _rand_problem(rng, N, F, T)
    th = np.concatenate([rng.uniform(2, 3.5, N), [0.05]])
    m1 = orc.model(K, freqs, 230.0, 0.0, th, flags=NO_21CM)
    m2 = orc.model(2 * K, freqs, 230.0, 0.0, th, flags=NO_21CM)
    assert np.array_equal(m2, 2 * m1)
    Ka = rng.integers(1, 4096, size=(N, F, T)).astype(np.float32)
    Kb = rng.integers(1, 4096, size=(N, F, T)).astype(np.float32)
    ma = orc.model(Ka, freqs, 230.0, 0.0, th, flags=NO_21CM)
    mb = orc.model(Kb, freqs, 230.0, 0.0, th, flags=NO_21CM)
    mab = orc.model(Ka + Kb, freqs, 230.0, 0.0, th, flags=NO_21CM)
    assert np.allclose(mab, ma + mb, rtol=1e-14, atol=0)


def pin_permutation(orc):
    """Relabelling the regions (K and beta permuted together) leaves M and
    lnL unchanged up to the rounding of the reordered region sum."""
    rng = _rng(17)
    N, F, T = 6, 11, 4
    K, freqs = _rand_problem(rng, N, F, T)
    th = _rand_theta(rng, N, 4)
    D = rng.normal(200.0, 50.0, size=(F, T))
    perm = rng.permutation(N)
    Kp = np.ascontiguousarray(K[perm])
    thp = th.copy()
    thp[:, :N] = th[:, perm]
    a = orc.loglike(K, freqs, D, 230.0, 2.725, th)
    b = orc.loglike(Kp, freqs, D, 230.0, 2.725, thp)
    assert np.allclose(a, b, rtol=1e-12, atol=0), (a, b)
    ma = orc.model(K, freqs, 230.0, 2.725, th[0])
    mb = orc.model(Kp, freqs, 230.0, 2.725, thp[0])
    assert np.allclose(ma, mb, rtol=1e-14, atol=0)
    # a permutation that is not applied to beta must change the model
    thq = th[0].copy()
    mc = orc.model(Kp, freqs, 230.0, 2.725, thq)
    assert not np.allclose(ma, mc, rtol=1e-6)


def pin_nesting(orc):
    """Strict nesting (Sec. 4): splitting region j into two regions with
    K/2 each (exact in FP32) and the same spectral index leaves M unchanged
    up to rounding, for every j."""
    rng = _rng(19)
    N, F, T = 4, 13, 3
    K, freqs = _rand_problem(rng, N, F, T)
    th = _rand_theta(rng, N, 1)[0]
    m0 = orc.model(K, freqs, 230.0, 2.725, th)
    for j in range(N):
        Ks = np.concatenate([K[:j], K[j:j + 1] * np.float32(0.5),
                             K[j:j + 1] * np.float32(0.5), K[j + 1:]])
        ths = np.concatenate([th[:j], [th[j], th[j]], th[j + 1:]])
        m1 = orc.model(np.ascontiguousarray(Ks), freqs, 230.0, 2.725, ths)
        assert np.allclose(m1, m0, rtol=2e-15, atol=0), j


def pin_gaussian_library(orc):
    """Eq. likelihood is the textbook Gaussian: lnL equals the sum of
    scipy.stats.norm.logpdf(D, M, sigma), with M taken value by value from
    the 50-digit model."""
    rng = _rng(23)
    N, F, T = 3, 6, 4
    K, freqs = _rand_problem(rng, N, F, T)
    th = _rand_theta(rng, N, 2)
    th[:, -1] = [0.7, 2.5]
    D = rng.normal(100.0, 20.0, size=(F, T))
    got = orc.loglike(K, freqs, D, 230.0, 2.725, th)
    for b in range(2):
        mm = mp_model(K, freqs, 230.0, 2.725, th[b])
        M = np.array([[float(mm[f][t]) for t in range(T)] for f in range(F)])
        ref = math.fsum(stats.norm.logpdf(D, M, th[b, -1]).ravel())
        assert _relerr(got[b], ref) <= 1e-11, (b, got[b], ref)


def pin_noise_free(orc):
    """D = M(theta*) exactly: chi-square is zero, so
    lnL(theta*) = -FT/2 ln(2 pi sigma^2) in closed form; with
    D = M(theta*) + delta, lnL = -FT delta^2/(2 sigma^2) - FT/2 ln(2 pi sigma^2)."""
    rng = _rng(29)
    N, F, T = 5, 17, 6
    K, freqs = _rand_problem(rng, N, F, T)
    th = _rand_theta(rng, N, 1)[0]
    th[-1] = 0.025
    D = orc.model(K, freqs, 230.0, 2.725, th)
    got = orc.loglike(K, freqs, D, 230.0, 2.725, th[None])[0]
    n = F * T
    ref = -0.5 * n * float(mp.log(2 * mp.pi * mp.mpf("0.025") ** 2))
    assert _relerr(got, ref) <= 1e-14, (got, ref)
    delta = 0.01
    got2 = orc.loglike(K, freqs, D + delta, 230.0, 2.725, th[None])[0]
    ref2 = -n * delta ** 2 / (2 * 0.025 ** 2) + ref
    assert _relerr(got2, ref2) <= 1e-9, (got2, ref2)


def pin_invalid_rows(orc):
    """Rows with sigma <= 0, w <= 0 or a non-finite entry give -inf; the
    other rows of the same batch are unaffected; without the 21-cm term
    the width is not a parameter."""
    rng = _rng(31)
    N, F, T = 2, 5, 2
    K, freqs = _rand_problem(rng, N, F, T)
    D = rng.normal(50.0, 5.0, size=(F, T))
    th = _rand_theta(rng, N, 6)
    th[1, -1] = 0.0
    th[2, N + 2] = -1.0
    th[3, 0] = np.nan
    th[4, N] = np.inf
    got = orc.loglike(K, freqs, D, 230.0, 2.725, th)
    assert np.isfinite(got[0]) and np.isfinite(got[5])
    assert np.all(got[1:5] == -np.inf), got
    ok = orc.loglike(K, freqs, D, 230.0, 2.725, th[[0, 5]])
    assert np.array_equal(ok, got[[0, 5]])
    th2 = np.array([[2.5, 2.6, 0.1]])
    assert np.isfinite(orc.loglike(K, freqs, D, 230.0, 2.725, th2, flags=NO_21CM)[0])
    # spectral indices are valid up to |beta| = 64 inclusive
    th3 = np.repeat(th[:1], 3, axis=0)
    th3[0, 0] = 64.0
    th3[1, 1] = -64.0
    th3[2, 0] = 64.0 + 1e-9
    got3 = orc.loglike(K, freqs, D, 230.0, 2.725, th3)
    assert np.all(np.isfinite(got3[:2])) and got3[2] == -np.inf, got3


def pin_batch_rows(orc):
    """Rows are independent: permuting the batch permutes the output
    exactly, and one row alone equals the same row inside a batch."""
    rng = _rng(37)
    N, F, T = 3, 8, 3
    K, freqs = _rand_problem(rng, N, F, T)
    D = rng.normal(80.0, 10.0, size=(F, T))
    th = _rand_theta(rng, N, 9)
    a = orc.loglike(K, freqs, D, 230.0, 2.725, th)
    p = rng.permutation(9)
    b = orc.loglike(K, freqs, D, 230.0, 2.725, th[p])
    assert np.array_equal(a[p], b)
    c = orc.loglike(K, freqs, D, 230.0, 2.725, th[4:5], threads=1)
    assert c[0] == a[4]


# ---------------------------------------------------------------------------
# amplitude masks crossed with spectral-index masks (Eq. fast_forward_model
# with n_alpha > 0): K [n_alpha, n_beta, F, T], rows
# [beta_0.., alpha_0.., A, nu21, w, sigma]

def _rand_theta_masks(rng, NA, NB, B=1, alo=0.5, ahi=2.0):
    th = np.empty((B, NB + NA + 4))
    th[:, :NB] = rng.uniform(2.0, 3.5, size=(B, NB))
    th[:, NB:NB + NA] = rng.uniform(alo, ahi, size=(B, NA))
    th[:, NB + NA] = rng.uniform(-0.5, 0.0, size=B)
    th[:, NB + NA + 1] = rng.uniform(50, 200, size=B)
    th[:, NB + NA + 2] = rng.uniform(5, 40, size=B)
    th[:, NB + NA + 3] = np.exp(rng.uniform(math.log(1e-3), math.log(0.1), size=B))
    return th


def mp_model_masks(K4, freqs, nu_ref, t_cmb, th):
    """50-digit evaluation of Eq. fast_forward_model with both mask sets,
    plus Eq. t21model."""
    NA, NB, F, T = K4.shape
    beta = [mp.mpf(float(b)) for b in th[:NB]]
    alpha = [mp.mpf(float(a)) for a in th[NB:NB + NA]]
    A, nu0, w = (mp.mpf(float(v)) for v in th[NB + NA:NB + NA + 3])
    out = [[None] * T for _ in range(F)]
    for f in range(F):
        nu = mp.mpf(float(freqs[f]))
        x = nu / mp.mpf(float(nu_ref))
        p = [mp.power(x, -b) for b in beta]
        s21 = A * mp.exp(-(nu - nu0) ** 2 / (2 * w * w))
        for t in range(T):
            acc = mp.mpf(0)
            for i in range(NA):
                for j in range(NB):
                    acc += alpha[i] * mp.mpf(float(K4[i, j, f, t])) * p[j]
            out[f][t] = acc + mp.mpf(float(t_cmb)) + s21
    return out


def pin_masks_brute_force(orc, seeds=range(5)):
    """Tiny problems with 1-3 amplitude masks and 1-3 spectral-index masks
    against 50-digit mpmath: lnL to 1e-13 and every model value to 1e-14
    relative."""
    for s in seeds:
        rng = _rng(300 + s)
        NA, NB = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        F, T = int(rng.integers(1, 5)), int(rng.integers(1, 4))
        K, freqs = _rand_problem(rng, NA * NB, F, T)
        K4 = K.reshape(NA, NB, F, T)
        th = _rand_theta_masks(rng, NA, NB, 3)
        D = rng.normal(40.0, 10.0, size=(F, T))
        got = orc.loglike_masks(K4, freqs, D, 230.0, 2.725, th)
        for b in range(3):
            mm = mp_model_masks(K4, freqs, 230.0, 2.725, th[b])
            sig = mp.mpf(float(th[b, -1]))
            chi2 = mp.mpf(0)
            for f in range(F):
                for t in range(T):
                    r = mp.mpf(float(D[f, t])) - mm[f][t]
                    chi2 += r * r
            ref = -chi2 / (2 * sig * sig) - mp.mpf(F * T) / 2 * mp.log(2 * mp.pi * sig * sig)
            assert _relerr(got[b], ref) <= 1e-13, (s, b, got[b], float(ref))
            m = orc.model_masks(K4, freqs, 230.0, 2.725, th[b])
            for f in range(F):
                for t in range(T):
                    assert _relerr(m[f, t], mm[f][t]) <= 1e-14, (s, f, t)


def pin_masks_power_of_two_alpha(orc):
    """With every alpha_i a power of two, alpha_i K_ij is exact in FP32, so
    the crossed model equals, bit for bit, the spectral-index-only model
    whose region (i, j) has response alpha_i K_ij and index beta_j."""
    rng = _rng(41)
    NA, NB, F, T = 3, 4, 9, 5
    K, freqs = _rand_problem(rng, NA * NB, F, T)
    K4 = K.reshape(NA, NB, F, T)
    th = _rand_theta_masks(rng, NA, NB, 6)
    th[:, NB:NB + NA] = 2.0 ** rng.integers(-3, 4, size=(6, NA))
    D = rng.normal(150.0, 30.0, size=(F, T))
    got = orc.loglike_masks(K4, freqs, D, 230.0, 2.725, th)
    for b in range(6):
        a = th[b, NB:NB + NA]
        Kf = np.ascontiguousarray((K4 * a[:, None, None, None].astype(np.float32))
                                  .reshape(NA * NB, F, T))
        thf = np.concatenate([np.tile(th[b, :NB], NA), th[b, NB + NA:]])
        ref = orc.loglike(Kf, freqs, D, 230.0, 2.725, thf[None])[0]
        assert got[b] == ref, (b, got[b], ref)
        assert np.array_equal(orc.model_masks(K4, freqs, 230.0, 2.725, th[b]),
                              orc.model(Kf, freqs, 230.0, 2.725, thf))


def pin_masks_unit_power(orc):
    """beta = 0: every power is one, so M = sum_i alpha_i sum_j K_ij + T_CMB
    (summed exactly with fsum, then rounded)."""
    rng = _rng(43)
    NA, NB, F, T = 3, 2, 6, 3
    K, freqs = _rand_problem(rng, NA * NB, F, T)
    K4 = K.reshape(NA, NB, F, T)
    th = np.zeros(NB + NA + 1)
    th[NB:NB + NA] = [0.75, 1.3, 2.2]
    th[-1] = 0.1
    m = orc.model_masks(K4, freqs, 230.0, 2.725, th, flags=NO_21CM)
    for f in range(F):
        for t in range(T):
            terms = [th[NB + i] * float(K4[i, j, f, t]) for i in range(NA) for j in range(NB)]
            s = math.fsum(terms) + 2.725
            assert abs(m[f, t] - s) <= 4e-16 * s * NA * NB, (f, t, m[f, t], s)


def pin_masks_nesting(orc):
    """Strict nesting in both mask sets: splitting an amplitude mask into
    two with K/2 each and the same alpha, or a spectral-index mask into two
    with K/2 each and the same beta, leaves M unchanged up to rounding."""
    rng = _rng(47)
    NA, NB, F, T = 2, 3, 7, 2
    K, freqs = _rand_problem(rng, NA * NB, F, T)
    K4 = K.reshape(NA, NB, F, T)
    th = _rand_theta_masks(rng, NA, NB, 1)[0]
    beta, alpha, rest = th[:NB], th[NB:NB + NA], th[NB + NA:]
    m0 = orc.model_masks(K4, freqs, 230.0, 2.725, th)
    h = np.float32(0.5)
    for i in range(NA):
        Ks = np.concatenate([K4[:i], K4[i:i + 1] * h, K4[i:i + 1] * h, K4[i + 1:]])
        ths = np.concatenate([beta, alpha[:i], [alpha[i], alpha[i]], alpha[i + 1:], rest])
        m1 = orc.model_masks(np.ascontiguousarray(Ks), freqs, 230.0, 2.725, ths)
        assert np.allclose(m1, m0, rtol=2e-15, atol=0), ("alpha", i)
    for j in range(NB):
        Ks = np.concatenate([K4[:, :j], K4[:, j:j + 1] * h, K4[:, j:j + 1] * h,
                             K4[:, j + 1:]], axis=1)
        ths = np.concatenate([beta[:j], [beta[j], beta[j]], beta[j + 1:], alpha, rest])
        m1 = orc.model_masks(np.ascontiguousarray(Ks), freqs, 230.0, 2.725, ths)
        assert np.allclose(m1, m0, rtol=2e-15, atol=0), ("beta", j)


def pin_masks_invalid_alpha(orc):
    """An amplitude scale outside [2^-32, 2^32] (zero and negative included)
    makes the row -inf; the bounds themselves are valid."""
    rng = _rng(53)
    NA, NB, F, T = 2, 2, 4, 2
    K, freqs = _rand_problem(rng, NA * NB, F, T)
    K4 = K.reshape(NA, NB, F, T)
    D = rng.normal(50.0, 5.0, size=(F, T))
    th = _rand_theta_masks(rng, NA, NB, 7)
    bad = [0.0, -1.0, 2.0 ** 33, 2.0 ** -33]
    for r, v in enumerate(bad):
        th[r + 1, NB + (r % NA)] = v
    th[5, NB] = 2.0 ** 32
    th[6, NB + 1] = 2.0 ** -32
    got = orc.loglike_masks(K4, freqs, D, 230.0, 2.725, th)
    assert np.all(got[1:5] == -np.inf), got
    assert np.all(np.isfinite(got[[0, 5, 6]])), got


# ---------------------------------------------------------------------------
# gradient of lnL with respect to the row's parameters

def _mp_lnl_any(K4, freqs, D, nu_ref, t_cmb, th, NA):
    """50-digit lnL of either model at a row given as mpf values."""
    NAa, NB, F, T = K4.shape
    beta = th[:NB]
    alpha = th[NB:NB + NA] if NA else [mp.mpf(1)]
    A, nu0, w, sig = th[-4], th[-3], th[-2], th[-1]
    chi2 = mp.mpf(0)
    for f in range(F):
        nu = mp.mpf(float(freqs[f]))
        x = nu / mp.mpf(float(nu_ref))
        p = [mp.power(x, -b) for b in beta]
        s21 = A * mp.exp(-(nu - nu0) ** 2 / (2 * w * w))
        for t in range(T):
            acc = mp.mpf(0)
            for i in range(NAa):
                for j in range(NB):
                    acc += alpha[i] * mp.mpf(float(K4[i, j, f, t])) * p[j]
            r = mp.mpf(float(D[f, t])) - (acc + mp.mpf(float(t_cmb)) + s21)
            chi2 += r * r
    return -chi2 / (2 * sig * sig) - mp.mpf(F * T) / 2 * mp.log(2 * mp.pi * sig * sig)


def _mp_grad(K4, freqs, D, nu_ref, t_cmb, row, NA):
    """Central differences of the 50-digit lnL with step 1e-18 (truncation
    ~1e-36, rounding ~1e-32 relative): the gradient to ~25 digits."""
    th = [mp.mpf(float(v)) for v in row]
    h = mp.mpf("1e-18")
    out = []
    for k in range(len(th)):
        tp = list(th)
        tm = list(th)
        tp[k] += h
        tm[k] -= h
        out.append((_mp_lnl_any(K4, freqs, D, nu_ref, t_cmb, tp, NA)
                    - _mp_lnl_any(K4, freqs, D, nu_ref, t_cmb, tm, NA)) / (2 * h))
    return out


def pin_grad_brute_force(orc, seeds=range(4)):
    """The oracle's analytic gradient against central differences of the
    50-digit lnL, for spectral-index-only and crossed-mask problems, to
    1e-11 relative to the largest gradient entry's magnitude scale (the
    entries are sums of terms of both signs)."""
    for s in seeds:
        rng = _rng(500 + s)
        NA = int(s % 2) * int(rng.integers(1, 3))          # 0 (index only) or 1-2
        NB = int(rng.integers(1, 4))
        F, T = int(rng.integers(2, 5)), int(rng.integers(1, 4))
        N = max(NA, 1) * NB
        K, freqs = _rand_problem(rng, N, F, T)
        K4 = K.reshape(max(NA, 1), NB, F, T)
        if NA:
            th = _rand_theta_masks(rng, NA, NB, 2)
        else:
            th = _rand_theta(rng, NB, 2)
        th[:, -1] = [0.3, 2.0]
        D = rng.normal(60.0, 15.0, size=(F, T))
        ll, g = orc.grad(K, freqs, D, 230.0, 2.725, th, n_alpha=NA)
        ref_ll = orc.loglike_masks(K4, freqs, D, 230.0, 2.725, th) if NA else \
            orc.loglike(K, freqs, D, 230.0, 2.725, th)
        assert np.array_equal(ll, ref_ll), (s, ll, ref_ll)
        for b in range(2):
            ref = _mp_grad(K4, freqs, D, 230.0, 2.725, th[b], NA)
            for k, rk in enumerate(ref):
                assert abs(g[b, k] - float(rk)) <= 1e-11 * max(abs(float(rk)), 1e-6), \
                    (s, b, k, g[b, k], float(rk))


def pin_grad_noise_free(orc):
    """D = M(theta) exactly (the oracle's own model values): every residual is
    zero, so every derivative but sigma's vanishes exactly and
    dlnL/dsigma = -F T / sigma."""
    rng = _rng(59)
    for NA, NB in ((0, 4), (2, 3)):
        N = max(NA, 1) * NB
        K, freqs = _rand_problem(rng, N, 9, 4)
        K4 = K.reshape(max(NA, 1), NB, 9, 4)
        th = (_rand_theta_masks(rng, NA, NB, 1) if NA else _rand_theta(rng, NB, 1))[0]
        th[-1] = 0.025
        D = orc.model_masks(K4, freqs, 230.0, 2.725, th) if NA else \
            orc.model(K, freqs, 230.0, 2.725, th)
        _, g = orc.grad(K, freqs, D, 230.0, 2.725, th[None], n_alpha=NA)
        assert np.all(g[0, :-1] == 0.0), g
        assert abs(g[0, -1] - (-36 / 0.025)) <= 1e-12 * 36 / 0.025, g[0, -1]


def pin_grad_sigma_closed_form(orc):
    """lnL(sigma) = -chi2/(2 sigma^2) - n ln sigma - (n/2) ln 2 pi with chi2
    independent of sigma: chi2 recovered from lnL at two sigmas gives
    dlnL/dsigma = chi2/sigma^3 - n/sigma, and the other entries do not
    depend on sigma except through the factor 1/sigma^2."""
    rng = _rng(61)
    N, F, T = 3, 7, 5
    K, freqs = _rand_problem(rng, N, F, T)
    D = rng.normal(100.0, 10.0, size=(F, T))
    th = _rand_theta(rng, N, 1)
    th2 = th.copy()
    th[0, -1], th2[0, -1] = 0.5, 1.5
    l1, g1 = orc.grad(K, freqs, D, 230.0, 2.725, th)
    l2, g2 = orc.grad(K, freqs, D, 230.0, 2.725, th2)
    n = F * T
    # l1 - l2 = -chi2/2 (1/0.25 - 1/2.25) - n ln(0.5/1.5)
    chi2 = -(l1[0] - l2[0] + n * math.log(0.5 / 1.5)) / (0.5 * (4.0 - 1.0 / 2.25))
    assert abs(g1[0, -1] - (chi2 / 0.125 - n / 0.5)) <= 1e-9 * chi2 / 0.125
    assert np.allclose(g1[0, :-1] * 0.25, g2[0, :-1] * 2.25, rtol=1e-13, atol=0)


ALL_PINS = [pin_brute_force, pin_n1_closed_form, pin_unit_power,
            pin_t21_profile, pin_linearity, pin_permutation, pin_nesting,
            pin_gaussian_library, pin_noise_free, pin_invalid_rows,
            pin_batch_rows, pin_masks_brute_force, pin_masks_power_of_two_alpha,
            pin_masks_unit_power, pin_masks_nesting, pin_masks_invalid_alpha,
            pin_grad_brute_force, pin_grad_noise_free, pin_grad_sigma_closed_form]
