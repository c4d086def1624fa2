"""The batched nested slice sampler on problems with known answers (CPU).

Gaussian likelihoods inside a uniform box have an analytic evidence; the
sampler's log Z must fall within a few of its own error estimates of it,
and its posterior moments must match the Gaussian's.  The slice chains must
sample the constrained prior uniformly, and the volume bookkeeping must be
Eq. log_xgpu's.
"""
import math

import numpy as np
from scipy import stats

from paper_2603_13196_amd import sampler as ns


def _gauss(mu, cov):
    mu = np.asarray(mu, dtype=np.float64)
    icov = np.linalg.inv(cov)
    logdet = np.linalg.slogdet(cov)[1]
    d = mu.size

    def f(z):
        x = z - mu
        return -0.5 * np.einsum("bi,ij,bj->b", x, icov, x) - 0.5 * (d * math.log(2 * math.pi) + logdet)
    return f


def flat_model_evidence(S: float, n: int, a: float, b: float) -> float:
    """ln Z of the foreground model with zero responses and no 21-cm term:
    the model is T_CMB, so with s = ln sigma uniform on [a, b] and the
    spectral indices integrating to one,
      lnL(s) = -S e^(-2s) / 2 - n s - (n/2) ln(2 pi),  S = sum (D - T_CMB)^2,
      Z = (1 / (b - a)) int_a^b exp(lnL(s)) ds.
    With u = S e^(-2s) / 2 the integral is a gamma integral:
      int_a^b e^(-S e^(-2s)/2 - n s) ds
        = (1/2) (2/S)^(n/2) Gamma(n/2) [P(n/2, u(a)) - P(n/2, u(b))],
    P the regularised lower incomplete gamma function."""
    from scipy import special
    h = 0.5 * n
    ua, ub = 0.5 * S * math.exp(-2.0 * a), 0.5 * S * math.exp(-2.0 * b)
    mass = special.gammainc(h, ua) - special.gammainc(h, ub)
    return (math.log(0.5) + h * math.log(2.0 / S) + special.gammaln(h) + math.log(mass)
            - h * math.log(2.0 * math.pi) - math.log(b - a))


def flat_model_data(N=3, F=11, T=4, seed=31, t_cmb=2.725):
    """(K = 0 [N, F, T], freqs, data = T_CMB + 25 mK noise, t_cmb)."""
    freqs = np.linspace(60.0, 190.0, F)
    rng = np.random.Generator(np.random.PCG64(seed))
    data = t_cmb + rng.normal(0.0, 0.025, size=(F, T))
    return np.zeros((N, F, T), dtype=np.float32), freqs, data, t_cmb


def test_flat_model_evidence_closed_form():
    """The gamma-integral form against direct quadrature of the integral."""
    from scipy import integrate
    _, _, data, t_cmb = flat_model_data()
    S, n = float(np.sum((data - t_cmb) ** 2)), data.size
    a, b = math.log(1e-3), math.log(0.1)

    def lnl(s):
        return -0.5 * S * math.exp(-2.0 * s) - n * s - 0.5 * n * math.log(2.0 * math.pi)

    sp = 0.5 * math.log(S / n)
    val, _ = integrate.quad(lambda s: math.exp(lnl(s) - lnl(sp)), a, b, points=[sp],
                            epsabs=0.0, epsrel=1e-12, limit=200)
    quad = lnl(sp) + math.log(val) - math.log(b - a)
    assert abs(flat_model_evidence(S, n, a, b) - quad) < 1e-9


def test_sampler_on_oracle_reaches_flat_model_evidence():
    """The host sampler driven by the FP64 oracle's likelihood on the model
    with zero responses (where the oracle reduces to the constant model
    T_CMB) reaches the closed-form evidence."""
    import oracle
    orc = oracle.load()
    K, freqs, data, t_cmb = flat_model_data()
    lo, hi = ns.foreground_box(K.shape[0], no21=True)
    S = float(np.sum((data - t_cmb) ** 2))
    # the oracle's lnL is the closed form's lnL(s) on any row
    rng = np.random.Generator(np.random.PCG64(4))
    z = lo + (hi - lo) * rng.random((50, lo.size))
    want = (-0.5 * S * np.exp(-2.0 * z[:, -1]) - data.size * z[:, -1]
            - 0.5 * data.size * math.log(2.0 * math.pi))
    got = orc.loglike(K, freqs, data, 100.0, t_cmb, ns.to_theta(z), flags=1)
    assert np.allclose(got, want, rtol=1e-12, atol=0.0)
    r = ns.nested_slice_sampling(
        lambda q: orc.loglike(K, freqs, data, 100.0, t_cmb, ns.to_theta(q), flags=1),
        lo, hi, n_live=200, num_delete=40, num_inner_steps=2 * lo.size, seed=5)
    exact = flat_model_evidence(S, data.size, lo[-1], hi[-1])
    assert abs(r.logz - exact) < 3 * r.logz_err, (r.logz, exact, r.logz_err)


def test_logx_decrement_is_eq_log_xgpu():
    for n, b in ((100, 1), (400, 80), (1000, 200)):
        s = ns.expected_logx_decrement(n, b)
        assert abs(s + sum(1.0 / (n - i) for i in range(b))) < 1e-15
        # the closed-form approximation of the paper
        assert abs(s - math.log((n - b) / n)) < 1.5 * b / n ** 2 + 1e-12
    assert ns.expected_logx_decrement(10, 1) == -0.1


def test_gaussian_evidence_and_moments():
    d, half = 4, 2.0
    mu = np.array([0.3, -0.2, 0.1, 0.5])
    cov = np.diag([0.1, 0.2, 0.15, 0.1]) ** 2
    lo, hi = -half * np.ones(d), half * np.ones(d)
    truth = -d * math.log(2 * half)           # Gaussian mass inside the box ~ 1
    r = ns.nested_slice_sampling(_gauss(mu, cov), lo, hi, n_live=300, num_delete=60,
                                 num_inner_steps=4 * d, seed=1)
    assert abs(r.logz - truth) < 4 * r.logz_err + 0.05, (r.logz, truth, r.logz_err)
    m = r.posterior_mean()
    c = r.posterior_cov()
    assert np.all(np.abs(m - mu) < 0.25 * np.sqrt(np.diag(cov)) + 0.01), (m, mu)
    assert np.all(np.abs(np.sqrt(np.diag(c)) / np.sqrt(np.diag(cov)) - 1) < 0.2), np.diag(c)
    # posterior median of lnL = c - chi2_d median / 2 (Sec. 5 accuracy criterion input)
    c = -0.5 * (d * math.log(2 * math.pi) + np.linalg.slogdet(cov)[1])
    med = c - 0.5 * stats.chi2(d).median()
    assert abs(r.median_loglike() - med) < 0.3, (r.median_loglike(), med)
    assert r.sample_logl.shape == (r.samples.shape[0],)
    # the recorded volume follows the expected contraction
    assert abs(r.logx[0] - ns.expected_logx_decrement(300, 60)) < 1e-12
    assert abs(r.logx[-1] - r.iterations * ns.expected_logx_decrement(300, 60)) < 1e-9


def test_correlated_gaussian_uses_whitening():
    d = 3
    rho = 0.95
    cov = 0.05 ** 2 * (rho * np.ones((d, d)) + (1 - rho) * np.eye(d))
    mu = np.zeros(d)
    lo, hi = -np.ones(d), np.ones(d)
    truth = -d * math.log(2.0)
    r = ns.nested_slice_sampling(_gauss(mu, cov), lo, hi, n_live=250, num_delete=50,
                                 num_inner_steps=5 * d, seed=7)
    assert abs(r.logz - truth) < 4 * r.logz_err + 0.05, (r.logz, truth, r.logz_err)
    c = r.posterior_cov()
    corr = c[0, 1] / math.sqrt(c[0, 0] * c[1, 1])
    assert abs(corr - rho) < 0.05, corr


def test_slice_chains_sample_the_constrained_prior_uniformly():
    """Inside lnL = -|x|^2 > -1 within a large box the constrained prior is
    the unit ball: the volume fraction |x|^d of the chain endpoints must be
    uniform on [0, 1]."""
    d, m = 3, 4000
    rng = np.random.Generator(np.random.PCG64(3))
    like = ns._Counter(lambda z: -np.sum(z * z, axis=1))
    x0 = rng.normal(size=(m, d))
    x0 = 0.5 * x0 / np.linalg.norm(x0, axis=1, keepdims=True)       # start inside
    l0 = like(x0)
    x, lx = ns._slice_chains(like, x0, l0, -1.0, -3 * np.ones(d), 3 * np.ones(d),
                             np.eye(d) * 0.7, steps=6, rng=rng)
    assert np.all(lx > -1.0)
    u = np.linalg.norm(x, axis=1) ** d
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # and the directions are isotropic: each coordinate's sign is a fair coin
    assert np.all(np.abs((x > 0).mean(0) - 0.5) < 0.05)


def test_reproducible_from_seed():
    f = _gauss(np.zeros(2), 0.2 ** 2 * np.eye(2))
    kw = dict(n_live=60, num_delete=12, num_inner_steps=6, seed=5)
    a = ns.nested_slice_sampling(f, -np.ones(2), np.ones(2), **kw)
    b = ns.nested_slice_sampling(f, -np.ones(2), np.ones(2), **kw)
    assert a.logz == b.logz and a.n_like == b.n_like
    assert np.array_equal(a.samples, b.samples)


def test_foreground_box_and_transform():
    lo, hi = ns.foreground_box(3)
    assert lo.size == hi.size == 3 + 4
    z = np.array([[2.5, 2.6, 2.7, -0.1, 80.0, 15.0, math.log(0.025)]])
    th = ns.to_theta(z)
    assert abs(th[0, -1] - 0.025) < 1e-15 and np.array_equal(th[0, :-1], z[0, :-1])
    lo2, hi2 = ns.foreground_box(3, no21=True)
    assert lo2.size == 4
