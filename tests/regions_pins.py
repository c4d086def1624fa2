"""Pins of the region-construction oracle (oracle/regions.py) to facts fixed
by the paper and by mathematics.  Each pin takes the oracle module and
raises AssertionError on disagreement; tests/test_regions_oracle.py runs
them on the real oracle and on copies with planted mistakes."""
from __future__ import annotations

import os

import numpy as np

from workload.sky import Sky, make_sky

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "partition_worked_examples.txt")


def _small(seed=3, nlat=8, nlon=16, F=5, T=4):
    return make_sky(nlat, nlon, np.linspace(50.0, 200.0, F), T, seed=seed)


def _flat(sky, beam=None, horizon=None, t_ex=None, beta=None):
    return Sky(sky.omega, sky.t_ex if t_ex is None else t_ex,
               sky.beta if beta is None else beta,
               sky.beam if beam is None else beam,
               sky.horizon if horizon is None else horizon, sky.freqs, sky.shifts)


def pin_worked_examples(R):
    """Hand-worked partitions of both algorithms (tests/golden)."""
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        head, b, w, e = [x.strip() for x in line.split("|")]
        meth, k = head.split()
        got = R.partition(np.array(b.split(), float), np.array(w.split(), float), int(k), meth)
        assert np.array_equal(got, np.array(e.split(), float)), (line, got)
        n += 1
    assert n == 8


def pin_importance_normalised(R):
    """Each (nu, t) weight integrates to one over the sphere, so the
    importance of all sky pixels sums to T F, for every scheme."""
    s = _small()
    for sch in R.SCHEMES:
        I = R.importance(s, sch)
        assert abs(I.sum() - s.T * s.F) <= 1e-12 * s.T * s.F, (sch, I.sum())
        assert np.all(I >= 0)


def pin_importance_uniform_sky(R):
    """H = 1 everywhere and a uniform sky: every scheme but the beam one
    gives I(q) = T F omega(q); with a uniform beam too, so does the beam
    scheme."""
    s = _small()
    one = np.ones_like(s.horizon)
    u = _flat(s, beam=np.ones_like(s.beam), horizon=one, t_ex=np.full_like(s.t_ex, 50.0),
              beta=np.full_like(s.beta, 2.7))
    want = s.T * s.F * np.repeat(s.omega[:, None], s.nlon, axis=1) / (s.omega.sum() * s.nlon)
    for sch in R.SCHEMES:
        assert np.allclose(R.importance(u, sch), want, rtol=1e-12, atol=0), sch


def pin_importance_brute_force(R):
    """A 4 x 6 sky over 2 channels and 3 steps, every weight of Sec. 4.2
    evaluated pixel by pixel with plain loops from its definition."""
    s = _small(seed=11, nlat=4, nlon=6, F=2, T=3)
    # a beam that is non-zero below the horizon too, so H matters
    s = Sky(s.omega, s.t_ex, s.beta, (s.beam + np.float32(0.1)).astype(np.float32), s.horizon,
            s.freqs, np.array([0, 2, 5], np.int32))
    assert 0 < s.horizon.sum() < s.horizon.size
    nl, nw = s.nlat, s.nlon
    tsky = lambda r, q, f: s.t_ex[r, q] * (s.freqs[f] / s.nu0) ** (-s.beta[r, q]) + s.t_cmb
    for sch in R.SCHEMES:
        want = np.zeros((nl, nw))
        for t in range(s.T):
            sh = int(s.shifts[t])
            for f in range(s.F):
                def w(r, p):      # weight of local pixel (r, p) before normalising
                    q = (p + sh) % nw
                    v = float(s.horizon[r, p])
                    if sch != "horizon":
                        v *= tsky(r, q, f)
                    if sch == "beam":
                        v *= float(s.beam[f, r, p])
                    return v
                Z = sum(s.omega[r] * w(r, p) for r in range(nl) for p in range(nw))
                for r in range(nl):
                    for q in range(nw):
                        want[r, q] += s.omega[r] * w(r, (q - sh) % nw) / Z
        assert np.allclose(R.importance(s, sch), want, rtol=1e-12, atol=1e-16), sch


def pin_importance_follows_visibility(R):
    """Horizon scheme: a sky pixel's importance is proportional to the
    number of steps it spends above the horizon (the weight is H / int H)."""
    s = _small()
    I = R.importance(s, "horizon")
    vis = sum(np.roll(s.horizon.astype(float), int(sh), axis=1) for sh in s.shifts)
    tot = np.sum(s.omega[:, None] * s.horizon)
    want = s.F * s.omega[:, None] * vis / tot
    assert np.allclose(I, want, rtol=1e-12, atol=1e-15)


def pin_rotation_equivariance(R):
    """Turning the sky maps by c columns and every shift by c turns the
    importance map by c and leaves the chromatic functions unchanged."""
    s = _small()
    c = 5
    r = Sky(s.omega, np.roll(s.t_ex, c, 1), np.roll(s.beta, c, 1), s.beam, s.horizon,
            s.freqs, (s.shifts + c) % s.nlon)
    for sch in R.SCHEMES:
        assert np.allclose(R.importance(r, sch), np.roll(R.importance(s, sch), c, 1),
                           rtol=1e-12, atol=1e-15), sch
    reg = R.masks(s.beta, R.partition(s.beta, R.importance(s, "beam"), 4, "recursive"))
    assert np.allclose(R.chromatic(r, np.roll(reg, c, 1), 4), R.chromatic(s, reg, 4),
                       rtol=1e-12, atol=0)


def pin_cdf(R):
    """C is non-decreasing and ends at one; with equal weights it is the
    empirical distribution k/n of the sorted indices."""
    rng = np.random.Generator(np.random.PCG64(4))
    b = rng.normal(2.8, 0.2, 50)
    xs, cs = R.weighted_cdf(b, rng.random(50))
    assert np.all(np.diff(xs) >= 0) and np.all(np.diff(cs) >= 0) and cs[-1] == 1.0
    xs, cs = R.weighted_cdf(b, np.ones(50))
    assert np.array_equal(xs, np.sort(b))
    assert np.allclose(cs, np.arange(1, 51) / 50, rtol=1e-15)


def pin_nested_partitions(R):
    """The defining property of both schemes (Sec. 4): the partition into
    n + 1 regions refines the one into n (every edge is kept)."""
    s = _small()
    I = R.importance(s, "beam")
    for meth in ("recursive", "hierarchical"):
        prev = None
        for n in range(1, 13):
            e = R.partition(s.beta, I, n, meth)
            assert e.size == n + 1 and np.all(np.diff(e) >= 0), (meth, n)
            if prev is not None and not (meth == "hierarchical" and n & (n - 1) == 0):
                assert set(prev) <= set(e), (meth, n, prev, e)
            prev = e


def pin_recursive_dyadic(R):
    """Recursive edges are spectral-index midpoints: every edge is
    beta_min + k (beta_max - beta_min) / 2^m."""
    s = _small()
    e = R.partition(s.beta, R.importance(s, "sky"), 9, "recursive")
    lo, hi = e[0], e[-1]
    u = (e - lo) / (hi - lo) * 2 ** 10
    assert np.allclose(u, np.round(u), atol=1e-9), u


def pin_hierarchical_equal_mass(R):
    """With a power-of-two count, the hierarchical regions hold equal
    importance up to the weight of single pixels at the edges."""
    s = _small(nlat=16, nlon=32)
    I = R.importance(s, "beam")
    e = R.partition(s.beta, I, 8, "hierarchical")
    reg = R.masks(s.beta, e)
    m = np.array([I[reg == j].sum() for j in range(8)]) / I.sum()
    assert np.all(np.abs(m - 1 / 8) <= 1.01 * I.max() / I.sum()), m


def pin_masks(R):
    """Region j holds e_j <= beta < e_{j+1}, the last region closed; every
    pixel inside [e_0, e_N] belongs to exactly one region."""
    b = np.array([1.0, 1.5, 2.0, 2.5, 3.0])
    assert np.array_equal(R.masks(b, np.array([1.0, 2.0, 3.0])), [0, 0, 1, 1, 1])
    assert np.array_equal(R.masks(b, np.array([1.5, 2.5])), [-1, 0, 0, 0, -1])


def pin_chromatic_closed_forms(R):
    """Eq. chromatic_function: with D = 1, K_j = sum_{q in j} omega T_ex
    for every (nu, t); a one-pixel region gives omega T_ex D(p_t(q), nu);
    the regions add up to the one-region function."""
    s = _small()
    e = R.partition(s.beta, R.importance(s, "beam"), 5, "recursive")
    reg = R.masks(s.beta, e)
    u = _flat(s, beam=np.ones_like(s.beam))
    K = R.chromatic(u, reg, 5)
    for j in range(5):
        want = np.sum((s.omega[:, None] * s.t_ex)[reg == j])
        assert np.allclose(K[j], want, rtol=1e-12), j
    one = np.full_like(reg, -1)
    one[3, 7] = 0
    K1 = R.chromatic(s, one, 1)[0]
    for t, sh in enumerate(s.shifts):
        assert np.allclose(K1[:, t], s.omega[3] * s.t_ex[3, 7] * s.beam[:, 3, (7 - sh) % s.nlon],
                           rtol=1e-13), t
    Kall = R.chromatic(s, np.zeros_like(reg), 1)[0]
    assert np.allclose(R.chromatic(s, reg, 5).sum(axis=0), Kall, rtol=1e-12)


def pin_forward_model_exact_for_piecewise_beta(R):
    """With beta constant on each region, the fast forward model
    sum_j K_j (nu/nu0)^(-beta_j) + T_CMB sum omega D equals the pixel sum
    of Eq. skyapproximation through the beam (Eqs. chromatic_function,
    fast_forward_model)."""
    s = _small()
    e = R.partition(s.beta, R.importance(s, "beam"), 6, "hierarchical")
    reg = R.masks(s.beta, e)
    bj = np.array([2.5 + 0.1 * j for j in range(6)])
    pb = _flat(s, beta=bj[reg])
    K = R.chromatic(pb, reg, 6)
    Ts = R.sky_temperature(pb)
    for t, sh in enumerate(s.shifts):
        Ds = np.roll(s.beam.astype(np.float64), int(sh), axis=-1)
        pix = np.einsum("frq,frq->f", Ts * s.omega[None, :, None], Ds)
        fast = (np.einsum("jf,jf->f", K[:, :, t], (s.freqs[None, :] / s.nu0) ** -bj[:, None])
                + s.t_cmb * np.einsum("frq,r->f", Ds, s.omega))
        assert np.allclose(fast, pix, rtol=1e-12), t


ALL = [pin_worked_examples, pin_importance_normalised, pin_importance_uniform_sky,
       pin_importance_brute_force,
       pin_importance_follows_visibility, pin_rotation_equivariance, pin_cdf,
       pin_nested_partitions, pin_recursive_dyadic, pin_hierarchical_equal_mass, pin_masks,
       pin_chromatic_closed_forms, pin_forward_model_exact_for_piecewise_beta]
