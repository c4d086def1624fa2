"""Hypothesis-driven properties of the oracle on random small problems (CPU).

Shapes, responses, frequencies and parameter rows are drawn by hypothesis;
each example checks the oracle's lnL and model values against a 50-digit
mpmath evaluation of Eqs. fast_forward_model, t21model and likelihood, and
the invariances the method rests on: relabelling regions (K and beta
together) and splitting a region into two halves with the same spectral
index (the nesting of Sec. 4).
"""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests.pins import mp_loglike, mp_model

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@st.composite
def problems(draw):
    N = draw(st.integers(1, 3))
    F = draw(st.integers(1, 4))
    T = draw(st.integers(1, 3))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.Generator(np.random.PCG64(seed))
    K = rng.lognormal(math.log(draw(st.floats(0.5, 300.0))), 0.8, size=(N, F, T)).astype(np.float32)
    freqs = np.sort(rng.uniform(draw(st.floats(40.0, 120.0)), 230.0, size=F))
    th = np.empty(N + 4)
    th[:N] = [draw(st.floats(-4.0, 6.0)) for _ in range(N)]
    th[N] = draw(st.floats(-1.0, 1.0))
    th[N + 1] = draw(st.floats(40.0, 220.0))
    th[N + 2] = draw(st.floats(1.0, 50.0))
    th[N + 3] = math.exp(draw(st.floats(math.log(1e-3), math.log(1.0))))
    D = rng.normal(50.0, 20.0, size=(F, T))
    return K, freqs, D, th


def term_scale(K, freqs, th):
    """[F, T] sum of the magnitudes of the model's terms."""
    N = K.shape[0]
    P = (freqs[None, :] / 230.0) ** -th[:N, None]                 # [N, F]
    return (np.abs(K.astype(np.float64)) * P[:, :, None]).sum(0) + 2.725 + abs(th[N])


SETTINGS = settings(max_examples=40, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(problems())
def test_oracle_matches_50_digit_evaluation(orc, p):
    K, freqs, D, th = p
    got = orc.loglike(K, freqs, D, 230.0, 2.725, th[None, :])[0]
    ref = float(mp_loglike(K, freqs, D, 230.0, 2.725, th))
    assert abs(got - ref) <= 1e-13 * abs(ref) + 1e-300, (got, ref)
    m = orc.model(K, freqs, 230.0, 2.725, th)
    mref = mp_model(K, freqs, 230.0, 2.725, th)
    sc = term_scale(K, freqs, th)
    for f in range(K.shape[1]):
        for t in range(K.shape[2]):
            r = float(mref[f][t])
            # the model is a sum of terms of both signs (A may be positive
            # or negative): bound the error by the magnitude of its terms
            assert abs(m[f, t] - r) <= 1e-14 * sc[f, t], (f, t, m[f, t], r)


@SETTINGS
@given(problems(), st.integers(0, 2 ** 31 - 1))
def test_oracle_region_relabelling_and_nesting(orc, p, seed):
    K, freqs, D, th = p
    N = K.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    base = orc.loglike(K, freqs, D, 230.0, 2.725, th[None, :])[0]
    m0 = orc.model(K, freqs, 230.0, 2.725, th)
    # relabelling: K and beta permuted together
    perm = rng.permutation(N)
    thp = th.copy()
    thp[:N] = th[perm]
    lp = orc.loglike(np.ascontiguousarray(K[perm]), freqs, D, 230.0, 2.725, thp[None, :])[0]
    assert abs(lp - base) <= 1e-12 * abs(base) + 1e-9, (lp, base)
    # nesting: region j split into two halves with its spectral index
    j = int(rng.integers(0, N))
    Ks = np.concatenate([K[:j], K[j:j + 1] * np.float32(0.5), K[j:j + 1] * np.float32(0.5),
                         K[j + 1:]])
    ths = np.concatenate([th[:j], [th[j], th[j]], th[j + 1:]])
    m1 = orc.model(np.ascontiguousarray(Ks), freqs, 230.0, 2.725, ths)
    assert np.all(np.abs(m1 - m0) <= 1e-14 * term_scale(K, freqs, th))
