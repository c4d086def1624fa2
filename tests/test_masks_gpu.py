"""GPU parity of the crossed-mask model: amplitude masks crossed with
spectral-index masks (Eq. fast_forward_model with its amplitude scales),
created through fgl_model_create_masks, against the oracle's crossed-mask
likelihood.  Shapes span one region to the 128-region maximum, both forms
of the mixed evaluation, ragged tiles and several region chunks."""
import numpy as np
import pytest

import oracle
import workload
from paper_2603_13196_amd import sampler as ns
from tests.gpu_util import check, lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fgl():
    return lib()


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def _freqs(F):
    return np.linspace(50.0, 200.0, F) if F > 1 else np.array([120.0])


def _forms(fgl, w, ref, label):
    """Mixed in the library's form and in the forced direct form."""
    for flags in (0, fgl.FGL_MIXED_DIRECT):
        m = fgl.Model.from_workload(w, flags)
        check(m.loglike(w.theta, "mixed"), ref, "mixed", f"{label}/{m.form}")
        m.close()


@pytest.mark.parametrize("NA,NB,F,T,B", [
    (1, 1, 5, 1, 7),        # one region
    (2, 3, 9, 20, 300),     # thin (per-row FP64) form
    (3, 5, 7, 4, 65),       # thin form, 16 slots
    (2, 4, 6, 40, 90),      # thin form beyond one 32-bin tile
    (2, 3, 9, 70, 300),     # projected form, ragged row tile
    (4, 5, 7, 19, 65),      # direct form (T < N + 1)
    (2, 16, 11, 96, 200),   # the headline split, projected, one alpha per half chunk
    (4, 8, 6, 40, 100),     # 32 regions: projected with the peeled row
    (3, 11, 5, 40, 70),     # 33 regions: two chunks
    (8, 8, 4, 70, 40),      # 64 regions
    (2, 48, 3, 120, 33),    # 96 regions: largest projected form
    (4, 32, 3, 20, 33),     # 128 regions: largest direct form
])
def test_masks_all_rows(fgl, orc, NA, NB, F, T, B):
    for batch in ("prior", "shell"):
        w = workload.make_masks(NA, NB, _freqs(F), T, B, 1000 + NA * 131 + NB, batch=batch)
        say(f"masks {NA}x{NB} F={F} T={T} B={B} {batch}")
        ref = orc.loglike_w(w)
        _forms(fgl, w, ref, f"{NA}x{NB}/{batch}")
        m = fgl.Model.from_workload(w)
        check(m.loglike(w.theta, "fp64"), ref, "fp64", f"{NA}x{NB}/{batch}", w.theta, F * T)
        got32 = m.loglike(w.theta, "fp32")
        if batch == "prior":
            check(got32, ref, "fp32", f"{NA}x{NB}/{batch}")
        else:
            say(f"  fp32 shell (reported): max|d|={np.abs(got32 - ref).max():.3e}")
        m.close()


def test_masks_headline_split(fgl, orc):
    """2 amplitude x 16 spectral-index masks at F=301, T=96: the full
    B=16384 launch (oracle on 512 sampled rows) and a 1024-row posterior
    shell, every row."""
    w = workload.masks_config()
    say(f"{w.name}: P={w.P}")
    m = fgl.Model.from_workload(w)
    assert m.form == "projected" and m.P == 22
    rng = np.random.Generator(np.random.PCG64(6))
    idx = np.sort(rng.choice(w.B, 512, replace=False))
    ref = orc.loglike_w(w, w.theta[idx])
    for prec in ("mixed", "fp64"):
        check(m.loglike(w.theta, prec)[idx], ref, prec, "masks/full-sampled",
              w.theta[idx], w.F * w.T)
    m.close()
    sh = workload.masks_config(B=1024, batch="shell")
    _forms(fgl, sh, orc.loglike_w(sh), "masks/shell")


def test_masks_invalid_and_extreme_scales(fgl, orc):
    """Amplitude scales outside [2^-32, 2^32] (zero, negative, NaN) give
    -inf in every precision; the bounds themselves and widely spread scales
    within a row are evaluated to the usual bars."""
    w = workload.make_masks(3, 4, _freqs(13), 24, 16, 77, batch="prior")
    th = w.theta.copy()
    NB = 4
    th[1, NB] = 0.0
    th[2, NB + 1] = -0.5
    th[3, NB + 2] = 2.0 ** 33
    th[4, NB] = np.nan
    th[5, NB + 1] = 2.0 ** -33
    th[6, NB:NB + 3] = [2.0 ** 32, 1.0, 2.0 ** -32]
    th[7, NB:NB + 3] = [1e-3, 1e3, 1.0]
    th[8, NB:NB + 3] = [2.0 ** -32, 2.0 ** -32, 2.0 ** -32]
    ref = orc.loglike_w(w, th)
    assert np.all(ref[1:6] == -np.inf) and np.all(np.isfinite(ref[6:]))
    for flags in (0, fgl.FGL_MIXED_DIRECT):
        m = fgl.Model.from_workload(w, flags)
        check(m.loglike(th, "mixed"), ref, "mixed", f"extreme/{m.form}")
        check(m.loglike(th, "fp64"), ref, "fp64", f"extreme/{m.form}", th, w.F * w.T)
        got32 = m.loglike(th, "fp32")
        assert np.all(got32[1:6] == -np.inf) and np.all(np.isfinite(got32[6:]))
        m.close()


def test_masks_unit_scales_match_index_only_model(fgl, orc):
    """With every alpha = 1 the crossed model is the spectral-index-only
    model whose region (i, j) has index beta_j: both libraries' results
    agree with the oracle of the index-only model."""
    w = workload.make_masks(2, 5, _freqs(17), 30, 128, 91, batch="mixed")
    th = w.theta.copy()
    th[:, 5:7] = 1.0
    flat = np.concatenate([np.tile(th[:, :5], 2), th[:, 7:]], axis=1)
    ref = orc.loglike(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, flat)
    mm = fgl.Model.from_workload(w)
    mb = fgl.Model(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb)
    for prec in ("mixed", "fp64"):
        check(mm.loglike(th, prec), ref, prec, "unit-alpha/masks", th, w.F * w.T)
        check(mb.loglike(flat, prec), ref, prec, "unit-alpha/index-only", flat, w.F * w.T)
    mm.close()
    mb.close()


def test_masks_device_chains(fgl):
    """The device slice chains run on a crossed-mask model: they return the
    library's lnL at their end points and stay in the box."""
    w = workload.make_masks(2, 3, _freqs(11), 4, 8, 5, batch="prior")
    model = fgl.Model.from_workload(w)
    lo, hi = ns.foreground_box(3, n_alpha=2)
    assert lo.size == model.P
    n = 500
    x0 = np.repeat(((lo + hi) / 2)[None, :], n, axis=0)
    l0 = model.loglike(ns.to_theta(x0), "mixed")
    eng = fgl.Chains(model, n, lo, hi, seed=3)
    x, lx, ev, rounds = eng.run(x0, l0, -np.inf, np.diag((hi - lo) / 4), 10)
    say(f"masks chains: evals={ev} rounds={rounds}")
    assert np.all((x >= lo) & (x <= hi))
    assert np.allclose(lx, model.loglike(ns.to_theta(x), "mixed"), rtol=1e-12, atol=1e-9)
    eng.close()
    model.close()
