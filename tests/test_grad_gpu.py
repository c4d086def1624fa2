"""GPU gradient of lnL (fgl_loglike_grad_batch, FP64) against the oracle's
analytic gradient, which is pinned to 50-digit central differences.

An entry of the gradient is a sum over (nu, t) of terms of both signs; near
the posterior peak it cancels to far below its terms.  The bar is therefore
|d| <= 1e-9 (|g| + S), where S is the sum of the magnitudes of the entry's
terms, (1/sigma^2) sum |r dM/dtheta| with |r| widened by 1e-13 |M| (the
rounding of the model values), computed here from the oracle's model values.
"""
import math

import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import check, lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fgl():
    return lib()


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def term_scale(orc, w, theta):
    """S[b, k]: magnitude of the terms of d lnL / d theta_k for row b."""
    na = getattr(w, "n_alpha", 0)
    nb = w.N // max(na, 1)
    K4 = w.K.reshape(max(na, 1), nb, w.F, w.T).astype(np.float64)
    out = np.zeros(theta.shape)
    L = np.log(w.freqs / w.nu_ref)
    for b, th in enumerate(theta):
        if na:
            M = orc.model_masks(K4, w.freqs, w.nu_ref, w.t_cmb, th)
        else:
            M = orc.model(w.K, w.freqs, w.nu_ref, w.t_cmb, th)
        if M is None:
            continue
        ra = np.abs(w.data - M) + 1e-13 * np.abs(M)
        beta = th[:nb]
        alpha = th[nb:nb + na] if na else np.ones(1)
        Pj = np.exp(-np.outer(L, beta))                       # [F, nb]
        sig = th[-1]
        for j in range(nb):
            kj = np.abs(np.tensordot(alpha, K4[:, j], axes=1))   # [F, T]
            out[b, j] = np.sum(ra * np.abs(L)[:, None] * Pj[:, j:j + 1] * kj)
        for i in range(na):
            ki = np.abs(np.einsum("jft,fj->ft", K4[i], Pj))
            out[b, nb + i] = np.sum(ra * ki)
        A, nu0, wd = th[-4], th[-3], th[-2]
        dn = w.freqs - nu0
        g = np.exp(-0.5 * (dn / wd) ** 2)[:, None]
        dn = dn[:, None]
        out[b, -4] = np.sum(ra * g)
        out[b, -3] = np.sum(ra * abs(A) * g * np.abs(dn)) / wd ** 2
        out[b, -2] = np.sum(ra * abs(A) * g * dn ** 2) / wd ** 3
        out[b, :-1] /= sig ** 2
        chi2 = np.sum((w.data - M) ** 2)
        out[b, -1] = chi2 / sig ** 3 + w.F * w.T / sig
    return out


def check_grad(got, ref, scale, label):
    ok = np.isfinite(ref).all(axis=1)
    assert np.all(np.isnan(got[~ok])), f"{label}: invalid rows must give NaN"
    d = np.abs(got[ok] - ref[ok])
    t = 1e-9 * (np.abs(ref[ok]) + scale[ok])
    worst = np.unravel_index(np.argmax(d / t), d.shape) if d.size else (0, 0)
    say(f"  {label} grad: rows={ok.sum()} max|d|/tol={(d / t).max() if d.size else 0:.3e}")
    assert np.all(d <= t), (label, worst, got[ok][worst], ref[ok][worst])


def _cases():
    f = lambda F: np.linspace(50.0, 200.0, F) if F > 1 else np.array([120.0])
    out = []
    for N, F, T, B in [(1, 5, 1, 7), (4, 151, 1, 64), (3, 9, 20, 100), (16, 13, 33, 70),
                       (8, 11, 70, 50), (40, 5, 100, 30), (33, 5, 17, 40), (64, 4, 40, 33),
                       (128, 3, 20, 20)]:
        out.append(("index", N, F, T, B,
                    lambda N=N, F=F, T=T, B=B: workload.make(N, f(F), T, B, 300 + N + T,
                                                             batch="mixed")))
    for NA, NB, F, T, B in [(2, 3, 9, 20, 50), (3, 5, 6, 1, 40), (2, 16, 7, 96, 40),
                            (4, 32, 3, 20, 20)]:
        out.append(("masks", NA * NB, F, T, B,
                    lambda NA=NA, NB=NB, F=F, T=T, B=B: workload.make_masks(
                        NA, NB, f(F), T, B, 400 + NA + NB, batch="mixed")))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}-N{c[1]}-F{c[2]}-T{c[3]}-B{c[4]}")
def test_grad_all_rows(fgl, orc, case):
    kind, N, F, T, B, make = case
    w = make()
    rl, rg = orc.grad_w(w)
    scale = term_scale(orc, w, w.theta)
    # the gradient sums over time in the projected rows when the model has
    # them, else over the time grid (forced by the flag); both are run
    # unless the model's form is already the direct one
    for flags in (0, fgl.FGL_MIXED_DIRECT):
        m = fgl.Model.from_workload(w, flags)
        form = m.form
        say(f"gradient {kind} N={w.N} F={w.F} T={w.T} B={w.B} P={w.P} form={form}")
        ll, g = m.loglike_grad(w.theta)
        check(ll, rl, "fp64", f"{kind}-N{N}/{form}", w.theta, w.F * w.T)
        check_grad(g, rg, scale, f"{kind}-N{N}/{form}")
        m.close()
        if form == "direct":
            break


def test_grad_headline_sampled(fgl, orc):
    """The full N=32, F=301, T=96, B=16384 call through the device entry
    point; the oracle on 48 sampled prior rows and 16 posterior-shell rows;
    host and device entry points agree bitwise."""
    import torch
    w = workload.config(workload.HEADLINE)
    m = fgl.Model.from_workload(w)
    th = torch.from_numpy(w.theta).cuda()
    out, grad = m.loglike_grad_device(th)
    torch.cuda.synchronize()
    out, grad = out.cpu().numpy(), grad.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(12))
    idx = np.sort(rng.choice(w.B, 48, replace=False))
    rl, rg = orc.grad_w(w, w.theta[idx])
    check(out[idx], rl, "fp64", "headline/grad-sampled", w.theta[idx], w.F * w.T)
    check_grad(grad[idx], rg, term_scale(orc, w, w.theta[idx]), "headline/grad-sampled")
    hl, hg = m.loglike_grad(w.theta[idx])
    assert np.array_equal(hl, out[idx]) and np.array_equal(hg, grad[idx])
    sh = workload.posterior_shell(workload.HEADLINE, 16)
    rl, rg = orc.grad_w(sh)
    sc = term_scale(orc, sh, sh.theta)
    assert m.form == "projected"
    for mm in (m, fgl.Model.from_workload(sh, fgl.FGL_MIXED_DIRECT)):
        sl, sg = mm.loglike_grad(sh.theta)
        check(sl, rl, "fp64", f"headline/grad-shell/{mm.form}", sh.theta, sh.F * sh.T)
        check_grad(sg, rg, sc, f"headline/grad-shell/{mm.form}")
        mm.close()


def test_grad_invalid_rows_and_errors(fgl, orc):
    w = workload.make_masks(2, 3, np.linspace(60.0, 180.0, 7), 5, 6, 17, batch="prior")
    th = w.theta.copy()
    th[1, -1] = 0.0
    th[2, 3] = -1.0          # alpha
    th[3, 0] = np.nan
    m = fgl.Model.from_workload(w)
    ll, g = m.loglike_grad(th)
    assert np.all(ll[1:4] == -np.inf) and np.all(np.isnan(g[1:4]))
    assert np.all(np.isfinite(ll[[0, 4, 5]])) and np.all(np.isfinite(g[[0, 4, 5]]))
    for prec in ("mixed", "fp32"):
        with pytest.raises(fgl.FGLError) as e:
            m.loglike_grad(th, prec)
        assert e.value.code == fgl.FGL_EINVAL
    m.close()


def test_grad_no_21cm(fgl, orc):
    """Without the 21-cm term the row is [beta.., sigma] and so is the
    gradient."""
    w = workload.make(5, np.linspace(50.0, 200.0, 21), 7, 32, 55, batch="prior")
    th = np.concatenate([w.theta[:, :5], w.theta[:, -1:]], axis=1)
    m = fgl.Model(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, fgl.FGL_NO_21CM)
    ll, g = m.loglike_grad(th)
    rl, rg = orc.grad(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, th, flags=oracle.NO_21CM)
    check(ll, rl, "fp64", "no21", th, w.F * w.T)
    d = np.abs(g - rg)
    say(f"  no21 grad max rel {np.max(d / np.abs(rg)):.3e}")
    assert np.all(d <= 1e-9 * np.abs(rg) + 1e-9 * np.abs(rg).max(axis=1, keepdims=True))
    m.close()
