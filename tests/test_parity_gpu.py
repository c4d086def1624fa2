"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle.

Small workloads are compared row by row on every row; the full-size
workloads run in the launch configuration the benchmark times and are
compared on sampled rows.  Every case names its workload before it runs.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import check, lib, record, say, thin_form

pytestmark = pytest.mark.gpu

PRECS = ("mixed", "fp32", "fp64")


@pytest.fixture(scope="module")
def fgl():
    return lib()


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def _model(fgl, w, flags=0):
    return fgl.Model(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, flags)


def _mixed_forms(fgl, w, theta, ref, label, expect=None):
    """The mixed evaluation in both of its forms (the library's choice and
    the direct form forced by FGL_MIXED_DIRECT) against the oracle."""
    for flags in (0, fgl.FGL_MIXED_DIRECT):
        m = _model(fgl, w, flags)
        form = m.form
        if flags:
            assert form == "direct"
        elif expect is not None:
            assert form == expect, (label, form)
        check(m.loglike(theta, "mixed"), ref, "mixed", f"{label}/{form}")
        m.close()


@pytest.mark.parametrize("k", [workload.SMALL, workload.MEDIUM])
def test_small_workloads_all_rows(fgl, orc, k):
    """The small workloads (N=4, F=151, T=1 and N=16, F=151, T=20): every row
    of the prior batch and of a 1024-row posterior shell."""
    for kind in ("prior", "shell"):
        w = workload.config(k) if kind == "prior" else workload.posterior_shell(k)
        say(f"workload {k} {kind}: N={w.N} F={w.F} T={w.T} B={w.B}")
        ref = orc.loglike_w(w)
        m = _model(fgl, w)
        for prec in PRECS:
            got = m.loglike(w.theta, prec)
            if prec == "fp32" and kind == "shell":
                d = np.abs(got - ref)
                say(f"  fp32 shell (reported, not asserted): max|d|={d.max():.3e}")
                continue
            check(got, ref, prec, f"{k}/{kind}", w.theta, w.F * w.T)
        m.close()


def test_headline_shape_reduced_batch(fgl, orc):
    """N=32, F=301, T=96 (the headline shape): 1024 prior rows and the
    1024-row posterior shell, every row."""
    wp = workload.config(workload.HEADLINE, B=1024)
    ws = workload.posterior_shell(workload.HEADLINE, 1024)
    say(f"headline workload reduced: N={wp.N} F={wp.F} T={wp.T}")
    m = _model(fgl, wp)
    for w, kind in ((wp, "prior"), (ws, "shell")):
        ref = orc.loglike_w(w)
        _mixed_forms(fgl, w, w.theta, ref, f"headline/{kind}", expect="projected")
        check(m.loglike(w.theta, "fp64"), ref, "fp64", f"headline/{kind}", w.theta, w.F * w.T)
        got32 = m.loglike(w.theta, "fp32")
        d = np.abs(got32 - ref)
        say(f"  fp32 {kind}: max|d|={d.max():.3e} "
            f"max|d|/mixed-tol={(d / (1e-6 * np.abs(ref) + 1e-3)).max():.3e}")
    m.close()


def test_headline_full_batch_sampled(fgl, orc):
    """Full N=32, F=301, T=96, B=16384 call (the benchmark's launch), with
    the oracle on 512 sampled rows, plus a full posterior shell."""
    w = workload.config(workload.HEADLINE)
    say(f"headline workload full: B={w.B}")
    m = _model(fgl, w)
    rng = np.random.Generator(np.random.PCG64(5))
    idx = np.sort(rng.choice(w.B, 512, replace=False))
    ref = orc.loglike_w(w, w.theta[idx])
    for prec in ("mixed", "fp64"):
        got = m.loglike(w.theta, prec)
        check(got[idx], ref, prec, "headline/full-sampled", w.theta[idx], w.F * w.T)
    m.close()


def test_balanced_chunks_full_batch(fgl, orc):
    """At B = 16384 the 8-wave, 8-channel tile cuts each row tile's 301
    channels into 36 chunks of 8 and then 4 of 4, the small ones dispatched
    last on every XCD (the chunk plan the CPU test pins), while 4-channel
    blocks stay uniform.  Both launches give the same bits, in both forms,
    and agree with the oracle on sampled rows."""
    w = workload.config(workload.HEADLINE)
    rng = np.random.Generator(np.random.PCG64(13))
    idx = np.sort(rng.choice(w.B, 128, replace=False))
    ref = orc.loglike_w(w, w.theta[idx])
    for flags, occ in ((0, 3), (fgl.FGL_MIXED_DIRECT, 2)):
        m = _model(fgl, w, flags)
        outs = []
        for fc in (8, 4):
            say(f"balanced chunks: {m.form} form, tile 8 waves x {fc} channels, B={w.B}")
            m.set_tile(w.B, "mixed", 8, fc, occ)
            outs.append(m.loglike(w.theta, "mixed"))
        assert np.array_equal(outs[0], outs[1]), m.form
        check(outs[0][idx], ref, "mixed", f"balanced/{m.form}")
        m.close()


def test_large_workload_subsample(fgl, orc):
    """N=64, F=401, T=240, B=65536: full launch, oracle on 256 rows."""
    w = workload.config(workload.LARGE)
    say(f"large workload: N={w.N} F={w.F} T={w.T} B={w.B}")
    m = _model(fgl, w)
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.sort(rng.choice(w.B, 256, replace=False))
    ref = orc.loglike_w(w, w.theta[idx])
    assert m.form == "projected"
    got = m.loglike(w.theta, "mixed")
    check(got[idx], ref, "mixed", "large/sampled")
    m.close()
    md = _model(fgl, w, fgl.FGL_MIXED_DIRECT)
    check(md.loglike(w.theta, "mixed")[idx], ref, "mixed", "large/sampled/direct")
    md.close()
    sh = workload.posterior_shell(workload.LARGE, 256)
    _mixed_forms(fgl, sh, sh.theta, orc.loglike_w(sh), "large/shell", expect="projected")


@pytest.mark.parametrize("N,F,T,B,rich", [
    (32, 301, 96, 1024, False), (32, 301, 96, 1024, True), (33, 11, 70, 100, True),
    (64, 6, 65, 70, True), (96, 3, 130, 40, True), (7, 5, 70, 257, True), (1, 3, 80, 65, True)])
def test_plain_projected_form(fgl, orc, N, F, T, B, rich):
    """FGL_PLAIN_PROJECTED: the plain FP64 kernel on the projected rows meets
    the FP64 bar (prior and shell rows); the plain FP32 kernel on them is
    reported and held to the loose FP32 bar on prior rows; the mixed
    evaluation is unchanged by the flag."""
    if (N, F, T) == (32, 301, 96):
        w = workload.config(workload.HEADLINE, B=B, batch="mixed", rich=rich)
    else:
        w = workload.make(N, np.linspace(55.0, 190.0, F), T, B, 4000 + N + T,
                          chroma=0.05, batch="mixed", rich=rich)
    say(f"plain projected N={N} F={F} T={T} B={B} rich={rich}")
    ref = orc.loglike_w(w)
    m = fgl.Model.from_workload(w, fgl.FGL_PLAIN_PROJECTED)
    m0 = fgl.Model.from_workload(w)
    assert m.form == "projected"
    lab = f"plain-proj/N{N}F{F}T{T}" + ("/rich" if rich else "")
    check(m.loglike(w.theta, "fp64"), ref, "fp64", lab, w.theta, w.F * w.T)
    got32 = m.loglike(w.theta, "fp32")
    # one FP32 rounding of a projected row stands for the T roundings of the
    # time bins it sums, so this baseline is held only to a gross bound
    # (1e-3 relative) on the prior rows (the first half) and reported
    half = w.B // 2
    d = np.abs(got32[:half] - ref[:half])
    t = 1e-3 * np.abs(ref[:half]) + 1e-3
    record(lab + "/prior", "fp32", d, t)
    assert np.all(d <= t), (lab, float((d / t).max()))
    d = np.abs(got32 - ref)
    say(f"  fp32 projected (reported): max|d|={d.max():.3e} "
        f"max|d|/mixed-tol={(d / (1e-6 * np.abs(ref) + 1e-3)).max():.3e}")
    assert np.array_equal(m.loglike(w.theta, "mixed"), m0.loglike(w.theta, "mixed"))
    m.close()
    m0.close()


@pytest.mark.parametrize("name,B", [(workload.HEADLINE, 1024), (workload.LARGE, 256)])
def test_full_rank_responses(fgl, orc, name, B):
    """Full-rank responses (time harmonics and a per-value scatter for every
    region, a chromatic ripple; the data simulated from them): the
    posterior shell and a prior batch, every row, in both mixed forms and
    in FP64, at the headline shape and at N=64, F=401, T=240."""
    for kind in ("shell", "prior"):
        w = workload.config(name, B=B, batch=kind, rich=True)
        say(f"full-rank {name} {kind}: N={w.N} F={w.F} T={w.T} B={w.B}")
        ref = orc.loglike_w(w)
        _mixed_forms(fgl, w, w.theta, ref, f"{name}/rich/{kind}", expect="projected")
        m = _model(fgl, w)
        check(m.loglike(w.theta, "fp64"), ref, "fp64", f"{name}/rich/{kind}", w.theta,
              w.F * w.T)
        m.close()


@pytest.mark.parametrize("N,F,T,B", [
    (1, 7, 1, 1), (3, 5, 2, 257), (31, 13, 31, 300), (32, 9, 32, 64),
    (33, 11, 33, 100), (64, 6, 65, 70), (100, 5, 17, 40), (128, 3, 40, 33),
    (7, 1, 96, 512), (12, 40, 130, 129), (32, 6, 40, 100), (32, 5, 33, 64),
    (40, 9, 96, 200), (70, 4, 100, 50), (96, 3, 130, 40), (1, 3, 50, 65),
    (8, 9, 16, 300), (17, 5, 3, 70), (32, 7, 16, 257), (31, 4, 9, 33), (33, 5, 2, 40),
    (11, 6, 5, 90), (14, 5, 12, 66), (16, 7, 25, 70), (8, 5, 48, 90), (4, 3, 64, 40),
    (20, 5, 10, 33)])
def test_shapes_and_ragged_tails(fgl, orc, N, F, T, B):
    """Region chunks (N over 32), ragged time tiles, ragged batches, a single
    channel, a single row, with chromatic K and mixed prior/shell rows; the
    mixed evaluation in both forms wherever the projected one applies
    (T >= N + 1 with fewer row tiles; with and without the peeled row), and
    the per-row FP64 form of small models beside the forced direct form."""
    freqs = np.linspace(55.0, 190.0, F) if F > 1 else np.array([123.0])
    w = workload.make(N, freqs, T, B, 1000 + N * 7 + T, chroma=0.05, batch="mixed")
    say(f"shape N={N} F={F} T={T} B={B}")
    ref = orc.loglike_w(w)
    proj = T >= N + 1 and N <= 96 and (N + 1 - (N % 32 == 0) + 31) // 32 < (T + 31) // 32
    thin = thin_form(N, T)
    _mixed_forms(fgl, w, w.theta, ref, f"N{N}F{F}T{T}B{B}",
                 expect="thin" if thin else ("projected" if proj else "direct"))
    m = _model(fgl, w)
    for prec in ("fp32", "fp64"):
        got = m.loglike(w.theta, prec)
        if prec == "fp32":
            half = B // 2      # prior half only
            check(got[:half], ref[:half], prec, f"N{N}F{F}T{T}B{B}")
        else:
            check(got, ref, prec, f"N{N}F{F}T{T}B{B}", w.theta, w.F * w.T)
    m.close()


def test_edge_rows_and_values(fgl, orc):
    """Invalid rows give -inf; signed and tiny K, a channel at nu_ref, a
    large 21-cm amplitude, beta at the +-64 limit, nu near 2^+-8 nu_ref."""
    rng = np.random.Generator(np.random.PCG64(77))
    N, T = 5, 7
    freqs = np.array([1.0, 50.0, 230.0, 231.0, 5000.0, 58000.0])
    F = freqs.size
    K = rng.normal(0.0, 3.0, size=(N, F, T)).astype(np.float32)
    K[1] *= np.float32(1e-6)
    D = rng.normal(20.0, 5.0, size=(F, T))
    th = np.zeros((12, N + 4))
    th[:, :N] = rng.uniform(-2.0, 4.0, size=(12, N))
    th[:, N:] = [-0.1, 120.0, 15.0, 0.5]
    th[1, N + 3] = 0.0          # sigma = 0
    th[2, N + 2] = -3.0         # w < 0
    th[3, 2] = np.nan
    th[4, 0] = 65.0             # beyond the beta limit
    th[5, N] = np.inf
    th[6, 0] = 4.5              # steep spectrum across 2^+-8 of nu_ref
    th[6, 1] = -2.5
    th[7, N] = 1e6              # huge 21-cm amplitude
    th[8, N + 2] = 1e-3         # very narrow profile
    th[9, :N] = 0.0             # unit powers
    th[10, N + 3] = 1e3         # broad noise
    m = fgl.Model(K, freqs, D, 230.0, 2.725)
    ref = orc.loglike(K, freqs, D, 230.0, 2.725, th)
    say(f"edge rows: ref={ref}")
    assert np.all(ref[1:6] == -np.inf)
    for prec in ("mixed", "fp64"):
        check(m.loglike(th, prec), ref, prec, "edge", th, F * T)
    # the digit kernel on the same edges (the model above is evaluated per row)
    md = fgl.Model(K, freqs, D, 230.0, 2.725, fgl.FGL_MIXED_DIRECT)
    assert m.form == "thin" and md.form == "direct"
    check(md.loglike(th, "mixed"), ref, "mixed", "edge/direct", th, F * T)
    md.close()
    got32 = m.loglike(th, "fp32")
    assert np.all(got32[1:6] == -np.inf)
    m.close()
    # spectral indices at the +-64 validity limit on a narrow band
    f2 = np.linspace(200.0, 260.0, 9)
    K2 = rng.lognormal(1.0, 0.5, size=(3, 9, 4)).astype(np.float32)
    D2 = rng.normal(30.0, 3.0, size=(9, 4))
    th2 = np.array([[64.0, -64.0, 0.5, -0.1, 220.0, 10.0, 2.0],
                    [-64.0, 64.0, 63.9, 0.0, 210.0, 5.0, 1.0],
                    [64.0000001, 1.0, 1.0, 0.0, 210.0, 5.0, 1.0]])
    m2 = fgl.Model(K2, f2, D2, 230.0, 2.725)
    ref2 = orc.loglike(K2, f2, D2, 230.0, 2.725, th2)
    assert np.all(np.isfinite(ref2[:2])) and ref2[2] == -np.inf
    for prec in ("mixed", "fp64"):
        check(m2.loglike(th2, prec), ref2, prec, "beta-limit", th2, 9 * 4)
    m2.close()


def test_edge_rows_projected_form(fgl, orc):
    """The projected form on degenerate responses: a region with K = 0, two
    identical regions (rank-deficient), a region constant in time (zero
    after centring), data constant in time, T = N + 1, and the invalid and
    extreme rows of the direct-form edge test."""
    rng = np.random.Generator(np.random.PCG64(78))
    for N, T in ((6, 70), (32, 33), (33, 96)):
        F = 7
        freqs = np.linspace(60.0, 180.0, F)
        K = rng.lognormal(2.0, 0.5, size=(N, F, T)).astype(np.float32)
        K[1] = 0.0
        K[3] = K[2]
        K[4] = K[4, :, :1]
        D = rng.normal(200.0, 5.0, size=(F, T))
        D[2] = 123.0
        th = np.zeros((10, N + 4))
        th[:, :N] = rng.uniform(1.5, 3.5, size=(10, N))
        th[:, N:] = [-0.1, 120.0, 15.0, 0.05]
        th[1, N + 3] = 0.0
        th[2, 3] = np.nan
        th[3, 0] = -64.0
        th[4, N] = 1e6
        th[5, :N] = 0.0
        th[6, N + 3] = 1e-6
        m = fgl.Model(K, freqs, D, 230.0, 2.725)
        say(f"projected edge N={N} T={T}: form={m.form}")
        assert m.form == "projected"
        ref = orc.loglike(K, freqs, D, 230.0, 2.725, th)
        check(m.loglike(th, "mixed"), ref, "mixed", f"proj-edge N{N}T{T}")
        m.close()


def test_nesting_projected_form(fgl, orc):
    """Strict nesting through the projected form: splitting a region into
    two halves with the same spectral index leaves lnL unchanged (the split
    model is rank-deficient)."""
    w = workload.make(8, np.linspace(50.0, 200.0, 31), 72, 256, 4242, chroma=0.05, batch="mixed")
    K2 = np.concatenate([w.K[:3], w.K[3:4] * np.float32(0.5), w.K[3:4] * np.float32(0.5), w.K[4:]])
    th2 = np.concatenate([w.theta[:, :4], w.theta[:, 3:4], w.theta[:, 4:]], axis=1)
    ref = orc.loglike_w(w)
    m1 = _model(fgl, w)
    m2 = fgl.Model(K2, w.freqs, w.data, w.nu_ref, w.t_cmb)
    assert m1.form == m2.form == "projected"
    a, b = m1.loglike(w.theta, "mixed"), m2.loglike(th2, "mixed")
    check(a, ref, "mixed", "nest/original")
    check(b, ref, "mixed", "nest/split")
    m1.close()
    m2.close()


@pytest.mark.parametrize("k", [workload.MEDIUM, workload.HEADLINE])
def test_no_21cm_flag(fgl, orc, k):
    w = workload.config(k, B=512)
    th = np.concatenate([w.theta[:, :w.N], w.theta[:, -1:]], axis=1)
    m = fgl.Model(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, flags=fgl.FGL_NO_21CM)
    assert m.P == w.N + 1
    say(f"no21 workload {k}: form={m.form}")
    ref = orc.loglike(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, th, flags=1)
    check(m.loglike(th, "mixed"), ref, "mixed", "no21")
    check(m.loglike(th, "fp64"), ref, "fp64", "no21", th, w.F * w.T)
    m.close()


def test_determinism_and_row_independence(fgl):
    """Bitwise: repeated calls (eager, then graph capture, then replays with
    other work in between), one row alone vs inside a large batch, batch
    permutation, and tuned vs default tiles."""
    w = workload.config(workload.HEADLINE, B=4096, batch="mixed")
    m = _model(fgl, w)
    other = _model(fgl, workload.config(workload.MEDIUM, B=64))
    for prec in PRECS:
        say(f"determinism {prec}")
        a = m.loglike(w.theta, prec)
        for rep in range(4):
            other.loglike(workload.config(workload.MEDIUM, B=64).theta, prec)
            b = m.loglike(w.theta, prec)
            assert np.array_equal(a, b), (prec, rep)
        one = m.loglike(w.theta[123:124], prec)
        assert one[0] == a[123]
        p = np.random.Generator(np.random.PCG64(3)).permutation(w.B)
        assert np.array_equal(m.loglike(w.theta[p], prec), a[p])
        m.tune(w.B, prec)
        assert np.array_equal(m.loglike(w.theta, prec), a), f"{prec}: tile changed bits"
    m.close()
    other.close()


def test_form_rule(fgl):
    """The library's choice of form follows the documented rule over a grid
    of (N, T): thin by the cost rule, else projected when N + 1 rows take
    fewer 32-row tiles than T, else direct."""
    rng = np.random.Generator(np.random.PCG64(5))
    freqs = np.array([70.0, 150.0])
    n = 0
    for N in (1, 3, 4, 5, 8, 9, 12, 13, 16, 17, 20, 24, 25, 31, 32, 33):
        for T in (1, 6, 8, 9, 10, 20, 25, 26, 32, 33, 40, 48, 49, 58, 64, 65):
            K = rng.uniform(0.5, 2.0, size=(N, 2, T)).astype(np.float32)
            D = rng.normal(100.0, 1.0, size=(2, T))
            m = fgl.Model(K, freqs, D, 230.0, 2.725)
            peel = 1 if N % 32 == 0 else 0
            proj = T >= N + 1 and (N + 1 - peel + 31) // 32 < (T + 31) // 32
            want = "thin" if thin_form(N, T) else ("projected" if proj else "direct")
            assert m.form == want, (N, T, m.form, want)
            m.close()
            n += 1
    say(f"form rule: {n} models")


def test_every_tile_same_bits(fgl):
    """Every candidate tile (waves, channels per workgroup, register budget)
    gives bitwise the same lnL, in each form and precision."""
    cases = [("thin", workload.config(workload.MEDIUM, B=700, batch="mixed"), 0),
             ("projected", workload.config(workload.HEADLINE, B=1024, batch="mixed"), 0),
             ("direct", workload.config(workload.HEADLINE, B=1024, batch="mixed"), fgl.FGL_MIXED_DIRECT),
             ("masks", workload.make_masks(2, 5, np.linspace(60.0, 190.0, 41), 40, 700, 31,
                                           batch="mixed"), 0)]
    for label, w, flags in cases:
        m = fgl.Model.from_workload(w, flags)
        for prec in PRECS:
            ref, n = None, 0
            for W in (1, 2, 4, 8):
                for fc in range(1, 33):
                    for occ in (2, 3):
                        try:
                            m.set_tile(w.B, prec, W, fc, occ)
                        except fgl.FGLError:
                            continue
                        got = m.loglike(w.theta, prec)
                        if ref is None:
                            ref = got
                        assert np.array_equal(got, ref), (label, prec, W, fc, occ)
                        n += 1
            say(f"tiles {label}/{m.form}/{prec}: {n} candidates, same bits")
            assert n >= 2
        m.close()


def test_kernel_timing_every_nth_call(fgl):
    """fgl_kernel_timing(m, n) records the kernel of calls 0, n, 2n, ... and
    changes no result; n < 0 is refused."""
    w = workload.config(workload.SMALL, B=64)
    m = _model(fgl, w)
    ref = m.loglike(w.theta, "mixed")
    m.kernel_timing(True, every=3)
    for _ in range(7):
        assert np.array_equal(m.loglike(w.theta, "mixed"), ref)
    ms, n = m.kernel_time()
    assert n == 3 and ms > 0.0, (n, ms)
    m.kernel_timing(False)
    with pytest.raises(fgl.FGLError) as e:
        m.kernel_timing(True, every=-1)
    assert e.value.code == fgl.FGL_EINVAL
    m.close()


def test_device_entry_point_matches_host(fgl):
    import torch
    w = workload.config(workload.HEADLINE, B=2048, batch="mixed")
    m = _model(fgl, w)
    th = torch.from_numpy(w.theta).to("cuda")
    for prec in PRECS:
        out = m.loglike_device(th, prec=prec)
        torch.cuda.synchronize()
        host = m.loglike(w.theta, prec)
        assert np.array_equal(out.cpu().numpy(), host), prec
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = m.loglike_device(th, prec="mixed", stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), m.loglike(w.theta, "mixed"))
    m.close()


def test_errors_and_zero_rows(fgl):
    w = workload.config(workload.SMALL, B=8)
    m = _model(fgl, w)
    assert m.loglike(np.zeros((0, m.P))).shape == (0,)
    with pytest.raises(fgl.FGLError) as e:
        fgl.fgl_loglike_batch(m.handle, w.theta, 8, np.empty(8), 7)
    assert e.value.code == fgl.FGL_EINVAL
    with pytest.raises(fgl.FGLError):
        fgl.Model(w.K, -w.freqs, w.data)
    with pytest.raises(fgl.FGLError):
        fgl.Model(w.K, w.freqs, w.data, nu_ref=0.0)
    bad = w.K.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(fgl.FGLError):
        fgl.Model(bad, w.freqs, w.data)
    # more than 2^26 rows per call is refused before theta is read
    small = np.zeros(8)
    for B in (-1, 2**26 + 1):
        rc = fgl._lib.fgl_loglike_batch(m.handle, small.ctypes.data_as(fgl._dp), B,
                                        small.ctypes.data_as(fgl._dp), 0)
        assert rc == fgl.FGL_EINVAL and "B=" in fgl.fgl_last_error(), B
    m.close()
