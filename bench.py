#!/usr/bin/env python3
"""Benchmark of the batched foreground log-likelihood on one MI355X.

One step = one call of the whole path (row preparation, the fused
power-law / contraction / FP64 residual kernel, the fixed-order finalize)
over one batch of B parameter rows already resident in HBM.  The headline
workload is N=32 regions, F=301 channels, T=96 time bins, B=16384 rows,
mixed precision; the plain FP32 and FP64 forms are timed the same way on
the same rows, the serving mix is run briefly for its p50/p99 latency, and
the FP64 CPU oracle is timed on a bounded sample on the host cores.  Further
legs time the kernels of the other parts of the method (small batches, the
gradient, crossed masks, region construction, the noise reference
distribution of the accuracy criterion, nested sampling); each has a --no-*
switch.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector, published
PEAK_INT8_TOPS = 5000.0      # MI355X dense int8 matrix, published
PEAK_HBM_BPS = 8.0e12        # MI355X HBM3E, published
TIMING_EVERY = 10            # kernel events on every 10th timed call (an event pair adds ~9 us)
PRECS = ("mixed", "fp32", "fp64")
EXP_FLOPS = 20               # FP64 flops counted per power-law value


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    # the device clock ramps to its steady state over ~40 ms of load and
    # drops again after idling, so the warm-up runs ~60 ms and the timed
    # region ~100 ms of the headline call
    p.add_argument("--steps", type=int, default=500)
    p.add_argument("--warmup", type=int, default=300)
    p.add_argument("--workload", default="N32_F301_T96_B16384",
                   choices=["N4_F151_T1_B1000", "N16_F151_T20_B4096", "N32_F301_T96_B16384",
                            "N64_F401_T240_B65536"])
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--serve-seconds", type=float, default=1.2)
    p.add_argument("--serve-configs", default=None,
                   help="serving configurations to run instead of the sweep, as "
                        "SLOTS:SHARING[:HALF], e.g. 4:16 or 4:1:half")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--no-sampler", action="store_true",
                   help="skip the nested-sampling run (10 regions, T = 1, benchmark settings)")
    p.add_argument("--no-regions", action="store_true",
                   help="skip the region-construction leg (importance, partition, K)")
    p.add_argument("--no-small", action="store_true",
                   help="skip the launch-bound small-batch workloads")
    p.add_argument("--no-noise", action="store_true",
                   help="skip the residual-likelihood reference distribution leg")
    p.add_argument("--no-grad", action="store_true",
                   help="skip the FP64 gradient leg")
    p.add_argument("--no-large", action="store_true",
                   help="skip the N64 F401 T240 B65536 leg")
    p.add_argument("--no-masks", action="store_true",
                   help="skip the crossed-mask model (2 amplitude x 16 index masks)")
    p.add_argument("--no-tune", action="store_true",
                   help="time the default tiles instead of the autotuned ones")
    p.add_argument("--tile", default=None,
                   help="waves,chans,occupancy: force this tile for the mixed precision on the "
                        "headline workload (no tuning of it), so that separate profiler passes "
                        "measure the same kernel variant")
    p.add_argument("--calib-copy", action="store_true",
                   help="only run a 256 MiB device-to-device copy three times "
                        "(calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_prec(fgl, m, th, out, prec, steps, warmup):
    import torch
    for _ in range(warmup):
        m.loglike_device(th, out, prec)
    torch.cuda.synchronize()
    m.kernel_timing(True, every=TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.loglike_device(th, out, prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, n = m.kernel_time()
    m.kernel_timing(False)
    B = th.shape[0]
    ms = (t1 - t0) * 1e3 / steps
    return {"evals_per_s": B * steps / (t1 - t0), "ms_per_step": ms,
            "kernel_ms": kms / max(n, 1), "launches": n}


def traffic_from_profiles(kernel_src_hash):
    """HBM bytes per launch of the likelihood kernel from the committed
    rocprofv3 counter summary (lines "key: value"), if it was taken on the
    current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_mixed_N32_F301_T96_B16384_traffic.txt")
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(("#", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    except OSError:
        return None
    if kv.get("kernel_source_sha256") != kernel_src_hash:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _serve_run(fgl, clients, models, seconds, inflight, share, budget, log_every=1.0):
    """The closed-loop serving mix for `seconds`: each client waits Exp(2 ms)
    after a result before submitting its next batch (mixed precision)."""
    srv = fgl.Server(budget_bytes=budget, max_inflight=inflight)
    srv.set_sharing(share)
    rng = np.random.Generator(np.random.PCG64(31))
    state = []
    now = time.perf_counter()
    for c in clients:
        state.append({"next": now + rng.exponential(2e-3), "ticket": None, "k": 0})
    lat, rows = [], 0
    t_start = time.perf_counter()
    t_end = t_start + seconds
    next_log = t_start + log_every
    while True:
        now = time.perf_counter()
        if now >= next_log:
            log(f"serving (slots {inflight}, sharing {share}): {len(lat)} requests done")
            next_log += log_every
        busy = False
        for c, st, m in zip(clients, state, models):
            if st["ticket"] is not None:
                busy = True
                r = srv.poll(st["ticket"])
                if r is not None:
                    out, us = r
                    lat.append(us)
                    rows += out.size
                    st["ticket"] = None
                    st["next"] = now + rng.exponential(2e-3)
            elif now < t_end and now >= st["next"]:
                B = c.batches[st["k"] % len(c.batches)]
                st["ticket"] = srv.submit(m, c.work.theta[:B], "mixed")
                st["k"] += 1
                busy = True
        if now >= t_end and not busy:
            break
        time.sleep(20e-6)
    wall = time.perf_counter() - t_start
    launches, shared, groups = srv.stats()
    srv.close()
    lat = np.array(lat)
    return {"max_inflight": inflight, "sharing": share, "requests": int(lat.size),
            "p50_ms": float(np.percentile(lat, 50)) / 1e3,
            "p99_ms": float(np.percentile(lat, 99)) / 1e3,
            "evals_per_s": rows / wall, "seconds": wall, "launches": launches,
            "shared_launches": shared, "groups_in_shared": groups}


def _serve_open(fgl, clients, models, seconds, inflight, share, rate, seed=37):
    """Open-loop arrivals: requests arrive as a Poisson process of `rate`
    per second whatever the completions, each from a client drawn uniformly
    with its next batch size, for `seconds`; then the queue drains."""
    srv = fgl.Server(max_inflight=inflight)
    srv.set_sharing(share)
    rng = np.random.Generator(np.random.PCG64(seed))
    nxt = [0] * len(clients)
    pending, lat, rows = [], [], 0
    t_start = time.perf_counter()
    t_end = t_start + seconds
    arrival = t_start + rng.exponential(1.0 / rate)
    while True:
        now = time.perf_counter()
        while arrival <= now and arrival < t_end:
            c = int(rng.integers(len(clients)))
            cl = clients[c]
            B = cl.batches[nxt[c] % len(cl.batches)]
            nxt[c] += 1
            pending.append(srv.submit(models[c], cl.work.theta[:B], "mixed"))
            arrival += rng.exponential(1.0 / rate)
        still = []
        for t in pending:
            r = srv.poll(t)
            if r is None:
                still.append(t)
            else:
                out, us = r
                lat.append(us)
                rows += out.size
        pending = still
        if now >= t_end and not pending:
            break
        time.sleep(20e-6)
    wall = time.perf_counter() - t_start
    srv.close()
    lat = np.array(lat)
    return {"offered_rps": rate, "achieved_rps": lat.size / wall, "requests": int(lat.size),
            "p50_ms": float(np.percentile(lat, 50)) / 1e3,
            "p99_ms": float(np.percentile(lat, 99)) / 1e3,
            "evals_per_s": rows / wall, "seconds": wall}


def serving_leg(fgl, seconds, configs_arg=None):
    """The 64-client serving mix swept over 1..4 in-flight slots (the box
    runs 4 hardware queues per process), with per-model launches and with
    launches shared by up to 16 models of one kernel variant, every model
    resident; then at 2 and 4 slots under an HBM budget of half the
    models' resident bytes, where admission waits and evictions take part.
    The headline record is the resident configuration with the lowest p99;
    at that configuration an open-loop sweep then offers Poisson arrivals at
    0.5, 0.8 and 1.0 of the request rate it sustained closed-loop."""
    import workload
    clients = workload.serving_clients(64, n_requests=64)
    models = [fgl.Model.from_workload(c.work) for c in clients]
    total = sum(m.nbytes for m in models)
    half = max(total // 2, max(m.nbytes for m in models))
    sweep = []
    configs = [(i, sh, 0) for sh in (1, 16) for i in (1, 2, 3, 4)]
    configs += [(i, sh, half) for sh in (1, 16) for i in (2, 4)]
    if configs_arg:
        configs = []
        for c in configs_arg.split(","):
            f = c.split(":")
            configs.append((int(f[0]), int(f[1]), half if len(f) > 2 else 0))
    for inflight, share, budget in configs:
        r = _serve_run(fgl, clients, models, seconds, inflight, share, budget)
        r["budget_bytes"] = budget
        sweep.append(r)
        log(f"serving slots {inflight} sharing {share} budget {budget}: p50 {r['p50_ms']:.3f} ms, "
            f"p99 {r['p99_ms']:.3f} ms, {r['evals_per_s']:.3e} evals/s, "
            f"{r['shared_launches']} shared launches of {r['launches']}")
    best = min((r for r in sweep if not r["budget_bytes"]), key=lambda r: r["p99_ms"],
               default=sweep[0])
    # open loop at the best resident configuration: Poisson arrivals at 0.5,
    # 0.8 and 1.0 of the request rate that configuration sustained closed-loop
    cap = max((r["requests"] / r["seconds"] for r in sweep
               if not r["budget_bytes"] and r["max_inflight"] == best["max_inflight"]
               and r["sharing"] == best["sharing"]), default=1.0)
    open_loop = []
    for load in (0.5, 0.8, 1.0):
        r = _serve_open(fgl, clients, models, seconds, best["max_inflight"], best["sharing"],
                        load * cap)
        r["load"] = load
        open_loop.append(r)
        log(f"serving open loop at {load:.1f} x {cap:.0f} requests/s: p50 {r['p50_ms']:.3f} ms, "
            f"p99 {r['p99_ms']:.3f} ms, {r['achieved_rps']:.0f} requests/s")
    for m in models:
        m.close()
    return {"clients": len(clients), "models_bytes": total,
            "requests": best["requests"], "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
            "evals_per_s": best["evals_per_s"], "max_inflight": best["max_inflight"],
            "sharing": best["sharing"], "budget_bytes": 0, "sweep": sweep,
            "capacity_rps": cap, "open_loop": open_loop}


def sampler_leg(fgl, regions=10, T=1):
    """One nested-sampling run with the slice chains on the device, at the
    paper's benchmark hyperparameters (n_live = 25 d, num_inner_steps = 5 d,
    num_delete = n_live / 5) on a synthetic model with `regions` regions and
    T time bins (the time-integrated and time-resolved cases of the paper's
    benchmark)."""
    import math
    import workload
    from paper_2603_13196_amd import sampler as ns
    w = workload.make(regions, workload.freq_grid(50.0, 200.0, 1.0), T, 8, 1234 + regions + T,
                      batch="prior")
    m = fgl.Model.from_workload(w)
    lo, hi = ns.foreground_box(w.N)
    d = lo.size
    n_live, inner = 25 * d, 5 * d
    b = n_live // 5
    ch = ns.gpu_chains(m, lo, hi, b, "mixed", seed=1)
    t0 = time.perf_counter()
    r = ns.nested_slice_sampling(ns.model_loglike(m, "mixed"), lo, hi, n_live=n_live,
                                 num_delete=b, num_inner_steps=inner, seed=2, chains=ch)
    dt = time.perf_counter() - t0
    zt = np.concatenate([w.truth[:-1], [math.log(w.truth[-1])]])[None, :]
    l_truth = float(m.loglike(ns.to_theta(zt), "mixed")[0])
    ch.engine.close()
    m.close()
    # accuracy criterion (Sec. 5): the fit's median posterior lnL against 4096
    # noise-only data sets at the simulated noise level
    sig = float(w.truth[-1])
    ref = fgl.fgl_noise_loglike(w.F * T, 4096, sig, sig, seed=regions * 1000 + T)
    lbar = r.median_loglike()
    q, q_truth = fgl.fgl_noise_quantile(ref, [lbar, l_truth])
    return {"model": f"N{regions}_F{w.F}_T{T}", "d": d, "n_live": n_live, "num_delete": b,
            "num_inner_steps": inner, "seconds": dt, "iterations": r.iterations,
            "likelihood_evals": r.n_like, "evals_per_s": r.n_like / dt,
            "logz": r.logz, "logz_err": r.logz_err,
            "max_lnL_found": float(r.dead_logl.max()), "lnL_at_truth": l_truth,
            "accuracy": {"median_lnL": lbar, "q": float(q), "q_at_truth": float(q_truth),
                         "passes": bool(q >= 0.01)}}


def masks_leg(fgl, steps, warmup, tune):
    """The crossed-mask model (amplitude masks x spectral-index masks,
    Eq. fast_forward_model with alpha) at the headline shape: 2 x 16 masks,
    F=301, T=96, B=16384, each precision timed like the headline."""
    import torch
    import workload
    w = workload.masks_config()
    m = fgl.Model.from_workload(w)
    th = torch.from_numpy(w.theta).cuda()
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    res = {"workload": w.name, "n_alpha": w.n_alpha, "n_beta": w.N // w.n_alpha,
           "P": w.P, "form": m.form}
    for prec in PRECS:
        if tune:
            m.tune(w.B, prec)
        r = time_prec(fgl, m, th, out, prec, steps, warmup)
        res[prec] = {"value": r["evals_per_s"], "ms_per_step": r["ms_per_step"],
                     "kernel_ms": r["kernel_ms"],
                     "tile": dict(zip(("waves", "chans", "occupancy"), m.tile(w.B, prec)))}
        log(f"masks {prec}: {r['evals_per_s']:.4e} evals/s, kernel {r['kernel_ms']:.4f} ms")
    flops = w.B * (3.0 * w.F * w.T + EXP_FLOPS * w.N * w.F)
    res["roofline_frac"] = flops / (res["mixed"]["kernel_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
    res["mixed_over_fp32"] = res["mixed"]["value"] / res["fp32"]["value"]
    m.close()
    return res


def small_batch_leg(fgl, calls=200):
    """The launch-bound workloads (N4_F151_T1_B1000 and N16_F151_T20_B4096):
    median latency of a synchronous host-pointer call (θ in, lnL out over
    PCIe, the call's kernels replayed from a captured hipGraph) and the time
    per device-pointer call enqueued back to back, for each precision."""
    import torch
    import workload
    out = {}
    for k in (workload.SMALL, workload.MEDIUM):
        w = workload.config(k)
        m = fgl.Model.from_workload(w)
        th = torch.from_numpy(w.theta).cuda()
        o = torch.empty(w.B, dtype=torch.float64, device="cuda")
        r = {"B": w.B}
        for prec in PRECS:
            for _ in range(3):
                m.loglike(w.theta, prec)                   # eager, capture, replay
            lat = []
            for _ in range(calls):
                t0 = time.perf_counter()
                m.loglike(w.theta, prec)
                lat.append(time.perf_counter() - t0)
            host_us = float(np.median(lat)) * 1e6
            for _ in range(3):
                m.loglike_device(th, o, prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(calls):
                m.loglike_device(th, o, prec)
            torch.cuda.synchronize()
            dev_us = (time.perf_counter() - t0) / calls * 1e6
            r[prec] = {"host_call_median_us": host_us, "device_call_us": dev_us,
                       "evals_per_s_device": w.B / (dev_us * 1e-6)}
        m.close()
        # the device call replayed from captured graphs (FGL_DEVICE_GRAPHS=1)
        os.environ["FGL_DEVICE_GRAPHS"] = "1"
        mg = fgl.Model.from_workload(w)
        del os.environ["FGL_DEVICE_GRAPHS"]
        for _ in range(3):
            mg.loglike_device(th, o, "mixed")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            mg.loglike_device(th, o, "mixed")
        torch.cuda.synchronize()
        r["mixed"]["device_call_us_graph_replay"] = (time.perf_counter() - t0) / calls * 1e6
        mg.close()
        out[w.name] = r
    return out


def grad_leg(fgl, w, steps, warmup):
    """lnL and its gradient (FP64) for the headline rows, timed like the
    likelihood: grads/s and the gradient kernel's average time."""
    import torch
    m = fgl.Model.from_workload(w)
    th = torch.from_numpy(w.theta).cuda()
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    grad = torch.empty((w.B, w.P), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        m.loglike_grad_device(th, out, grad)
    torch.cuda.synchronize()
    m.kernel_timing(True, every=TIMING_EVERY)
    t0 = time.perf_counter()
    for _ in range(steps):
        m.loglike_grad_device(th, out, grad)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, n = m.kernel_time()
    m.kernel_timing(False)
    form = m.form
    m.close()
    k = kms / max(n, 1)
    # algorithmic FP64 work of the two contractions per row: the model over
    # the matrix rows (N + 1 projected rows, or T time bins) and the
    # transposed product K^T r, 2 flop per multiply-add each
    rows = w.N + 1 if form == "projected" else w.T
    flops = 4.0 * rows * w.N * w.F * w.B
    achieved = flops / (k * 1e-3) / 1e12
    return {"value": w.B * steps / dt, "unit": "gradients/s", "ms_per_step": dt * 1e3 / steps,
            "kernel_ms": k, "kernel": "k_grad64", "precision": "fp64", "form": form,
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                         "work": "4 (N+1) N F flop per row: model and transposed product"}}


def regions_leg(fgl, n_regions=32):
    """Region construction upstream of the likelihood (Sec. 4, Eq.
    chromatic_function) on the synthetic 256 x 512 sky, 301 channels, 96
    LST steps: beam-weighted importance map, recursive partition into
    n_regions regions, and the chromatic functions K [N][F][T]."""
    from workload.sky import sky_config, SKY_NAME
    s = sky_config()
    sm = fgl.SkyModel.from_sky(s)
    sm.importance(s.shifts, "beam")                       # warm-up
    t0 = time.perf_counter()
    imp = sm.importance(s.shifts, "beam")
    t1 = time.perf_counter()
    edges = fgl.fgl_partition(s.beta, imp, n_regions, "recursive")
    t2 = time.perf_counter()
    sm.chromatic(edges, s.shifts)                         # warm-up
    t3 = time.perf_counter()
    sm.chromatic(edges, s.shifts)
    t4 = time.perf_counter()
    kms = sm.kernel_ms()
    sm.close()
    npix = s.nlat * s.nlon
    flops = 2.0 * s.F * s.T * npix                        # one FMA per (pixel, channel, step)
    achieved = flops / (kms * 1e-3) / 1e12
    return {"workload": SKY_NAME, "pixels": npix, "regions": n_regions,
            "importance_s": t1 - t0, "partition_s": t2 - t1, "chromatic_s": t4 - t3,
            "chromatic_kernel_ms": kms,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                         "kernel": "k_sky_k"}}


def noise_leg(fgl, n=301 * 96, R=4096, reps=20, sigma=0.025):
    """Reference distribution of the accuracy criterion (Sec. 5): lnL of R
    data sets that the model describes up to 25 mK Gaussian noise, n
    residuals each (the 301-channel, 96-bin grid), drawn and reduced on the
    device.  The median over reps calls of the kernel's duration."""
    fgl.fgl_noise_loglike(n, R, sigma, sigma, 0)                 # warm-up
    kms = []
    t0 = time.perf_counter()
    for i in range(reps):
        kms.append(fgl.fgl_noise_loglike(n, R, sigma, sigma, i + 1, timed=True)[1])
    dt = (time.perf_counter() - t0) / reps
    k = float(np.median(kms))
    return {"realisations": R, "residuals": n, "kernel": "k_noise_lnl", "kernel_ms": k,
            "call_ms": dt * 1e3, "realisations_per_s": R / (k * 1e-3),
            "normals_per_s": R * n / (k * 1e-3)}


def _margins(got, ref, theta, n_ft):
    """|dlnL| against each bar: the mixed tolerance, and for FP64 1e-9 |lnL|
    (1e-9 S where the chi-square term and the normalisation cancel to less
    than a tenth of their magnitude S)."""
    fin = np.isfinite(ref)
    got, ref = np.asarray(got)[fin], np.asarray(ref)[fin]
    sig = np.asarray(theta)[fin, -1]
    d = np.abs(got - ref)
    tol_m = 1e-6 * np.abs(ref) + 1e-3
    norm = -0.5 * n_ft * np.log(2.0 * np.pi * sig * sig)
    S = np.abs(ref - norm) + np.abs(norm)
    tol_64 = 1e-9 * np.where(np.abs(ref) >= 0.1 * S, np.abs(ref), S)
    return d, tol_m, tol_64


def parity_record(fgl, orc, name, rows=1024):
    """Every precision and form against the oracle on the named workload's
    posterior shell (the regime where precision bites) and on the shell of
    its full-rank variant (several time harmonics and a per-value scatter
    per region): max |dlnL|, max and p99 of |dlnL| / tolerance, pass/fail."""
    import workload
    out = {}
    for label, rich in (("shell", False), ("shell_full_rank", True)):
        w = workload.posterior_shell(name, rows, rich=rich)
        ref = orc.loglike_w(w)
        rec = {"rows": w.B}
        models = {"": fgl.Model.from_workload(w),
                  "direct": fgl.Model.from_workload(w, fgl.FGL_MIXED_DIRECT),
                  "plain_projected": fgl.Model.from_workload(w, fgl.FGL_PLAIN_PROJECTED)}
        evals = {"mixed_" + models[""].form: models[""].loglike(w.theta, "mixed"),
                 "mixed_direct": models["direct"].loglike(w.theta, "mixed"),
                 "fp64_direct": models["direct"].loglike(w.theta, "fp64"),
                 "fp64_projected": models["plain_projected"].loglike(w.theta, "fp64"),
                 "fp32_direct": models["direct"].loglike(w.theta, "fp32"),
                 "fp32_projected": models["plain_projected"].loglike(w.theta, "fp32")}
        for mm in models.values():
            mm.close()
        for key, got in evals.items():
            d, tol_m, tol_64 = _margins(got, ref, w.theta, w.F * w.T)
            r = {"max_abs_dlogL": float(d.max())}
            if key.startswith("fp64"):
                r.update(max_over_fp64_bar=float((d / tol_64).max()),
                         within_fp64_bar=bool(np.all(d <= tol_64)))
            else:
                r.update(max_over_mixed_tol=float((d / tol_m).max()),
                         p99_over_mixed_tol=float(np.quantile(d / tol_m, 0.99)),
                         within_mixed_tol=bool(np.all(d <= tol_m)))
            rec[key] = r
        out[label] = rec
    out["bars"] = {"mixed": "1e-6|lnL| + 1e-3",
                   "fp64": "1e-9|lnL| (1e-9 S on rows whose two terms cancel below S/10)",
                   "fp32": "reported against the mixed tolerance"}
    return out


def large_leg(fgl, orc, steps, warmup, tune):
    """N=64, F=401 (50-250 MHz), T=240, B=65536: the mixed kernel in both
    forms against plain FP32 in both forms, the oracle on 256 prior and 256
    posterior-shell rows, and the mixed kernel's roofline."""
    import torch
    import workload
    w = workload.config(workload.LARGE)
    th = torch.from_numpy(w.theta).cuda()
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    res, outs = {}, {}
    for label, flags, precs in (("", 0, ("mixed",)),
                                ("direct", fgl.FGL_MIXED_DIRECT, ("mixed", "fp32")),
                                ("plain_projected", fgl.FGL_PLAIN_PROJECTED, ("fp32",))):
        m = fgl.Model.from_workload(w, flags)
        form = m.form
        for prec in precs:
            if tune:
                m.tune(w.B, prec)
            key = f"{prec}_{form}" if prec == "mixed" else f"{prec}_{'projected' if label == 'plain_projected' else 'direct'}"
            res[key] = time_prec(fgl, m, th, out, prec, steps, warmup)
            outs[key] = out.cpu().numpy().copy()
            log(f"large {key}: {res[key]['evals_per_s']:.4e} evals/s, kernel {res[key]['kernel_ms']:.4f} ms")
        m.close()
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.sort(rng.choice(w.B, 256, replace=False))
    ref = orc.loglike_w(w, w.theta[idx])
    line = {"workload": w.name, "N": w.N, "F": w.F, "T": w.T, "B": w.B}
    for key, r in res.items():
        d, tol_m, _ = _margins(outs[key][idx], ref, w.theta[idx], w.F * w.T)
        line[key] = {"value": r["evals_per_s"], "ms_per_step": r["ms_per_step"],
                     "kernel_ms": r["kernel_ms"],
                     "prior_rows_max_over_mixed_tol": float((d / tol_m).max())}
    sh = workload.posterior_shell(workload.LARGE, 256)
    ref_sh = orc.loglike_w(sh)
    for label, flags, prec in (("mixed_projected", 0, "mixed"),
                               ("mixed_direct", fgl.FGL_MIXED_DIRECT, "mixed"),
                               ("fp32_direct", fgl.FGL_MIXED_DIRECT, "fp32")):
        m = fgl.Model.from_workload(sh, flags)
        d, tol_m, _ = _margins(m.loglike(sh.theta, prec), ref_sh, sh.theta, sh.F * sh.T)
        m.close()
        line.setdefault(label, {})["shell_rows_max_over_mixed_tol"] = float((d / tol_m).max())
    mix = res["mixed_projected"]
    flops = w.B * (3.0 * w.F * w.T + EXP_FLOPS * w.N * w.F)
    achieved = flops / (mix["kernel_ms"] * 1e-3) / 1e12
    line["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                        "kernel": "k_mixed", "kernel_ms": mix["kernel_ms"]}
    line["mixed_over_fp32"] = {
        "projected_vs_direct": mix["evals_per_s"] / res["fp32_direct"]["evals_per_s"],
        "direct_vs_direct": res["mixed_direct"]["evals_per_s"] / res["fp32_direct"]["evals_per_s"],
        "projected_vs_projected": mix["evals_per_s"] / res["fp32_projected"]["evals_per_s"]}
    line["oracle_sample"] = "256 prior rows of the batch and 256 posterior-shell rows"
    return line


def cpu_leg(w, gpu_out, seconds):
    import oracle
    orc = oracle.load()
    cores = orc.max_threads()
    n = min(w.B, 256)
    t0 = time.perf_counter()
    ref = orc.loglike_w(w, w.theta[:n])
    dt = time.perf_counter() - t0
    target = int(n * seconds / max(dt, 1e-6))
    n2 = int(min(w.B, max(n, target)))
    if n2 > n:
        t0 = time.perf_counter()
        ref = orc.loglike_w(w, w.theta[:n2])
        dt = time.perf_counter() - t0
        n = n2
    # when the whole batch takes less than `seconds`, time repeated passes
    passes = max(1, int(round(seconds / max(dt, 1e-6)))) if n == w.B else 1
    if passes > 1:
        t0 = time.perf_counter()
        for _ in range(passes):
            orc.loglike_w(w, w.theta[:n])
        dt = time.perf_counter() - t0
    d = np.abs(gpu_out[:n] - ref)
    tol = 1e-6 * np.abs(ref) + 1e-3
    # the same oracle on one host thread, over about a fifth of the time
    # (last: the thread count stays set for the process)
    n1 = max(1, min(w.B, int(n * passes / dt / max(cores, 1) * seconds / 5)))
    t0 = time.perf_counter()
    orc.loglike_w(w, w.theta[:n1], threads=1)
    dt1 = time.perf_counter() - t0
    return ({"value": n * passes / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
             "sample": f"first {n} of the {w.B} rows x {passes} passes, all host threads",
             "seconds": dt,
             "single_thread": {"value": n1 / dt1, "unit": "evals/s",
                               "sample": f"first {n1} rows, one host thread", "seconds": dt1}},
            {"rows": n, "max_abs_dlogL": float(d.max()),
             "max_dlogL_over_tol": float((d / tol).max()),
             "p99_dlogL_over_tol": float(np.quantile(d / tol, 0.99)),
             "within_tol": bool(np.all(d <= tol))})


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; "
                                   "--gpus N with N > 1 is not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import workload
    from paper_2603_13196_amd import fgl
    torch.cuda.set_device(0)
    if a.calib_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": src.numel() * 8, "copies": 3}))
        return
    w = workload.config(a.workload)
    log(f"workload {w.name}: N={w.N} F={w.F} T={w.T} B={w.B}")
    m = fgl.Model.from_workload(w)
    th = torch.from_numpy(w.theta).cuda()
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    if not a.no_tune:
        for prec in (("mixed",) if a.no_plain else ("mixed", "fp32", "fp64")):
            if prec == "mixed" and a.tile:
                continue
            m.tune(w.B, prec)
    if a.tile:
        wv, fc, occ = (int(x) for x in a.tile.split(","))
        m.set_tile(w.B, "mixed", wv, fc, occ)
    res, outs = {}, {}
    for prec in (("mixed",) if a.no_plain else ("mixed", "fp32", "fp64")):
        res[prec] = time_prec(fgl, m, th, out, prec, a.steps, a.warmup)
        outs[prec] = out.cpu().numpy().copy()
        log(f"{prec}: {res[prec]['evals_per_s']:.4e} evals/s, "
            f"{res[prec]['ms_per_step']:.4f} ms/step, kernel {res[prec]['kernel_ms']:.4f} ms")
    gpu_out = outs["mixed"]
    form = m.form
    if not a.no_plain and form == "projected":
        # the same mixed evaluation in its direct form, and the plain
        # precisions in the projected form, for like-for-like ratios
        md = fgl.Model.from_workload(w, fgl.FGL_MIXED_DIRECT)
        if not a.no_tune:
            md.tune(w.B, "mixed")
        res["mixed_direct"] = time_prec(fgl, md, th, out, "mixed", a.steps, a.warmup)
        md.close()
        log(f"mixed (direct form): {res['mixed_direct']['evals_per_s']:.4e} evals/s")
        mp = fgl.Model.from_workload(w, fgl.FGL_PLAIN_PROJECTED)
        for prec in ("fp32", "fp64"):
            if not a.no_tune:
                mp.tune(w.B, prec)
            res[prec + "_projected"] = time_prec(fgl, mp, th, out, prec, a.steps, a.warmup)
            outs[prec + "_projected"] = out.cpu().numpy().copy()
            log(f"{prec} (projected form): {res[prec + '_projected']['evals_per_s']:.4e} evals/s, "
                f"kernel {res[prec + '_projected']['kernel_ms']:.4f} ms")
        mp.close()
    mix = res["mixed"]
    # roofline of the likelihood kernel: FP64 work the method needs per
    # evaluation (residual and chi-square: 3 F T; power laws: N F values at
    # EXP_FLOPS each) over the kernel's average launch time
    flops = w.B * (3.0 * w.F * w.T + EXP_FLOPS * w.N * w.F)
    achieved = flops / (mix["kernel_ms"] * 1e-3) / 1e12
    # as designed: the kernel's int8 digit products on the matrix cores
    # (21 v_mfma_i32_32x32x32_i8 per 32-row tile, region chunk and matrix tile
    # in the projected form, 18 in the direct form), against the int8 peak
    kc = (w.N + 31) // 32
    if form == "projected":
        peel = 1 if w.N % 32 == 0 else 0
        mt, prods = (w.N + 1 - peel + 31) // 32, 21
    else:
        mt, prods = (w.T + 31) // 32, 18
    bpad = max(256, (w.B + 255) // 256 * 256)
    mfma_ops = (bpad // 32) * w.F * kc * mt * prods * 2.0 * 32 * 32 * 32
    mfma_tops = mfma_ops / (mix["kernel_ms"] * 1e-3) / 1e12
    src = open(os.path.join(ROOT, "paper_2603_13196_amd", "csrc", "fgl_kernels.hip"), "rb").read()
    traffic = traffic_from_profiles(hashlib.sha256(src).hexdigest())
    tiles = {p: dict(zip(("waves", "chans", "occupancy"), m.tile(w.B, p))) for p in res if p in PRECS}
    line = {
        "metric": "logL evals/s at N=32,F=301,T=96 (mixed vs plain); serve p50/p99 latency",
        "value": mix["evals_per_s"], "unit": "evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": mix["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8-mfma+f64", "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "F": w.F, "T": w.T, "B": w.B,
                   "precision": "mixed", "form": form, "tiles": tiles,
                   "tuned": not a.no_tune},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic, "kernel": "k_mixed",
                     # the counted HBM bytes over the event-timed kernel time
                     "traffic_gbs": (traffic / (mix["kernel_ms"] * 1e-3) / 1e9
                                     if traffic else None),
                     "traffic_frac_of_hbm": (traffic / (mix["kernel_ms"] * 1e-3) / PEAK_HBM_BPS
                                             if traffic else None),
                     "kernel_ms": mix["kernel_ms"],
                     "as_designed": {"int8_mfma": mfma_tops, "peak": PEAK_INT8_TOPS,
                                     "unit": "TOP/s", "frac": mfma_tops / PEAK_INT8_TOPS}},
    }
    def rate(key):
        return {"value": res[key]["evals_per_s"], "ms_per_step": res[key]["ms_per_step"],
                "kernel_ms": res[key]["kernel_ms"]}
    if "fp32" in res:
        line["plain_fp32"] = rate("fp32")
        line["plain_fp64"] = rate("fp64")
        # the headline ratio: the mixed path as run against the paper's
        # formulation in plain FP32 (the model on the time grid)
        line["mixed_over_fp32"] = mix["evals_per_s"] / res["fp32"]["evals_per_s"]
    if "mixed_direct" in res:
        line["mixed_direct_form"] = rate("mixed_direct")
        line["plain_fp32_projected"] = rate("fp32_projected")
        line["plain_fp64_projected"] = rate("fp64_projected")
        line["like_for_like"] = {
            "direct": {"mixed_over_fp32": res["mixed_direct"]["evals_per_s"] / res["fp32"]["evals_per_s"],
                       "mixed_over_fp64": res["mixed_direct"]["evals_per_s"] / res["fp64"]["evals_per_s"]},
            "projected": {"mixed_over_fp32": mix["evals_per_s"] / res["fp32_projected"]["evals_per_s"],
                          "mixed_over_fp64": mix["evals_per_s"] / res["fp64_projected"]["evals_per_s"]}}
    m.close()
    if not a.no_small and not a.no_plain:
        log("small-batch leg")
        line["small_batch"] = small_batch_leg(fgl)
    if not a.no_grad and not a.no_plain:
        log("gradient leg")
        line["gradient"] = grad_leg(fgl, w, a.steps, a.warmup)
    if not a.no_large and not a.no_plain:
        import oracle
        log("large-workload leg")
        line["large"] = large_leg(fgl, oracle.load(), max(20, a.steps // 10),
                                  max(10, a.warmup // 10), not a.no_tune)
    if not a.no_masks and not a.no_plain:
        log("crossed-mask leg")
        line["masks"] = masks_leg(fgl, a.steps, a.warmup, not a.no_tune)
    if not a.no_regions and not a.no_plain:
        log("region construction leg")
        line["region_construction"] = regions_leg(fgl)
    if not a.no_noise and not a.no_plain:
        log("noise reference leg")
        line["noise_reference"] = noise_leg(fgl)
    if not a.no_serve:
        log("serving leg")
        line["serving"] = serving_leg(fgl, a.serve_seconds, a.serve_configs)
    if not a.no_sampler:
        log("nested sampling leg")
        line["nested_sampling"] = [sampler_leg(fgl, 10, 1), sampler_leg(fgl, 10, 72)]
    if not a.no_cpu:
        import oracle
        log("cpu baseline leg")
        cb, par = cpu_leg(w, gpu_out, a.cpu_seconds)
        line["cpu_baseline"] = cb
        # the prior rows of the timed batch (every precision timed above),
        # then the posterior shells
        ref = oracle.load().loglike_w(w, w.theta[:par["rows"]])
        prior = {"rows": par["rows"]}
        for key, got in outs.items():
            d, tol_m, tol_64 = _margins(got[:par["rows"]], ref, w.theta[:par["rows"]], w.F * w.T)
            prior[key] = ({"max_abs_dlogL": float(d.max()),
                           "max_over_fp64_bar": float((d / tol_64).max()),
                           "within_fp64_bar": bool(np.all(d <= tol_64))}
                          if key.startswith("fp64") else
                          {"max_abs_dlogL": float(d.max()),
                           "max_over_mixed_tol": float((d / tol_m).max()),
                           "p99_over_mixed_tol": float(np.quantile(d / tol_m, 0.99)),
                           "within_mixed_tol": bool(np.all(d <= tol_m))})
        log("parity record leg")
        par = {"prior": prior}
        par.update(parity_record(fgl, oracle.load(), w.name))
        line["parity_vs_oracle"] = par
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
