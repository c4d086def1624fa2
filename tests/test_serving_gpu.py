"""GPU serving: continuous batching through the C-ABI (fgl_serve_*).

A served result must not depend on what else runs with it: each request's
output is compared bitwise with the same rows evaluated alone through
fgl_loglike_batch, and sampled rows with the oracle.  Admission by HBM
budget with eviction, a model larger than the budget, a host-forced
failure, destroying a busy model or server, and the argument errors are
exercised from the host; no case makes a kernel fail.
"""
import os
import time

import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import check, lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fgl():
    return lib()


def _wait(srv, tickets, timeout_s=120.0):
    """Poll until every ticket is done; returns {ticket: out or FGLError}."""
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < len(tickets):
        for t in tickets:
            if t in got:
                continue
            try:
                r = srv.poll(t)
            except Exception as e:          # a failed request reports done
                got[t] = e
                continue
            if r is not None:
                got[t] = r[0]
        assert time.time() < t_end, f"{len(tickets) - len(got)} requests never completed"
        time.sleep(1e-4)
    return got


def _requests(clients, per_client, seed):
    """(client index, rows, precision) for every request, interleaved."""
    rng = np.random.Generator(np.random.PCG64(seed))
    precs = ("mixed", "mixed", "fp64", "fp32")
    reqs = []
    for k in range(per_client):
        for ci, c in enumerate(clients):
            B = c.batches[k % len(c.batches)]
            rows = np.sort(rng.choice(c.work.B, size=B, replace=False))
            reqs.append((ci, rows, precs[(ci + k) % len(precs)]))
    return reqs


def _run_mix(fgl, clients, models, reqs, budget, inflight, share=1):
    """Submit every request to a held server, release it (the whole queue is
    then planned at once), and return the outputs in request order and the
    server's launch counters."""
    srv = fgl.Server(budget_bytes=budget, max_inflight=inflight)
    srv.set_sharing(share)
    thetas = [np.ascontiguousarray(clients[ci].work.theta[rows]) for ci, rows, _ in reqs]
    srv.hold(True)
    tickets = [srv.submit(models[ci], th, prec) for (ci, _, prec), th in zip(reqs, thetas)]
    with pytest.raises(RuntimeError):
        srv.drain()                  # held with requests queued: FGL_EAGAIN
    srv.hold(False)
    got = _wait(srv, tickets)
    srv.drain()
    stats = srv.stats()
    srv.close()
    return [got[t] for t in tickets], stats


def test_mix_equals_alone(fgl):
    """Twelve clients of the serving mix (N 4..40, T 1..96, F 151/301, both
    forms of the mixed evaluation), three requests each with mixed, FP64 and
    FP32 rows, two slots so that requests queue and merge: every served
    result is bitwise the result of the same rows alone."""
    clients = workload.serving_clients(12, n_requests=3, min_B=1, max_B=3000)
    models = [fgl.Model.from_workload(c.work) for c in clients]
    say("forms: " + " ".join(f"N{c.work.N}T{c.work.T}:{m.form}" for c, m in zip(clients, models)))
    reqs = _requests(clients, 3, seed=11)
    served, _ = _run_mix(fgl, clients, models, reqs, budget=0, inflight=2)
    orc = oracle.load()
    for (ci, rows, prec), out in zip(reqs, served):
        assert not isinstance(out, Exception), out
        alone = models[ci].loglike(clients[ci].work.theta[rows], prec)
        assert np.array_equal(out, alone), (ci, prec, rows.size)
    # the same requests with launches shared by models of one kernel variant
    shared, stats = _run_mix(fgl, clients, models, reqs, budget=0, inflight=2, share=16)
    say(f"  sharing: launches {stats[0]}, shared {stats[1]} carrying {stats[2]} model groups")
    assert stats[1] >= 1 and stats[2] >= 2 * stats[1]
    for (ci, rows, prec), out, ref in zip(reqs, shared, served):
        assert np.array_equal(out, ref), (ci, prec, rows.size)
    # sampled rows of the mixed requests against the oracle
    for (ci, rows, prec), out in zip(reqs[:12], served[:12]):
        if prec != "mixed":
            continue
        w = clients[ci].work
        sub = rows[:16]
        ref = orc.loglike_w(w, w.theta[sub])
        check(out[:16], ref, "mixed", f"served client {ci}")
    for m in models:
        m.close()


@pytest.mark.parametrize("share,budgeted", [(1, True), (16, True), (16, False)])
def test_full_mix_equals_alone(fgl, share, budgeted):
    """All 64 clients of the serving mix (N 4..40, T 1..96, F 151/301, B up
    to 8192), two requests each in mixed, FP64 and FP32, four slots, with
    and without shared launches, and with an HBM budget of half the models'
    bytes (waits and evictions) or none: every served result is bitwise the
    same rows alone.  The requests are submitted to a held server and
    released together; without a budget, shared launches must then occur
    (under it, models with requests in flight cannot be evicted, so a
    candidate model rarely fits beside the first)."""
    clients = workload.serving_clients(64, n_requests=2)
    models = [fgl.Model.from_workload(c.work) for c in clients]
    total = sum(m.nbytes for m in models)
    # half the models' bytes (at least the largest model)
    budget = max(total // 2, max(m.nbytes for m in models)) if budgeted else 0
    reqs = _requests(clients, 2, seed=13)
    served, stats = _run_mix(fgl, clients, models, reqs, budget=budget, inflight=4,
                             share=share)
    say(f"  64-client mix, share {share}: {len(reqs)} requests, budget {budget} of {total} "
        f"bytes, launches {stats[0]}, shared {stats[1]} ({stats[2]} groups)")
    for (ci, rows, prec), out in zip(reqs, served):
        assert not isinstance(out, Exception), out
        alone = models[ci].loglike(clients[ci].work.theta[rows], prec)
        assert np.array_equal(out, alone), (ci, prec, rows.size)
    if share > 1 and not budgeted:
        assert stats[1] >= 1
    for m in models:
        m.close()


def test_budget_admission_and_eviction(fgl):
    """An HBM budget of about two models for six: requests wait for room,
    idle models are evicted and re-uploaded, results are unchanged."""
    clients = workload.serving_clients(6, n_requests=2, seed=99, min_B=64, max_B=2048)
    models = [fgl.Model.from_workload(c.work) for c in clients]
    sizes = sorted(m.nbytes for m in models)
    budget = sizes[-1] + sizes[-2]
    say(f"model bytes {sizes}, budget {budget}")
    reqs = _requests(clients, 2, seed=12)
    served, _ = _run_mix(fgl, clients, models, reqs, budget=budget, inflight=3)
    for (ci, rows, prec), out in zip(reqs, served):
        assert not isinstance(out, Exception), out
        alone = models[ci].loglike(clients[ci].work.theta[rows], prec)
        assert np.array_equal(out, alone), (ci, prec)
    # a model larger than the whole budget is refused at submission
    srv = fgl.Server(budget_bytes=sizes[0] // 2, max_inflight=1)
    bi = max(range(len(models)), key=lambda i: models[i].nbytes)
    with pytest.raises(fgl.FGLError) as e:
        srv.submit(models[bi], clients[bi].work.theta[:1])
    assert e.value.code == fgl.FGL_EAGAIN
    srv.close()
    for m in models:
        m.close()


def test_forced_failure_is_reported(fgl, monkeypatch):
    """The request named by FGL_SERVE_FAIL_TICKET fails from the host; the
    others complete normally."""
    monkeypatch.setenv("FGL_SERVE_FAIL_TICKET", "3")
    w = workload.config(workload.MEDIUM, B=1024)
    m = fgl.Model.from_workload(w)
    srv = fgl.Server(max_inflight=2)
    tickets = [srv.submit(m, w.theta[k * 100:(k + 1) * 100]) for k in range(6)]
    got = _wait(srv, tickets)
    for k, t in enumerate(tickets):
        if t == 3:
            assert isinstance(got[t], fgl.FGLError) and got[t].code == fgl.FGL_EDEVICE
        else:
            assert np.array_equal(got[t], m.loglike(w.theta[k * 100:(k + 1) * 100]))
    srv.close()
    m.close()


def test_destroy_while_busy(fgl):
    """fgl_model_destroy and fgl_serve_destroy return FGL_EBUSY, freeing
    nothing, while requests on them are queued (the server is held, so they
    stay queued) or running; after release and a drain both succeed and the
    completions stay pollable until then."""
    ws = workload.config(workload.SMALL, B=256)
    small = fgl.Model.from_workload(ws)
    srv = fgl.Server(max_inflight=1)
    srv.hold(True)
    ts = [srv.submit(small, ws.theta) for _ in range(3)]
    rc = fgl._lib.fgl_model_destroy(small.handle)
    assert rc == fgl.FGL_EBUSY, rc
    rc = fgl._lib.fgl_serve_destroy(srv.handle)
    assert rc == fgl.FGL_EBUSY, rc
    assert fgl._lib.fgl_serve_drain(srv.handle) == fgl.FGL_EAGAIN
    srv.hold(False)
    srv.drain()
    got = _wait(srv, ts)
    for t in ts:
        assert np.array_equal(got[t], small.loglike(ws.theta))
    srv.close()
    small.close()


def test_cancel_and_wait_limit(fgl):
    """A queued request can be cancelled (its poll reports FGL_ECANCELED and
    nothing is written); a launched or completed one cannot (FGL_EBUSY).
    With a wait limit, requests still queued past it (the server is held)
    report FGL_ETIMEDOUT; the others' results are unchanged."""
    ws = workload.config(workload.SMALL, B=256)
    m = fgl.Model.from_workload(ws)
    ref = m.loglike(ws.theta)
    srv = fgl.Server(max_inflight=2)
    srv.hold(True)
    ts = [srv.submit(m, ws.theta) for _ in range(3)]
    srv.cancel(ts[1])
    with pytest.raises(fgl.FGLError) as e:
        srv.cancel(ts[1])
    assert e.value.code == fgl.FGL_EBUSY
    with pytest.raises(fgl.FGLError) as e:
        srv.poll(ts[1])
    assert e.value.code == fgl.FGL_ECANCELED
    srv.hold(False)
    srv.drain()
    with pytest.raises(fgl.FGLError) as e:
        srv.cancel(ts[0])
    assert e.value.code == fgl.FGL_EBUSY
    got = _wait(srv, [ts[0], ts[2]])
    assert np.array_equal(got[ts[0]], ref) and np.array_equal(got[ts[2]], ref)
    # wait limit
    srv.set_timeout(3000.0)
    srv.hold(True)
    ts = [srv.submit(m, ws.theta) for _ in range(2)]
    for t in ts:
        t_end = time.time() + 5.0
        while True:
            try:
                r = srv.poll(t)
            except fgl.FGLError as err:
                assert err.code == fgl.FGL_ETIMEDOUT, err
                break
            assert r is None, "a held request completed"
            assert time.time() < t_end, "no timeout reported"
            time.sleep(0.001)
    srv.hold(False)
    srv.set_timeout(0.0)
    t = srv.submit(m, ws.theta)
    srv.drain()
    assert np.array_equal(_wait(srv, [t])[t], ref)
    srv.close()
    m.close()
    say("cancel and wait limit: ok")


def test_serving_argument_errors(fgl):
    w = workload.config(workload.SMALL, B=8)
    m = fgl.Model.from_workload(w)
    with pytest.raises(fgl.FGLError):
        fgl.Server(max_inflight=0)
    srv = fgl.Server(max_inflight=1)
    with pytest.raises(fgl.FGLError) as e:
        fgl.fgl_serve_submit(srv.handle, m.handle, w.theta, 0, np.empty(1), "mixed")
    assert e.value.code == fgl.FGL_EINVAL
    with pytest.raises(fgl.FGLError) as e:
        fgl.fgl_serve_submit(srv.handle, m.handle, w.theta, 8, np.empty(8), 9)
    assert e.value.code == fgl.FGL_EINVAL
    with pytest.raises(fgl.FGLError) as e:
        fgl.fgl_serve_poll(srv.handle, 12345)
    assert e.value.code == fgl.FGL_EINVAL
    t = srv.submit(m, w.theta)
    got = _wait(srv, [t])
    assert np.array_equal(got[t], m.loglike(w.theta))
    with pytest.raises(fgl.FGLError):       # retired by the poll that reported it
        fgl.fgl_serve_poll(srv.handle, t)
    srv.close()
    m.close()
    assert os.environ.get("FGL_SERVE_FAIL_TICKET") is None
