"""Batched nested slice sampling: the sampler that drives the likelihood.

Nested sampling (Sec. 3.1.2) evolves n live points drawn from the prior; each
iteration discards the b lowest-likelihood points at once and replaces them
by b independent slice-sampling chains constrained to lnL > lnL*, where lnL*
is the largest likelihood of the discarded batch.  The expected log prior
volume shrinks by sum_{i<b} 1/(n - i) per iteration (Eq. log_xgpu), and the
evidence is the sum of the discarded likelihoods weighted by the volume each
one closes (Eq. evidence_sum).

Each new point starts from a randomly chosen surviving live point and takes
`num_inner_steps` hit-and-run slice steps (Sec. 3.1.3): a direction drawn
uniformly in the geometry whitened by the live points' covariance (a
Cholesky factor), a unit-width interval placed at a random offset around
the current point, stepping out until both ends leave the constrained
region, then shrinking until a point inside is found.  The target within
the constraint is the prior, which is uniform in the sampler's coordinates
(a box), so a proposal is inside when it lies in the box and its
likelihood exceeds lnL*.

All chains advance together: every round proposes one point per unfinished
chain and evaluates the round's proposals in one batched likelihood call,
which is what feeds the GPU.  Random numbers come from numpy's PCG64, so a
run is reproducible from its seed for a given likelihood.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

# chain stages
_LEFT, _RIGHT, _SHRINK, _DONE = 0, 1, 2, 3


@dataclass
class NSResult:
    logz: float                     # log evidence
    logz_err: float                 # sqrt(H / n_live)
    information: float              # H, nats
    dead: np.ndarray                # [n_dead, d] discarded points (sampler coordinates)
    dead_logl: np.ndarray           # [n_dead]
    log_weights: np.ndarray         # [n_dead + n_live] normalised posterior log weights
    samples: np.ndarray             # [n_dead + n_live, d] dead points then final live points
    sample_logl: np.ndarray         # [n_dead + n_live] lnL of each sample
    n_like: int                     # likelihood evaluations
    n_calls: int                    # batched likelihood calls
    iterations: int
    seconds: float
    logx: List[float] = field(default_factory=list)   # log X after each iteration

    def posterior_mean(self) -> np.ndarray:
        w = np.exp(self.log_weights - self.log_weights.max())
        return (w[:, None] * self.samples).sum(0) / w.sum()

    def posterior_cov(self) -> np.ndarray:
        w = np.exp(self.log_weights - self.log_weights.max())
        w = w / w.sum()
        mu = (w[:, None] * self.samples).sum(0)
        x = self.samples - mu
        return (w[:, None] * x).T @ x

    def median_loglike(self) -> float:
        """Median of lnL under the posterior weights: the fit's median a
        posteriori likelihood that the accuracy criterion (Sec. 5) compares
        with the noise-only reference distribution.  The smallest sample lnL
        at which the posterior mass of lnL <= it reaches one half."""
        order = np.argsort(self.sample_logl, kind="stable")
        w = np.exp(self.log_weights[order] - self.log_weights.max())
        c = np.cumsum(w)
        k = int(np.searchsorted(c, 0.5 * c[-1], side="left"))
        return float(self.sample_logl[order][k])


def expected_logx_decrement(n: int, b: int) -> float:
    """Expected log-volume contraction of one iteration that discards the b
    lowest of n live points (Eq. log_xgpu): -sum_{i=0}^{b-1} 1/(n - i)."""
    return -sum(1.0 / (n - i) for i in range(b))


def _logsumexp(a: np.ndarray) -> float:
    m = float(np.max(a))
    if not np.isfinite(m):
        return m
    return m + math.log(float(np.sum(np.exp(a - m))))


class _Counter:
    def __init__(self, loglike):
        self.loglike = loglike
        self.n = 0
        self.calls = 0

    def __call__(self, z: np.ndarray) -> np.ndarray:
        if z.shape[0] == 0:
            return np.empty(0)
        self.n += z.shape[0]
        self.calls += 1
        out = np.asarray(self.loglike(np.ascontiguousarray(z)), dtype=np.float64)
        return np.where(np.isnan(out), -np.inf, out)


def _slice_chains(like: _Counter, x0: np.ndarray, l0: np.ndarray, lstar: float,
                  lo: np.ndarray, hi: np.ndarray, chol: np.ndarray, steps: int,
                  rng: np.random.Generator, max_expand: int = 64):
    """Run len(x0) hit-and-run slice chains of `steps` steps each under
    lnL > lstar, all chains advancing one proposal per round."""
    m, d = x0.shape
    x = x0.copy()
    lx = l0.copy()
    done_steps = np.zeros(m, dtype=np.int64)
    stage = np.full(m, _LEFT, dtype=np.int64)
    expand = np.zeros(m, dtype=np.int64)
    dirs = np.empty((m, d))
    a = np.empty(m)
    b = np.empty(m)
    t = np.zeros(m)

    def new_step(idx):
        u = rng.standard_normal((idx.size, d))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        dirs[idx] = u @ chol.T                      # unit length in whitened coordinates
        r = rng.random(idx.size)
        a[idx] = -r
        b[idx] = 1.0 - r
        stage[idx] = _LEFT
        expand[idx] = 0

    new_step(np.arange(m))
    if steps <= 0:
        stage[:] = _DONE
    while True:
        act = np.flatnonzero(stage != _DONE)
        if act.size == 0:
            break
        st = stage[act]
        shr = act[st == _SHRINK]
        t[shr] = a[shr] + (b[shr] - a[shr]) * rng.random(shr.size)
        t[act[st == _LEFT]] = a[act[st == _LEFT]]
        t[act[st == _RIGHT]] = b[act[st == _RIGHT]]
        p = x[act] + t[act, None] * dirs[act]
        inbox = np.all((p >= lo) & (p <= hi), axis=1)
        lp = np.full(act.size, -np.inf)
        if inbox.any():
            lp[inbox] = like(p[inbox])
        inside = inbox & (lp > lstar)
        for s in (_LEFT, _RIGHT):
            sel = st == s
            ok = sel & inside & (expand[act] < max_expand)
            idx = act[ok]
            if s == _LEFT:
                a[idx] -= 1.0
            else:
                b[idx] += 1.0
            expand[idx] += 1
            nxt = act[sel & ~ok]
            stage[nxt] = _RIGHT if s == _LEFT else _SHRINK
            expand[nxt] = 0
        sel = st == _SHRINK
        acc = act[sel & inside]
        if acc.size:
            x[acc] = p[sel & inside]
            lx[acc] = lp[sel & inside]
            done_steps[acc] += 1
            fin = acc[done_steps[acc] >= steps]
            stage[fin] = _DONE
            cont = acc[done_steps[acc] < steps]
            if cont.size:
                new_step(cont)
        rej = act[sel & ~inside]
        neg = t[rej] < 0.0
        a[rej[neg]] = t[rej[neg]]
        b[rej[~neg]] = t[rej[~neg]]
        # an interval shrunk to nothing around the start point (possible only
        # on a likelihood plateau at lnL*): the step keeps the current point
        stuck = rej[(b[rej] - a[rej]) < 1e-12]
        if stuck.size:
            done_steps[stuck] += 1
            stage[stuck[done_steps[stuck] >= steps]] = _DONE
            cont = stuck[done_steps[stuck] < steps]
            if cont.size:
                new_step(cont)
    return x, lx


def nested_slice_sampling(loglike: Callable[[np.ndarray], np.ndarray],
                          lo, hi, *, n_live: int, num_delete: int,
                          num_inner_steps: int, seed: int = 0,
                          tol: float = 1e-3, max_iterations: int = 100000,
                          init: Optional[np.ndarray] = None,
                          chains=None) -> NSResult:
    """Batched nested slice sampling over the box [lo, hi] (uniform prior).

    loglike(z) takes z [B, d] (B >= 1) and returns lnL [B]; it scores the
    initial live points and, unless `chains` is given, every round of
    proposals.  chains(x0, l0, lstar, chol, steps) -> (x, lnL, evaluations)
    replaces the host-side slice chains (e.g. the device engine of
    gpu_chains).  Stops when the live points' largest possible remaining
    contribution, X max(lnL_live), falls below tol times the evidence
    accumulated so far."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = lo.size
    if not (1 <= num_delete < n_live):
        raise ValueError("need 1 <= num_delete < n_live")
    rng = np.random.Generator(np.random.PCG64(seed))
    like = _Counter(loglike)
    t0 = time.perf_counter()
    live = lo + (hi - lo) * rng.random((n_live, d)) if init is None else np.array(init, dtype=np.float64)
    llive = like(live)
    logx = 0.0
    dead, dead_l, dead_lw = [], [], []
    logz = -np.inf
    logx_hist = []
    it = 0
    while it < max_iterations:
        order = np.argsort(llive, kind="stable")
        kill = order[:num_delete]
        keep = order[num_delete:]
        lstar = float(llive[kill[-1]])
        # volume closed by each discarded point (Eq. log_xgpu, point by point)
        for i, k in enumerate(kill):
            nlogx = logx - 1.0 / (n_live - i)
            lw = logx + math.log1p(-math.exp(nlogx - logx))      # log(X_prev - X_new)
            dead.append(live[k].copy())
            dead_l.append(float(llive[k]))
            dead_lw.append(lw)
            logz = np.logaddexp(logz, lw + llive[k])
            logx = nlogx
        logx_hist.append(logx)
        it += 1
        # whitening from the surviving live points
        cov = np.cov(live[keep].T).reshape(d, d) + 1e-12 * np.eye(d)
        chol = np.linalg.cholesky(cov)
        starts = keep[rng.integers(0, keep.size, size=num_delete)]
        if chains is None:
            newx, newl = _slice_chains(like, live[starts], llive[starts], lstar, lo, hi, chol,
                                       num_inner_steps, rng)
        else:
            newx, newl, nev = chains(live[starts], llive[starts], lstar, chol, num_inner_steps)
            like.n += int(nev)
            like.calls += 1
        live[kill] = newx
        llive[kill] = newl
        # stop when the live points cannot change log Z by more than tol
        if logx + float(np.max(llive)) < logz + math.log(tol):
            break
    # the final live points share the remaining volume equally
    lw_live = logx - math.log(n_live)
    samples = np.concatenate([np.array(dead).reshape(-1, d), live], axis=0)
    logl_all = np.concatenate([np.array(dead_l), llive])
    lw_all = np.concatenate([np.array(dead_lw), np.full(n_live, lw_live)])
    logz = _logsumexp(lw_all + logl_all)
    logp = lw_all + logl_all - logz                                  # posterior weights
    p = np.exp(logp)
    finite = np.isfinite(logl_all)
    h = float(np.sum(p[finite] * (logl_all[finite] - logz)))
    return NSResult(logz=float(logz), logz_err=math.sqrt(max(h, 0.0) / n_live),
                    information=h, dead=np.array(dead).reshape(-1, d),
                    dead_logl=np.array(dead_l), log_weights=logp, samples=samples,
                    sample_logl=logl_all,
                    n_like=like.n, n_calls=like.calls, iterations=it,
                    seconds=time.perf_counter() - t0, logx=logx_hist)


# --- the foreground model in sampler coordinates --------------------------------

def foreground_box(N: int, no21: bool = False, beta=(2.0, 3.5), A=(-0.5, 0.0),
                   nu0=(50.0, 200.0), w=(5.0, 40.0), sigma=(1e-3, 0.1),
                   n_alpha: int = 0, alpha=(0.8, 1.2)):
    """Prior box of the foreground model's parameters in sampler coordinates:
    [beta_0..beta_{N-1}, A, nu21, w, log sigma] (log sigma: the log-uniform
    noise prior of Table priors), or [beta.., log sigma] without the 21-cm
    term.  With n_alpha > 0 (amplitude masks crossed with N spectral-index
    masks) the n_alpha uniform amplitude scales follow the indices."""
    lo = ([beta[0]] * N + [alpha[0]] * n_alpha + ([] if no21 else [A[0], nu0[0], w[0]])
          + [math.log(sigma[0])])
    hi = ([beta[1]] * N + [alpha[1]] * n_alpha + ([] if no21 else [A[1], nu0[1], w[1]])
          + [math.log(sigma[1])])
    return np.array(lo), np.array(hi)


def to_theta(z: np.ndarray) -> np.ndarray:
    """Sampler coordinates -> likelihood rows (log sigma -> sigma)."""
    th = np.array(z, dtype=np.float64, copy=True)
    th[:, -1] = np.exp(th[:, -1])
    return th


def model_loglike(model, prec: str = "mixed") -> Callable[[np.ndarray], np.ndarray]:
    """Batched likelihood of a resident model (paper_2603_13196_amd.fgl.Model)
    in sampler coordinates: one fgl_loglike_batch call per round."""
    def f(z):
        return model.loglike(to_theta(z), prec)
    return f


def gpu_chains(model, lo, hi, max_chains: int, prec: str = "mixed", seed: int = 0):
    """A `chains` argument for nested_slice_sampling that runs the slice
    chains on the device (fgl_chains_run), in the coordinates of
    foreground_box."""
    from . import fgl
    eng = fgl.Chains(model, max_chains, lo, hi, seed)

    def run(x0, l0, lstar, chol, steps):
        x, lx, ev, _ = eng.run(x0, l0, lstar, chol, steps, prec)
        return x, lx, ev
    run.engine = eng
    return run
