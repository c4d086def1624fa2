"""Seeded synthetic workloads for the batched foreground log-likelihood.

This module only draws random numbers and lays them out.  It evaluates no
part of the likelihood (no region power-law sum over theta rows, no residual,
no chi-square): the oracle and the HIP library each do that themselves.

What stands in for the paper's data
-----------------------------------
The paper simulates REACH observations from GSM2008 maps, a conical
log-spiral beam and a horizon mask (Sec. 2.1, Eqs. spectralindexmap,
skyapproximation, simantenna).  None of those inputs is available, so the
workloads here keep the paper's shapes and distributions instead:

* band 50-200 MHz (Sec. 1), 25 mK Gaussian noise (Sec. 2.1, after
  Eq. t21model), a 21-cm Gaussian of a few hundred mK at tens of MHz width
  (Eq. t21model), spectral indices in the prior box of Table priors;
* chromatic response functions ``K[i, nu, t]`` (Eq. chromatic_function) drawn
  per region as log-normal amplitudes, with an optional sinusoidal
  modulation in time (sky rotation) and an optional smooth chromatic ripple
  in frequency (beam chromaticity);
* the observed spectrum ``D`` is a *sky simulation*, not the fitted model:
  each region is made of ``SUBPIX`` sub-pixels with their own spectral index
  scattered around the region's value (the continuous beta field of
  Eq. spectralindexmap seen through a region mask), each sub-pixel carrying a
  share of the region's response, following Eqs. skyapproximation and
  simantenna.  The region model then approximates the data to well below the
  noise, as it does in the paper, without being the data's generator.

Every value is drawn from numpy's PCG64 with the seed ``2603_13196 + k`` for
workload ``k``; draws happen in a fixed order (amplitudes, phases, truth,
sub-pixel scatter, noise, theta batch) so a workload is reproducible from its
index alone.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 2603_13196
T_CMB = 2.725          # K
NU_REF = 230.0         # MHz
NOISE_K = 0.025        # K, Sec. 2.1
SUBPIX = 4             # sub-pixels per region in the sky simulation
SUBPIX_BETA_STD = 2e-4 # scatter of sub-pixel spectral indices inside a region

# theta prior box used for batches (ranges of the benchmark workloads; the
# distribution families follow Table priors: uniform beta, A, nu0, w and
# log-uniform sigma)
PRIOR_BETA = (2.0, 3.5)
PRIOR_A = (-0.5, 0.0)
PRIOR_NU0 = (50.0, 200.0)
PRIOR_W = (5.0, 40.0)
PRIOR_LOGSIG = (math.log(1e-3), math.log(0.1))
# amplitude scales of amplitude masks (Eq. fast_forward_model): the paper
# gives no prior for them; they are gain corrections about one
PRIOR_ALPHA = (0.8, 1.2)


@dataclasses.dataclass
class Workload:
    """One synthetic observation plus a batch of parameter vectors.

    Arrays (C-contiguous):
      K      float32 [N, F, T]  chromatic response per region (K)
      freqs  float64 [F]        channel centres (MHz)
      data   float64 [F, T]     simulated antenna temperature (K)
      theta  float64 [B, N+4]   rows [beta_0..beta_{N-1}, A, nu0, w, sigma]
      truth  float64 [N+4]      parameters the data were simulated at

    With n_alpha > 0 the N regions are n_alpha amplitude masks crossed with
    n_beta = N / n_alpha spectral-index masks (region i * n_beta + j), and
    rows are [beta_0..beta_{n_beta-1}, alpha_0..alpha_{n_alpha-1}, A, nu0,
    w, sigma].
    """
    name: str
    K: np.ndarray
    freqs: np.ndarray
    data: np.ndarray
    theta: np.ndarray
    truth: np.ndarray
    nu_ref: float = NU_REF
    t_cmb: float = T_CMB
    n_alpha: int = 0

    @property
    def N(self) -> int:
        return self.K.shape[0]

    @property
    def F(self) -> int:
        return self.K.shape[1]

    @property
    def T(self) -> int:
        return self.K.shape[2]

    @property
    def B(self) -> int:
        return self.theta.shape[0]

    @property
    def P(self) -> int:
        return self.theta.shape[1]


def freq_grid(lo: float, hi: float, step: float) -> np.ndarray:
    n = int(round((hi - lo) / step)) + 1
    return lo + step * np.arange(n, dtype=np.float64)


# Time structure of the "rich" responses: harmonics per region and the
# scatter of each (region, channel, time) value (see _draw_K).
RICH_HARMONICS = 12
RICH_SCATTER = 0.05


def _draw_K(rng: np.random.Generator, N: int, freqs: np.ndarray, T: int,
            t_mod: float, chroma: float, rich: bool = False) -> np.ndarray:
    """Region responses: a_i ~ LogNormal(ln(300/N), 0.5) times an optional
    time modulation (1 + t_mod sin(2 pi t / T + phi_i)) and an optional
    chromatic ripple (1 + chroma sin(2 pi nu / 17 MHz + psi_i)).

    With ``rich`` the time modulation is instead a sum of RICH_HARMONICS
    harmonics h = 1, 2, ... of the day with amplitudes ~ U[0, 1]/h and
    phases ~ U[0, 2 pi) per region (scaled to an r.m.s. of t_mod / sqrt(2)),
    and every value carries a log-normal scatter exp(RICH_SCATTER e),
    e ~ N(0, 1) per (region, channel, time): the regions then differ in
    their time dependence and K varies with nu, so the time-centred
    responses of a channel have full rank."""
    a = rng.lognormal(mean=math.log(300.0 / N), sigma=0.5, size=N)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=N)
    psi = rng.uniform(0.0, 2.0 * math.pi, size=N)
    t = np.arange(T, dtype=np.float64)
    if T > 1 and t_mod != 0.0 and rich:
        H = RICH_HARMONICS
        amp = rng.uniform(0.0, 1.0, size=(N, H)) / np.arange(1, H + 1)[None, :]
        ph = rng.uniform(0.0, 2.0 * math.pi, size=(N, H))
        ang = 2.0 * math.pi * np.arange(1, H + 1)[None, :, None] * t[None, None, :] / T
        wave = np.sum(amp[:, :, None] * np.sin(ang + ph[:, :, None]), axis=1)     # [N, T]
        rms = np.sqrt(np.mean(wave ** 2, axis=1, keepdims=True))
        tm = 1.0 + (t_mod / math.sqrt(2.0)) * wave / np.where(rms > 0, rms, 1.0)
    elif T > 1 and t_mod != 0.0:
        tm = 1.0 + t_mod * np.sin(2.0 * math.pi * t[None, :] / T + phi[:, None])
    else:
        tm = np.ones((N, T))
    if chroma != 0.0:
        cm = 1.0 + chroma * np.sin(2.0 * math.pi * freqs[None, :] / 17.0 + psi[:, None])
    else:
        cm = np.ones((N, freqs.size))
    K = a[:, None, None] * cm[:, :, None] * tm[:, None, :]
    if rich:
        K = K * np.exp(RICH_SCATTER * rng.standard_normal(size=K.shape))
    return np.ascontiguousarray(K.astype(np.float32))


def _simulate_sky(rng: np.random.Generator, K: np.ndarray, freqs: np.ndarray,
                  nu_ref: float, t_cmb: float, beta_true: np.ndarray,
                  a21: float, nu21: float, w21: float,
                  noise: float) -> np.ndarray:
    """Antenna temperature of a sky whose regions are made of sub-pixels.

    Each region i is split into SUBPIX sub-pixels with response shares
    s_ip (summing to one) and spectral indices beta_i + d_ip, the d_ip
    centred so that sum_p s_ip d_ip = 0.  The sky term follows
    Eq. skyapproximation per sub-pixel and Eq. simantenna sums it with the
    21-cm profile of Eq. t21model and white noise."""
    N, F, T = K.shape
    shares = rng.dirichlet(np.ones(SUBPIX) * 4.0, size=N)            # [N, S]
    d = rng.normal(0.0, SUBPIX_BETA_STD, size=(N, SUBPIX))
    d -= (shares * d).sum(axis=1, keepdims=True)                      # centred
    lr = np.log(freqs / nu_ref)                                       # [F]
    sky = np.zeros((F, T))
    K64 = K.astype(np.float64)
    for i in range(N):
        spec = np.zeros(F)
        for p in range(SUBPIX):
            spec += shares[i, p] * np.exp(-(beta_true[i] + d[i, p]) * lr)
        sky += K64[i] * spec[:, None]
    sig21 = a21 * np.exp(-0.5 * ((freqs - nu21) / w21) ** 2)
    eps = rng.normal(0.0, noise, size=(F, T))
    return np.ascontiguousarray(sky + t_cmb + sig21[:, None] + eps)


def prior_batch(rng: np.random.Generator, N: int, B: int) -> np.ndarray:
    """B rows from the benchmark prior box (uniform beta, A, nu0, w;
    log-uniform sigma)."""
    th = np.empty((B, N + 4))
    th[:, :N] = rng.uniform(*PRIOR_BETA, size=(B, N))
    th[:, N] = rng.uniform(*PRIOR_A, size=B)
    th[:, N + 1] = rng.uniform(*PRIOR_NU0, size=B)
    th[:, N + 2] = rng.uniform(*PRIOR_W, size=B)
    th[:, N + 3] = np.exp(rng.uniform(*PRIOR_LOGSIG, size=B))
    return th


def shell_batch(rng: np.random.Generator, truth: np.ndarray, B: int,
                n_exact: int = 16) -> np.ndarray:
    """Rows near the posterior peak: truth plus Gaussian jitter (1e-4 per
    beta, 10 mK on A, 1 MHz on nu0 and w) and sigma = 25 mK * U[0.8, 1.25].
    The first ``n_exact`` rows keep beta, A, nu0 and w exactly at the truth,
    where |logL| is smallest and the tolerance tightest."""
    N = truth.size - 4
    th = np.repeat(truth[None, :], B, axis=0)
    jit = np.concatenate([np.full(N, 1e-4), [0.01, 1.0, 1.0]])
    th[:, :N + 3] += rng.normal(0.0, 1.0, size=(B, N + 3)) * jit[None, :]
    th[:n_exact, :N + 3] = truth[None, :N + 3]
    th[:, N + 3] = NOISE_K * rng.uniform(0.8, 1.25, size=B)
    return th


def make(N: int, freqs: np.ndarray, T: int, B: int, seed: int, *,
         t_mod: float = 0.3, chroma: float = 0.0, batch: str = "prior",
         name: str = "custom", nu_ref: float = NU_REF,
         t_cmb: float = T_CMB, rich: bool = False) -> Workload:
    """Generic workload: K, simulated data at a drawn truth, and a batch of
    B rows ('prior', 'shell', or 'mixed' = half of each).  ``rich`` draws
    full-rank responses (see _draw_K)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = _draw_K(rng, N, freqs, T, t_mod, chroma, rich)
    beta_true = rng.uniform(2.45, 3.15, size=N)
    a21, nu21, w21 = -0.15, 80.0, 15.0
    data = _simulate_sky(rng, K, freqs, nu_ref, t_cmb, beta_true, a21, nu21,
                         w21, NOISE_K)
    truth = np.concatenate([beta_true, [a21, nu21, w21, NOISE_K]])
    if batch == "prior":
        theta = prior_batch(rng, N, B)
    elif batch == "shell":
        theta = shell_batch(rng, truth, B)
    elif batch == "mixed":
        h = B // 2
        theta = np.concatenate([prior_batch(rng, N, h),
                                shell_batch(rng, truth, B - h)])
    else:
        raise ValueError(f"unknown batch kind {batch!r}")
    return Workload(name, K, np.ascontiguousarray(freqs), data,
                    np.ascontiguousarray(theta), truth, nu_ref, t_cmb)


# The benchmark workloads by name: the small plain-FP64 case, the plain-FP32
# case, the mixed-precision headline case and the large case, each with its
# own seed (the serving mix, seed SEED_BASE + 3, is drawn by
# serving_clients).
SMALL = "N4_F151_T1_B1000"
MEDIUM = "N16_F151_T20_B4096"
HEADLINE = "N32_F301_T96_B16384"
LARGE = "N64_F401_T240_B65536"
WORKLOADS = {
    SMALL: dict(N=4, grid=(50.0, 200.0, 1.0), T=1, B=1000, t_mod=0.0, seed=SEED_BASE + 0),
    MEDIUM: dict(N=16, grid=(50.0, 200.0, 1.0), T=20, B=4096, t_mod=0.3, seed=SEED_BASE + 1),
    HEADLINE: dict(N=32, grid=(50.0, 200.0, 0.5), T=96, B=16384, t_mod=0.3, seed=SEED_BASE + 2),
    LARGE: dict(N=64, grid=(50.0, 250.0, 0.5), T=240, B=65536, t_mod=0.3, seed=SEED_BASE + 4),
}


def make_masks(n_alpha: int, n_beta: int, freqs: np.ndarray, T: int, B: int,
               seed: int, *, t_mod: float = 0.3, batch: str = "prior",
               name: str = "masks", nu_ref: float = NU_REF,
               t_cmb: float = T_CMB) -> Workload:
    """Workload of the crossed-mask model: K for n_alpha * n_beta regions
    (drawn as in ``make``), a truth with beta_j ~ U[2.45, 3.15] and
    alpha_i ~ U[0.95, 1.05], data simulated with region responses
    alpha_i K_ij, and a batch of B rows ('prior', 'shell' or 'mixed'); the
    alpha prior is PRIOR_ALPHA and the shell jitter on alpha is 1e-4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = n_alpha * n_beta
    K = _draw_K(rng, N, freqs, T, t_mod, 0.0)
    beta_true = rng.uniform(2.45, 3.15, size=n_beta)
    alpha_true = rng.uniform(0.95, 1.05, size=n_alpha)
    a21, nu21, w21 = -0.15, 80.0, 15.0
    K_eff = K.astype(np.float64) * np.repeat(alpha_true, n_beta)[:, None, None]
    data = _simulate_sky(rng, K_eff, freqs, nu_ref, t_cmb,
                         np.tile(beta_true, n_alpha), a21, nu21, w21, NOISE_K)
    truth = np.concatenate([beta_true, alpha_true, [a21, nu21, w21, NOISE_K]])
    nb, na = n_beta, n_alpha

    def prior(n):
        th = np.empty((n, nb + na + 4))
        th[:, :nb] = rng.uniform(*PRIOR_BETA, size=(n, nb))
        th[:, nb:nb + na] = rng.uniform(*PRIOR_ALPHA, size=(n, na))
        th[:, nb + na] = rng.uniform(*PRIOR_A, size=n)
        th[:, nb + na + 1] = rng.uniform(*PRIOR_NU0, size=n)
        th[:, nb + na + 2] = rng.uniform(*PRIOR_W, size=n)
        th[:, nb + na + 3] = np.exp(rng.uniform(*PRIOR_LOGSIG, size=n))
        return th

    def shell(n, n_exact=16):
        th = np.repeat(truth[None, :], n, axis=0)
        jit = np.concatenate([np.full(nb + na, 1e-4), [0.01, 1.0, 1.0]])
        th[:, :-1] += rng.normal(0.0, 1.0, size=(n, nb + na + 3)) * jit[None, :]
        th[:n_exact, :-1] = truth[None, :-1]
        th[:, -1] = NOISE_K * rng.uniform(0.8, 1.25, size=n)
        return th

    if batch == "prior":
        theta = prior(B)
    elif batch == "shell":
        theta = shell(B)
    elif batch == "mixed":
        theta = np.concatenate([prior(B // 2), shell(B - B // 2)])
    else:
        raise ValueError(f"unknown batch kind {batch!r}")
    return Workload(name, K, np.ascontiguousarray(freqs), data,
                    np.ascontiguousarray(theta), truth, nu_ref, t_cmb, n_alpha)


# The crossed-mask counterpart of the headline workload: its 32 regions as
# 2 amplitude masks x 16 spectral-index masks (N32, F301, T96, B16384).
MASKS_NAME = "A2xB16_F301_T96_B16384"


def masks_config(*, B: int = 16384, batch: str = "prior") -> Workload:
    c = WORKLOADS[HEADLINE]
    return make_masks(2, 16, freq_grid(*c["grid"]), c["T"], B, SEED_BASE + 5,
                      t_mod=c["t_mod"], batch=batch, name=MASKS_NAME)


def config(name: str, *, B: Optional[int] = None, batch: str = "prior",
           chroma: float = 0.0, rich: bool = False) -> Workload:
    """The named benchmark workload (SMALL, MEDIUM, HEADLINE or LARGE),
    optionally with another batch size or batch kind.  ``rich`` swaps the
    responses for full-rank ones (several time harmonics per region, a
    per-value scatter) with a chromatic ripple of 5 % unless ``chroma`` is
    given, under a seed of its own (the workload's seed + 100)."""
    c = WORKLOADS[name]
    freqs = freq_grid(*c["grid"])
    if rich:
        return make(c["N"], freqs, c["T"], c["B"] if B is None else B,
                    c["seed"] + 100, t_mod=c["t_mod"], chroma=chroma or 0.05,
                    batch=batch, name=name + "_rich", rich=True)
    return make(c["N"], freqs, c["T"], c["B"] if B is None else B,
                c["seed"], t_mod=c["t_mod"], chroma=chroma, batch=batch, name=name)


def posterior_shell(name: str, B: int = 1024, rich: bool = False) -> Workload:
    """The named workload with its theta batch replaced by a posterior shell."""
    return config(name, B=B, batch="shell", rich=rich)


@dataclasses.dataclass
class Client:
    """One synthetic nested-sampling run of the serving mix."""
    cid: int
    work: Workload
    batches: List[int]          # B of each successive request
    think_ms: List[float]       # wait before each submission


def serving_clients(n_clients: int = 64, n_requests: int = 4,
                    seed: int = SEED_BASE + 3, max_B: int = 8192,
                    min_B: int = 500) -> List[Client]:
    """The serving mix: per client N ~ U{4..40}, T ~ U{1..96},
    F in {151, 301}, B ~ U[min_B, max_B], think time ~ Exp(mean 2 ms)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for c in range(n_clients):
        N = int(rng.integers(4, 41))
        T = int(rng.integers(1, 97))
        F = 151 if rng.integers(0, 2) == 0 else 301
        step = 1.0 if F == 151 else 0.5
        bs = [int(rng.integers(min_B, max_B + 1)) for _ in range(n_requests)]
        think = [float(rng.exponential(2.0)) for _ in range(n_requests)]
        w = make(N, freq_grid(50.0, 200.0, step), T, max(bs),
                 int(rng.integers(0, 2**31)), t_mod=0.3, batch="mixed",
                 name=f"client{c}")
        out.append(Client(c, w, bs, think))
    return out
