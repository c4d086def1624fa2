"""FP64 oracle of the residual-likelihood reference distribution (Sec. 5).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark, never by
the library.  Plain numpy; shares nothing with the HIP code.

The accuracy criterion of Sec. 5 compares the median posterior likelihood of
a fit with the distribution of the likelihood over data sets that the model
describes exactly, up to realisations of the assumed noise (uncorrelated
Gaussian, 25 mK in the paper).  For such a data set D = M(theta) + e the
residual at theta is the noise itself, so Eq. likelihood gives

    lnL_noise = -sum_k e_k^2 / (2 sigma_like^2) - (n/2) ln(2 pi sigma_like^2),

with n = F T residuals, e_k = sigma_noise z_k and z_k standard normal; the
fraction of these values at or below a fit's median lnL is q_i
(the quantile of the accuracy criterion, Sec. 5).

Random numbers.  Each realisation r draws its n normals from the
counter-based generator Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011) under key (seed, 0),
in two streams: block b of stream s is Philox on counter (b, r, s, 0) and
gives four 64-bit words.  Normals 2j and 2j+1 are the Box-Muller pair (Box
and Muller 1958) of u1 = (floor(w / 2^11) + 1) 2^-53 in (0, 1], w the word
j % 4 of stream-0 block j // 4, and u2 = floor(v / 2^11) 2^-53 in [0, 1),
v the same word of stream 1: rho = sqrt(-2 ln u1), z = rho cos(2 pi u2),
rho sin(2 pi u2).  When n is odd the last pair is used in part.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
# Philox4x64 multipliers and Weyl key increments (Salmon et al. 2011)
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
PHILOX_ROUNDS = 10


def _mulhilo64(a: np.ndarray, m: int):
    """High and low 64-bit halves of the 128-bit products a * m (uint64)."""
    a = a.astype(np.uint64)
    lo32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & lo32, a >> s32
    m_lo, m_hi = np.uint64(m & 0xFFFFFFFF), np.uint64(m >> 32)
    ll = a_lo * m_lo
    lh = a_lo * m_hi
    hl = a_hi * m_lo
    hh = a_hi * m_hi
    mid = (ll >> s32) + (lh & lo32) + (hl & lo32)        # < 3 * 2^32, no wrap
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    lo = (mid << s32) | (ll & lo32)
    return hi, lo


def philox4x64(ctr, key):
    """Philox4x64-10 of counters ctr (uint64 [..., 4]) under key (two ints);
    returns uint64 [..., 4]."""
    c = np.array(ctr, dtype=np.uint64, copy=True)
    c0, c1, c2, c3 = (c[..., i] for i in range(4))
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    with np.errstate(over="ignore"):
        for rnd in range(PHILOX_ROUNDS):
            if rnd:
                k0 = (k0 + PHILOX_W0) & MASK64
                k1 = (k1 + PHILOX_W1) & MASK64
            hi0, lo0 = _mulhilo64(c0, PHILOX_M0)
            hi1, lo1 = _mulhilo64(c2, PHILOX_M1)
            c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                              hi0 ^ c3 ^ np.uint64(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=-1)


def normals(n: int, r: int, seed: int) -> np.ndarray:
    """The n standard normals of realisation r (FP64)."""
    npair = (n + 1) // 2
    nblk = (npair + 3) // 4
    ctr = np.zeros((nblk, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint64)
    ctr[:, 1] = np.uint64(r)
    w = philox4x64(ctr, (seed, 0)).reshape(-1)[:npair]        # stream 0: u1
    ctr[:, 2] = np.uint64(1)
    v = philox4x64(ctr, (seed, 0)).reshape(-1)[:npair]        # stream 1: u2
    scale = 2.0 ** -53
    u1 = ((w >> np.uint64(11)).astype(np.float64) + 1.0) * scale
    u2 = (v >> np.uint64(11)).astype(np.float64) * scale
    rho = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    z = np.stack([rho * np.cos(ang), rho * np.sin(ang)], axis=-1).reshape(-1)
    return z[:n]


def noise_loglike(n: int, R: int, sigma_noise: float, sigma_like: float,
                  seed: int, first: int = 0) -> np.ndarray:
    """lnL_noise of realisations first..first+R-1: Eq. likelihood with the
    residual replaced by sigma_noise times that realisation's normals."""
    out = np.empty(R, dtype=np.float64)
    norm = 0.5 * n * math.log(2.0 * math.pi * sigma_like * sigma_like)
    for i in range(R):
        e = sigma_noise * normals(n, first + i, seed)
        out[i] = -np.sum(e * e) / (2.0 * sigma_like * sigma_like) - norm
    return out


def quantile(lnl_noise, lbar) -> np.ndarray:
    """q_i = P(lnL_noise <= lbar_i), the fraction of the R reference values at
    or below each lbar_i (the quantile of the accuracy criterion, Sec. 5)."""
    ref = np.asarray(lnl_noise, dtype=np.float64)
    lb = np.asarray(lbar, dtype=np.float64)
    return np.array([np.count_nonzero(ref <= x) for x in lb],
                    dtype=np.float64) / ref.size
