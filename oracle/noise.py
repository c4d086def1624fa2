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
counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011) under the key
(low 32 bits of the seed, high 32 bits), in two streams: block b of stream s
is Philox on the counter (b, r, s, 0x6e6f6973) and gives four 32-bit words.
Normals 2j and 2j+1 are the Box-Muller pair (Box and Muller 1958) of
u1 = (w + 1) 2^-32 in (0, 1], w the word j % 4 of stream-0 block j // 4,
and u2 = v 2^-32 in [0, 1), v the same word of stream 1:
rho = sqrt(-2 ln u1), z = rho cos(2 pi u2), rho sin(2 pi u2).  When n is odd
the last pair is used in part.
"""
from __future__ import annotations

import math

import numpy as np

MASK32 = 0xFFFFFFFF
# Philox4x32 round multipliers and Weyl key increments (Salmon et al. 2011)
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
PHILOX_ROUNDS = 10
NOISE_TAG = 0x6E6F6973                    # counter word 3 of every noise block


def _mulhilo32(a: np.ndarray, m: int):
    """High and low 32-bit halves of the 64-bit products a * m (a uint32)."""
    p = a.astype(np.uint64) * np.uint64(m)
    return (p >> np.uint64(32)).astype(np.uint32), (p & np.uint64(MASK32)).astype(np.uint32)


def philox4x32(ctr, key):
    """Philox4x32-10 of counters ctr (uint32 [..., 4]) under key (two 32-bit
    ints); returns uint32 [..., 4]."""
    c = np.array(ctr, dtype=np.uint32, copy=True)
    c0, c1, c2, c3 = (c[..., i] for i in range(4))
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for rnd in range(PHILOX_ROUNDS):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        hi0, lo0 = _mulhilo32(c0, PHILOX_M0)
        hi1, lo1 = _mulhilo32(c2, PHILOX_M1)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint32(k0), lo1,
                          hi0 ^ c3 ^ np.uint32(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=-1)


def normals(n: int, r: int, seed: int) -> np.ndarray:
    """The n standard normals of realisation r (FP64)."""
    npair = (n + 1) // 2
    nblk = (npair + 3) // 4
    key = (seed & MASK32, (seed >> 32) & MASK32)
    ctr = np.zeros((nblk, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint32)
    ctr[:, 1] = np.uint32(r)
    ctr[:, 3] = np.uint32(NOISE_TAG)
    w = philox4x32(ctr, key).reshape(-1)[:npair]               # stream 0: u1
    ctr[:, 2] = np.uint32(1)
    v = philox4x32(ctr, key).reshape(-1)[:npair]               # stream 1: u2
    scale = 2.0 ** -32
    u1 = (w.astype(np.float64) + 1.0) * scale
    u2 = v.astype(np.float64) * scale
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
