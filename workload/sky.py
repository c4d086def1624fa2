"""Seeded synthetic sky, beam and horizon for the region construction.

The paper builds its regions from the GSM2008 sky, a conical log-spiral
beam and a horizon mask (Sec. 2.1, Sec. 4); none of these is available, so
this module draws stand-ins with the same structure, on an equirectangular
grid in equatorial coordinates (declination rings x right-ascension
columns):

* sky frame: the base map above the CMB, T_base - T_CMB (K at nu0), bright
  along a tilted band standing in for the Galactic plane and falling off
  towards its poles, with log-normal small-scale structure; the spectral
  index map beta (Eq. spectralindexmap), flatter (about 2.5) in the band and
  steeper (about 3.1) away from it, with a little noise;
* local frame (declination x hour angle, fixed to the antenna): a chromatic
  beam D(nu) peaked at the zenith declination with a width that grows
  towards low frequencies, and a binary horizon mask H with a ragged
  horizon profile;
* time: LST step t turns the sky by s_t right-ascension columns, so the
  local pixel (ring, ha) sees the sky pixel (ring, (ha + s_t) mod nlon).

Only random numbers and their layout live here; the importance weights,
CDFs, partitions and chromatic functions are computed by the oracle and by
the library, each on its own.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_SKY = 2603_13196 + 7
T_CMB = 2.725
NU0 = 230.0


@dataclasses.dataclass
class Sky:
    omega: np.ndarray     # [nlat] pixel solid angle of each ring / (4 pi)
    t_ex: np.ndarray      # [nlat, nlon] T_base - T_CMB (K), sky frame
    beta: np.ndarray      # [nlat, nlon] spectral index, sky frame
    beam: np.ndarray      # [F, nlat, nlon] float32 D(nu), local frame
    horizon: np.ndarray   # [nlat, nlon] uint8 H, local frame
    freqs: np.ndarray     # [F] MHz
    shifts: np.ndarray    # [T] int32 right-ascension shift of each time step
    nu0: float = NU0
    t_cmb: float = T_CMB

    @property
    def nlat(self) -> int:
        return self.t_ex.shape[0]

    @property
    def nlon(self) -> int:
        return self.t_ex.shape[1]

    @property
    def F(self) -> int:
        return self.freqs.size

    @property
    def T(self) -> int:
        return self.shifts.size


def make_sky(nlat: int, nlon: int, freqs: np.ndarray, T: int, *, seed: int = SEED_SKY,
             lst_hours: float = 4.0, site_dec: float = -30.7) -> Sky:
    """A sky of nlat x nlon pixels seen over T LST steps spanning lst_hours
    (at least one column per step), by an antenna at declination site_dec."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dec = (np.arange(nlat) + 0.5) / nlat * math.pi - math.pi / 2
    ra = (np.arange(nlon) + 0.5) / nlon * 2 * math.pi
    dd, rr = math.pi / nlat, 2 * math.pi / nlon
    omega = np.cos(dec) * dd * rr / (4 * math.pi)
    # a tilted "Galactic" band: angular distance from a great circle
    tilt = math.radians(62.9)
    x = np.cos(dec)[:, None] * np.cos(ra)[None, :]
    y = np.cos(dec)[:, None] * np.sin(ra)[None, :]
    z = np.sin(dec)[:, None] * np.ones((1, nlon))
    b = np.arcsin(np.clip(z * math.cos(tilt) - y * math.sin(tilt), -1, 1))   # "latitude"
    lon_g = np.arctan2(z * math.sin(tilt) + y * math.cos(tilt), x)
    core = np.exp(-(lon_g / 0.6) ** 2)                   # bright "centre"
    band = np.exp(-np.abs(b) / math.radians(8.0)) * (1.0 + 4.0 * core)
    t_ex = 18.0 + 260.0 * band
    t_ex = t_ex * rng.lognormal(0.0, 0.15, size=t_ex.shape)
    beta = 3.1 - 0.6 * np.exp(-np.abs(b) / math.radians(15.0)) + rng.normal(0.0, 0.02, t_ex.shape)
    # local frame: zenith at (site_dec, ha = 0)
    sd = math.radians(site_dec)
    ha = (np.arange(nlon) + 0.5) / nlon * 2 * math.pi - math.pi
    cos_z = (np.sin(dec)[:, None] * math.sin(sd)
             + np.cos(dec)[:, None] * math.cos(sd) * np.cos(ha)[None, :])
    horizon_profile = math.radians(3.0) * (1.0 + 0.5 * np.sin(3 * ha + rng.uniform(0, 6.3)))
    elev = np.arcsin(np.clip(cos_z, -1, 1))
    horizon = (elev > horizon_profile[None, :]).astype(np.uint8)
    width = 1.2 * (freqs / 100.0) ** -0.35                # beam exponent per channel
    beam = np.empty((freqs.size, nlat, nlon), dtype=np.float32)
    cz = np.clip(cos_z, 0.0, 1.0)
    for f, wv in enumerate(width):
        ripple = 1.0 + 0.05 * np.sin(freqs[f] / 7.0) * cz
        beam[f] = (cz ** (1.0 / wv) * ripple).astype(np.float32)
    steps = max(1, int(round(lst_hours / 24.0 * nlon / max(T, 1))))
    shifts = (np.arange(T) * steps % nlon).astype(np.int32)
    return Sky(omega, np.ascontiguousarray(t_ex), np.ascontiguousarray(beta),
               np.ascontiguousarray(beam), np.ascontiguousarray(horizon),
               np.ascontiguousarray(freqs, dtype=np.float64), shifts)


# The sky of the K-builder benchmark: 256 x 512 pixels (0.7 degree), the
# headline's 301 channels (50-200 MHz) and 96 LST steps over 4 hours.
SKY_NAME = "sky256x512_F301_T96"


def sky_config() -> Sky:
    freqs = 50.0 + 0.5 * np.arange(301)
    return make_sky(256, 512, freqs, 96)
