"""Plain FP64 oracle of the region construction (Sec. 4) and of the
chromatic response functions (Eq. chromatic_function).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU
baseline, never by the library.  Written from the paper's definitions, in
their order, with numpy as the only primitive; it shares nothing with the
HIP library.

Discretisation.  Pixels are an equirectangular grid (rings x columns) with
solid angle omega[ring] * 4 pi.  Sky-frame maps (T_ex = T_base - T_CMB and
beta) are indexed (ring, ra); the beam D(nu) and horizon H are fixed to the
antenna, indexed (ring, ha); at LST step t the local pixel (ring, ha) sees
the sky pixel (ring, (ha + s_t) mod nlon), so the sky pixel (ring, ra) sits
at the local pixel (ring, (ra - s_t) mod nlon).  Integrals over the sphere
are sums of omega-weighted pixels.

  Eq. skyapproximation   T_sky(q, nu) = T_ex(q) (nu/nu0)^(-beta(q)) + T_CMB
  importance weights     W(p, nu, t) for the three schemes of Sec. 4.2:
                         horizon  H(p)
                         sky      T_sky(q_t(p), nu) H(p)
                         beam     T_sky(q_t(p), nu) D(p, nu) H(p)
                         each divided by its integral over the sphere
  Eq. weighted_cdf       C(beta') = sum_{t, nu} sum_p omega W(p, nu, t)
                                    1[beta(q_t(p)) <= beta'], normalised to
                                    end at one; per sky pixel this is the
                                    importance I(q) = sum_{t, nu} omega W
  Alg. method1 / method2 hierarchical and recursive partitions of the
                         spectral-index range on C
  Eq. chromatic_function K_j(nu, t) = sum_q omega M_j(q) T_ex(q) D(p_t(q), nu)

Readings where the paper leaves details open:
  * region j is the half-open index interval [e_j, e_{j+1}); the last one is
    closed;
  * C^{-1}(c) is the smallest pixel spectral index whose C reaches c; the
    mass of a region is the increase of C across it (its pixels' share);
  * ties in Algorithms 1 and 2 (equal widths or masses) go to the region
    with the lowest indices;
  * the horizon-aware weight does not depend on frequency; it is still
    summed over the band (a constant factor, removed by the normalisation).
"""
from __future__ import annotations

import math

import numpy as np

SCHEMES = ("horizon", "sky", "beam")


def sky_temperature(sky) -> np.ndarray:
    """Eq. skyapproximation: T_sky[nu, ring, ra] (K)."""
    ratio = sky.freqs / sky.nu0
    return (sky.t_ex[None] * ratio[:, None, None] ** (-sky.beta[None]) + sky.t_cmb)


def _to_sky_frame(local: np.ndarray, s: int) -> np.ndarray:
    """A local-frame map [..., ring, ha] as seen by the sky pixels at a step
    with shift s: out[..., ring, ra] = local[..., ring, (ra - s) mod nlon]."""
    return np.roll(local, s, axis=-1)


def importance(sky, scheme: str) -> np.ndarray:
    """I[ring, ra] = sum_{t, nu} omega W(p_t(q), nu, t) (Sec. 4.2)."""
    if scheme not in SCHEMES:
        raise ValueError(scheme)
    om = sky.omega[:, None]
    H = sky.horizon.astype(np.float64)
    Ts = sky_temperature(sky) if scheme != "horizon" else None
    I = np.zeros((sky.nlat, sky.nlon))
    for t in range(sky.T):
        Hs = _to_sky_frame(H, int(sky.shifts[t]))
        for f in range(sky.F):
            if scheme == "horizon":
                w = Hs
            elif scheme == "sky":
                w = Ts[f] * Hs
            else:
                w = Ts[f] * _to_sky_frame(sky.beam[f].astype(np.float64), int(sky.shifts[t])) * Hs
            total = np.sum(om * w)
            I += om * w / total
    return I


def weighted_cdf(beta: np.ndarray, imp: np.ndarray):
    """Eq. weighted_cdf as a step function: the pixels' spectral indices in
    ascending order (stable) and C at each, normalised to end at one."""
    b = beta.ravel()
    w = imp.ravel()
    order = np.argsort(b, kind="stable")
    xs = b[order]
    cs = np.cumsum(w[order])
    cs = cs / cs[-1]
    return xs, cs


def cdf_at(xs, cs, x: float) -> float:
    """C(x): the importance of pixels with beta <= x."""
    k = np.searchsorted(xs, x, side="right")
    return 0.0 if k == 0 else float(cs[k - 1])


def cdf_inverse(xs, cs, c: float) -> float:
    """C^{-1}(c): the smallest pixel index with C >= c."""
    k = int(np.searchsorted(cs, c, side="left"))
    return float(xs[min(k, xs.size - 1)])


def region_mass(xs, cs, a: float, b: float, last: bool) -> float:
    """m_r = int_r dC: the increase of C over the pixels with a <= beta < b
    (<= b for the last region)."""
    lo = int(np.searchsorted(xs, a, side="left"))
    hi = int(np.searchsorted(xs, b, side="right" if last else "left"))
    top = float(cs[hi - 1]) if hi > 0 else 0.0
    bottom = float(cs[lo - 1]) if lo > 0 else 0.0
    return top - bottom


def hierarchical(xs, cs, n_total: int) -> np.ndarray:
    """Alg. method1: equal-mass base partition into the largest power of two
    <= n_total, then the widest regions bisected at their importance
    midpoint until n_total regions exist."""
    n_base = 1 << int(math.floor(math.log2(n_total)))
    edges = [float(xs[0])]
    for k in range(1, n_base):
        edges.append(cdf_inverse(xs, cs, k / n_base))
    edges.append(float(xs[-1]))
    for _ in range(n_total - n_base):
        widths = [edges[j + 1] - edges[j] for j in range(len(edges) - 1)]
        j = int(np.argmax(widths))                  # first of the widest
        a, b = edges[j], edges[j + 1]
        cm = 0.5 * (cdf_at(xs, cs, a) + cdf_at(xs, cs, b))
        edges.insert(j + 1, cdf_inverse(xs, cs, cm))
    return np.array(edges)


def recursive(xs, cs, n_total: int) -> np.ndarray:
    """Alg. method2: start from [beta_min, beta_max]; repeatedly bisect, at
    its spectral-index midpoint, the region holding the most importance."""
    edges = [float(xs[0]), float(xs[-1])]
    while len(edges) - 1 < n_total:
        n = len(edges) - 1
        masses = [region_mass(xs, cs, edges[j], edges[j + 1], j == n - 1)
                  for j in range(n)]
        j = int(np.argmax(masses))                  # first of the heaviest
        edges.insert(j + 1, 0.5 * (edges[j] + edges[j + 1]))
    return np.array(edges)


def partition(beta: np.ndarray, imp: np.ndarray, n_total: int, method: str) -> np.ndarray:
    xs, cs = weighted_cdf(beta, imp)
    if method == "hierarchical":
        return hierarchical(xs, cs, n_total)
    if method == "recursive":
        return recursive(xs, cs, n_total)
    raise ValueError(method)


def masks(beta: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Region index of every pixel: j with e_j <= beta < e_{j+1}, the last
    region closed; pixels outside [e_0, e_N] get -1."""
    n = edges.size - 1
    reg = np.searchsorted(edges, beta, side="right") - 1
    reg = np.where(beta == edges[-1], n - 1, reg)
    return np.where((beta < edges[0]) | (beta > edges[-1]), -1, reg)


def chromatic(sky, region: np.ndarray, n_regions: int) -> np.ndarray:
    """Eq. chromatic_function: K[j, nu, t] = sum_q omega M_j(q) T_ex(q)
    D(p_t(q), nu), with the 1/(4 pi) in omega."""
    K = np.zeros((n_regions, sky.F, sky.T))
    src = sky.omega[:, None] * sky.t_ex
    onehot = np.stack([(region == j) * src for j in range(n_regions)])   # [N, ring, ra]
    for t in range(sky.T):
        Ds = _to_sky_frame(sky.beam.astype(np.float64), int(sky.shifts[t]))   # [F, ring, ra]
        K[:, :, t] = np.einsum("jrq,frq->jf", onehot, Ds)
    return K
