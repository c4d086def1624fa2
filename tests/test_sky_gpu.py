"""GPU region construction: importance maps (Sec. 4.2, three weightings) and
chromatic response functions (Eq. chromatic_function) from libfgl against
the FP64 oracle, plus the whole chain importance -> partition -> K."""
import numpy as np
import pytest

from oracle import regions
from workload.sky import Sky, make_sky, sky_config
from tests.gpu_util import lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fgl():
    return lib()


def _close(got, want, label, rtol=1e-12):
    scale = np.abs(want).max()
    d = np.abs(got - want)
    say(f"  {label}: max|d|/max|ref|={d.max() / scale:.3e}")
    assert np.all(d <= rtol * (np.abs(want) + scale * 1e-3)), label


@pytest.mark.parametrize("shape", [(8, 16, 3, 2), (33, 70, 9, 7), (64, 128, 31, 24),
                                   (12, 40, 6, 150)])
def test_importance_matches_oracle(fgl, shape):
    nlat, nlon, F, T = shape
    s = make_sky(nlat, nlon, np.linspace(50.0, 200.0, F), T, seed=nlat + nlon)
    say(f"sky {nlat}x{nlon} F={F} T={T}")
    sm = fgl.SkyModel.from_sky(s)
    for sch in regions.SCHEMES:
        got = sm.importance(s.shifts, sch)
        _close(got, regions.importance(s, sch), f"importance/{sch}")
        assert abs(got.sum() - F * T) <= 1e-10 * F * T
    sm.close()


@pytest.mark.parametrize("N", [1, 5, 32, 100])
def test_chromatic_matches_oracle(fgl, N):
    s = make_sky(33, 70, np.linspace(50.0, 200.0, 9), 7, seed=5)
    I = regions.importance(s, "beam")
    e = regions.partition(s.beta, I, N, "recursive")
    sm = fgl.SkyModel.from_sky(s)
    got = sm.chromatic(e, s.shifts)
    _close(got, regions.chromatic(s, regions.masks(s.beta, e), N), f"chromatic/N{N}")
    # edges inside the index range: outer pixels belong to no region
    inner = np.linspace(np.quantile(s.beta, 0.1), np.quantile(s.beta, 0.9), 4)
    got = sm.chromatic(inner, s.shifts)
    _close(got, regions.chromatic(s, regions.masks(s.beta, inner), 3), "chromatic/inner")
    sm.close()


def test_chromatic_more_steps_than_one_launch(fgl):
    """T = 150 steps: the normaliser and K kernels run two launches of at
    most 128 steps each (two lanes per step in up to 256 lanes)."""
    s = make_sky(12, 40, np.linspace(50.0, 200.0, 6), 150, seed=17)
    say("sky 12x40 F=6 T=150")
    I = regions.importance(s, "beam")
    e = regions.partition(s.beta, I, 5, "recursive")
    sm = fgl.SkyModel.from_sky(s)
    got = sm.chromatic(e, s.shifts)
    _close(got, regions.chromatic(s, regions.masks(s.beta, e), 5), "chromatic/T150")
    sm.close()


def test_pipeline_matches_oracle(fgl):
    """Importance (GPU) -> partition (library host code) -> K (GPU) gives
    the oracle's edges and functions, for both algorithms."""
    s = make_sky(40, 80, np.linspace(50.0, 200.0, 11), 9, seed=23)
    sm = fgl.SkyModel.from_sky(s)
    for method in ("hierarchical", "recursive"):
        for sch in regions.SCHEMES:
            Ig = sm.importance(s.shifts, sch)
            Io = regions.importance(s, sch)
            eg = fgl.fgl_partition(s.beta, Ig, 12, method)
            eo = regions.partition(s.beta, Io, 12, method)
            assert np.array_equal(eg, eo), (method, sch, eg, eo)
        Kg = sm.chromatic(eg, s.shifts)
        _close(Kg, regions.chromatic(s, regions.masks(s.beta, eo), 12), f"pipeline/{method}")
    sm.close()


def test_full_sky_sampled(fgl):
    """The benchmark sky (256 x 512 pixels, 301 channels, 96 steps), 32
    recursive beam-weighted regions: the full K call, checked against the
    oracle on 3 channels x 4 steps."""
    s = sky_config()
    sm = fgl.SkyModel.from_sky(s)
    I = sm.importance(s.shifts, "beam")
    e = fgl.fgl_partition(s.beta, I, 32, "recursive")
    K = sm.chromatic(e, s.shifts)
    say(f"full sky: chromatic kernel {sm.kernel_ms():.3f} ms")
    fs, ts = np.array([0, 150, 300]), np.array([0, 47, 95])
    sub = Sky(s.omega, s.t_ex, s.beta, s.beam[fs], s.horizon, s.freqs[fs], s.shifts[ts])
    want = regions.chromatic(sub, regions.masks(s.beta, e), 32)
    _close(K[:, fs][:, :, ts], want, "full-sky/sampled")
    sm.close()


def test_errors(fgl):
    s = make_sky(8, 16, np.linspace(50.0, 200.0, 3), 2, seed=1)
    sm = fgl.SkyModel.from_sky(s)
    for bad in ([-1, 0], [0, 16]):
        with pytest.raises(fgl.FGLError) as e:
            sm.importance(bad, "beam")
        assert e.value.code == fgl.FGL_EINVAL
    with pytest.raises(fgl.FGLError):
        sm.importance(s.shifts, 7)
    with pytest.raises(fgl.FGLError):
        sm.chromatic([3.0, 2.0], s.shifts)
    sm.close()
    dark = fgl.SkyModel(s.omega, s.t_ex, s.beta, s.beam, np.zeros_like(s.horizon), s.freqs)
    with pytest.raises(fgl.FGLError) as e:
        dark.importance(s.shifts, "horizon")
    assert e.value.code == fgl.FGL_EINVAL and "integrates" in fgl.fgl_last_error()
    dark.close()
