"""The region-construction oracle against its pins, and planted mistakes
in copies of it that the pins must catch (CPU only)."""
import importlib.util
import os

import pytest

from oracle import regions
from tests import regions_pins as pins

MUTANTS = {
    "roll_direction": ("return np.roll(local, s, axis=-1)", "return np.roll(local, -s, axis=-1)"),
    "no_normalisation": ("I += om * w / total", "I += om * w"),
    "no_omega_weight": ("I += om * w / total", "I += w / total"),
    "beam_scheme_drops_horizon": (
        "w = Ts[f] * _to_sky_frame(sky.beam[f].astype(np.float64), int(sky.shifts[t])) * Hs",
        "w = Ts[f] * _to_sky_frame(sky.beam[f].astype(np.float64), int(sky.shifts[t]))"),
    "beta_sign": ("** (-sky.beta[None])", "** (sky.beta[None])"),
    "cdf_unsorted": ('order = np.argsort(b, kind="stable")', "order = np.arange(b.size)"),
    "inverse_side": ('k = int(np.searchsorted(cs, c, side="left"))',
                     'k = int(np.searchsorted(cs, c, side="right"))'),
    "base_not_power_of_two": ("n_base = 1 << int(math.floor(math.log2(n_total)))",
                              "n_base = n_total"),
    "hier_widest_is_narrowest": ("j = int(np.argmax(widths))", "j = int(np.argmin(widths))"),
    "hier_midpoint_physical": ("edges.insert(j + 1, cdf_inverse(xs, cs, cm))",
                               "edges.insert(j + 1, 0.5 * (a + b))"),
    "rec_heaviest_is_lightest": ("j = int(np.argmax(masses))", "j = int(np.argmin(masses))"),
    "rec_midpoint_by_mass": ("edges.insert(j + 1, 0.5 * (edges[j] + edges[j + 1]))",
                             "edges.insert(j + 1, cdf_inverse(xs, cs, 0.5 * (cdf_at(xs, cs, edges[j]) + cdf_at(xs, cs, edges[j + 1]))))"),
    "mask_closed_left_open": ('reg = np.searchsorted(edges, beta, side="right") - 1',
                              'reg = np.searchsorted(edges, beta, side="left") - 1'),
    "chromatic_uses_t_base": ("src = sky.omega[:, None] * sky.t_ex",
                              "src = sky.omega[:, None] * (sky.t_ex + sky.t_cmb)"),
    "chromatic_no_omega": ("src = sky.omega[:, None] * sky.t_ex", "src = sky.t_ex"),
}


@pytest.mark.parametrize("pin", pins.ALL, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(regions)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(regions.__file__).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/absent"
    path = os.path.join(tmp_path, "regions_mutant.py")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("regions_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = []
    for pin in pins.ALL:
        try:
            pin(mod)
        except (AssertionError, IndexError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
