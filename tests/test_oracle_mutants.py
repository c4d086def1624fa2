"""Plant plausible mistakes in copies of the oracle (on the CPU) and check
that the pin suite catches every one of them.

Each mutant is one textual edit of oracle/fgl_oracle.c: a dropped term, a
flipped sign, a wrong index, a transposed operand, a lost factor.  The
edited copy is compiled into a temporary directory; the real oracle is not
touched.
"""
import os

import pytest

import oracle
from tests import pins

MUTANTS = {
    "beta_sign": ("powv[j] = pow(ratio, -beta[j]);", "powv[j] = pow(ratio, beta[j]);"),
    "ratio_inverted": ("double ratio = nu / nu_ref;", "double ratio = nu_ref / nu;"),
    "power_in_float": ("powv[j] = pow(ratio, -beta[j]);",
                       "powv[j] = (float)pow(ratio, -beta[j]);"),
    "dropped_last_region": ("for (int j = 0; j < NB; ++j) {\n                const float",
                            "for (int j = 0; j < NB - 1; ++j) {\n                const float"),
    "K_transposed": ("K + (((size_t)i * NB + j) * F + f) * T",
                     "K + (((size_t)f * NB + j) * n_amp + i) * T"),
    "K_time_index": ("row[t] += (a * (double)Kij[t]) * powv[j];",
                     "row[t] += (a * (double)Kij[0]) * powv[j];"),
    # amplitude masks
    "alpha_dropped": ("double a = NA > 0 ? alpha[i] : 1.0;", "double a = 1.0;"),
    "alpha_index_j": ("double a = NA > 0 ? alpha[i] : 1.0;",
                      "double a = NA > 0 ? alpha[(i + 1) % NA] : 1.0;"),
    "alpha_squared": ("row[t] += (a * (double)Kij[t]) * powv[j];",
                      "row[t] += (a * a * (double)Kij[t]) * powv[j];"),
    "alpha_row_offset": ("const double *alpha = theta_row + NB;",
                         "const double *alpha = theta_row + NB - 1;"),
    "region_index_swapped": ("K + (((size_t)i * NB + j) * F + f) * T",
                             "K + (((size_t)j * n_amp + i) * F + f) * T"),
    # gradient
    "grad_beta_sign": ("nm_add(&acc[j], r * (-lr * amp * kp));",
                       "nm_add(&acc[j], r * (lr * amp * kp));"),
    "grad_beta_no_alpha": ("nm_add(&acc[j], r * (-lr * amp * kp));",
                           "nm_add(&acc[j], r * (-lr * kp));"),
    "grad_alpha_times_alpha": ("if (NA > 0) nm_add(&acc[NB + i], r * kp);",
                               "if (NA > 0) nm_add(&acc[NB + i], r * kp * amp);"),
    "grad_nu21_sign": ("r * (A * gnu * dnu / (w * w))", "r * (-A * gnu * dnu / (w * w))"),
    "grad_width_power": ("r * (A * gnu * dnu * dnu / (w * w * w))",
                         "r * (A * gnu * dnu * dnu / (w * w))"),
    "grad_amp_dropped_g": ("nm_add(&acc[P - 4], r * gnu);", "nm_add(&acc[P - 4], r);"),
    "grad_sigma_cube": ("g[P - 1] = c2 / (var * sigma) - n / sigma;",
                        "g[P - 1] = c2 / var - n / sigma;"),
    "grad_sigma_count": ("g[P - 1] = c2 / (var * sigma) - n / sigma;",
                         "g[P - 1] = c2 / (var * sigma) - 0.5 * n / sigma;"),
    "grad_not_over_sigma2": ("g[k] = (acc[k].s + acc[k].c) / var;",
                             "g[k] = (acc[k].s + acc[k].c) / sigma;"),
    "grad_residual_sign": ("double r = D[(size_t)f * T + t] - m[(size_t)f * T + t];",
                           "double r = m[(size_t)f * T + t] - D[(size_t)f * T + t];"),
    "alpha_not_checked": ("if (!(a >= 0x1p-32 && a <= 0x1p32)) return 0;", ""),
    "dropped_tcmb": ("row[t] = row[t] + t_cmb + sig21;", "row[t] = row[t] + sig21;"),
    "t21_sign": ("sig21 = A * exp(", "sig21 = -A * exp("),
    "t21_width": ("(2.0 * w * w)", "(w * w)"),
    "t21_exp_sign": ("exp(-(dv * dv)", "exp((dv * dv)"),
    "dropped_t21": ("row[t] = row[t] + t_cmb + sig21;", "row[t] = row[t] + t_cmb;"),
    "sigma_not_squared": ("double s2 = sigma * sigma;", "double s2 = sigma;"),
    "chi2_half_lost": ("return -0.5 * (chi2.s + chi2.c) / s2",
                       "return -1.0 * (chi2.s + chi2.c) / s2"),
    "dropped_normalisation": ("- 0.5 * n * log(2.0 * M_PI * s2);", ";"),
    "normalisation_not_2pi": ("log(2.0 * M_PI * s2)", "log(M_PI * s2)"),
    "residual_shifted": ("double r = D[k] - m[k];",
                         "double r = D[k] - m[k == 0 ? 0 : k - 1];"),
    "compensation_sign": ("a->c += (a->s - t) + x;", "a->c += (a->s - t) - x;"),
    "invalid_not_checked": ("if (!(sigma > 0.0)) return 0;", ""),
    "width_not_checked": ("if (!(w > 0.0)) return 0;", ""),
    "beta_bound_not_checked": ("if (fabs(th[j]) > 64.0) return 0;",
                               "if (fabs(th[j]) > 1e300) return 0;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/absent"
    mpath = os.path.join(tmp_path, "mutant.c")
    with open(mpath, "w") as fh:
        fh.write(src.replace(old, new))
    so = oracle.build(mpath, os.path.join(tmp_path, "libmutant.so"))
    orc = oracle.Oracle(so)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
