"""The oracle's pins catch plausible mistakes: each case plants one mistake
(a dropped term, a flipped sign, a lost factor, swapped phases) in a copy of
the oracle's source, compiles the copy, and runs the pin of that term on it;
the pin must fail.  The oracle itself is not modified: each mutant is built
from the source text into a temporary directory."""
import os

import numpy as np
import pytest

import test_oracle_forces as F

pytestmark = [pytest.mark.usefixtures("oracle_lib"), pytest.mark.slow]


def maxwell_pin_passes(lib):
    r = F.maxwell_jump_ratio(5.0, 64, 4.0, 15000, lib=lib)
    return abs(r - 1) < 0.06


def coulomb_pin_passes(lib):
    r, _ = F.coulomb_jump_ratio(64, 10000, lib=lib)
    return abs(r - 1) < 0.06


def shear_pin_passes(lib):
    nu_l, nu_v = F.shear_decay_rates(lib=lib)
    return abs(nu_l / (4.0 * 0.05 / 3.0) - 1) < 1e-3 and abs(nu_v / 0.05 - 1) < 1e-3


def translation_pin_passes(lib):
    moved, du, _ = F.layer_translation(3.0, lib=lib)
    return bool(np.isfinite(du) and abs(moved - 1) < 0.03 and du < 0.08)


# (name, text of the oracle, planted replacement, pin that must fail)
MUTANTS = [
    ("electric stress sign (Eq. 31)",
     "s->kappa * lap_phi -\n         0.5 * deps_of(s, phi)", "s->kappa * lap_phi +\n         0.5 * deps_of(s, phi)",
     maxwell_pin_passes),
    ("electric stress without its 1/2 (Eq. 31)",
     "s->kappa * lap_phi -\n         0.5 * deps_of(s, phi)", "s->kappa * lap_phi -\n         1.0 * deps_of(s, phi)",
     maxwell_pin_passes),
    ("electric stress dropped (Eq. 31)",
     "s->kappa * lap_phi -\n         0.5 * deps_of(s, phi)", "s->kappa * lap_phi -\n         0.0 * deps_of(s, phi)",
     maxwell_pin_passes),
    ("Coulomb force dropped (Eq. 30)",
     "double Fx = mu_c * gphx + q * Ex, Fy = mu_c * gphy + q * Ey;",
     "double Fx = mu_c * gphx, Fy = mu_c * gphy;", coulomb_pin_passes),
    ("Coulomb force reversed (Eq. 30)",
     "double Fx = mu_c * gphx + q * Ex, Fy = mu_c * gphy + q * Ey;",
     "double Fx = mu_c * gphx - q * Ex, Fy = mu_c * gphy - q * Ey;", coulomb_pin_passes),
    ("density law with the phases swapped (Eq. 36)",
     "return phi * (s->p.rho_l - s->p.rho_v) + s->p.rho_v;",
     "return phi * (s->p.rho_v - s->p.rho_l) + s->p.rho_l;", shear_pin_passes),
    ("viscosity law with the phases swapped (Eq. 36)",
     "return phi * (s->p.mu_l - s->p.mu_v) + s->p.mu_v;",
     "return phi * (s->p.mu_v - s->p.mu_l) + s->p.mu_l;", shear_pin_passes),
    ("tau_f from mu alone, without rho (Eq. 42)",
     "double tau_f = 0.5 + mu_of(s, phi) / (rho * cs2);", "double tau_f = 0.5 + mu_of(s, phi) / cs2;",
     shear_pin_passes),
    ("u.grad(rho) dropped from R_i (Eq. 39)",
     "out[i] = w[i] * (ugr + cF / cs2 + contr / cs2);", "out[i] = w[i] * (cF / cs2 + contr / cs2);",
     translation_pin_passes),
    ("(u grad rho):(c c - c_s^2 I) dropped from R_i (Eq. 39)",
     "out[i] = w[i] * (ugr + cF / cs2 + contr / cs2);", "out[i] = w[i] * (ugr + cF / cs2);",
     translation_pin_passes),
    ("u.grad(rho)/2 dropped from the pressure (Eq. 44)",
     "(sumf + 0.5 * (ux * grx + uy * gry) + rho * s_i(0, ux, uy));\n\n      double mu_c",
     "(sumf + rho * s_i(0, ux, uy));\n\n      double mu_c", translation_pin_passes),
    ("grad(rho) reversed (chain rule of Eq. 36)",
     "double grx = (s->p.rho_l - s->p.rho_v) * gphx, gry = (s->p.rho_l - s->p.rho_v) * gphy;\n\n      /* charge",
     "double grx = (s->p.rho_v - s->p.rho_l) * gphx, gry = (s->p.rho_v - s->p.rho_l) * gphy;\n\n      /* charge",
     translation_pin_passes),
]


@pytest.mark.parametrize("name,find,replace,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(name, find, replace, pin, tmp_path):
    import oracle
    src = oracle.source()
    assert src.count(find) == 1, f"the text to mutate must occur once: {find!r}"
    lib = oracle.build_variant(src.replace(find, replace), os.path.join(str(tmp_path), "mutant.so"))
    with np.errstate(all="ignore"):
        assert not pin(lib), f"the pin still passes with: {name}"


def test_pins_pass_on_the_oracle_itself():
    """The same pin functions accept the unmodified oracle (so a failure
    above is the mutant's, not the pin's)."""
    assert maxwell_pin_passes(None)
    assert coulomb_pin_passes(None)
    assert shear_pin_passes(None)
    assert translation_pin_passes(None)
