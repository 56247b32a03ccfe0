"""The oracle's pins have teeth: copies of the oracle, each with one plausible
mistake planted in its source (a dropped term, a flipped sign, a wrong
factor), are compiled on the CPU and must fail the pins that cover that
term.  Nothing here touches the GPU path; the planted mistakes live only in
temporary copies of the oracle.

Each mutation names the term it breaks (the readings of the pair terms,
update and stress stage of Sections I-II), the exact text it replaces in
``oracle/sph_oracle.c`` (the test fails loudly if that text is gone, so a
change to the oracle cannot silently disarm it) and the checks expected to
catch it.
"""
import os

import pytest

from tests import test_oracle_physics as phys
from tests import test_oracle_rates as rates
from oracle import build as obuild
from oracle import cpu

SRC = obuild.SRC

# (id, what is mistaken, original text, mutated text, checks that must fail)
MUTATIONS = [
    ("E_star_no_kinetic", "interface energy E* without |v*|^2 / 2",
     "double Es = 0.5 * (ei + ej) + 0.5 * ((vs[0] * vs[0] + vs[1] * vs[1]) + vs[2] * vs[2]);",
     "double Es = 0.5 * (ei + ej);",
     [rates.check_energy_rate_boost]),
    ("work_pbar", "pressure work with the mean pressure instead of the interface pressure",
     "out[4] = -A * (Phi * Es + ((t[0] * vs[0] + t[1] * vs[1]) + t[2] * vs[2]));",
     "out[4] = -A * (Phi * Es + pb * ((g[0] * vs[0] + g[1] * vs[1]) + g[2] * vs[2]));",
     [rates.check_energy_rate_boost]),
    ("work_vi", "pressure work against the target's velocity instead of v*",
     "out[4] = -A * (Phi * Es + ((t[0] * vs[0] + t[1] * vs[1]) + t[2] * vs[2]));",
     "out[4] = -A * (Phi * Es + ((t[0] * vi[0] + t[1] * vi[1]) + t[2] * vi[2]));",
     [rates.check_first_law]),
    ("energy_flux_sign", "sign of the advected energy flux",
     "out[4] = -A * (Phi * Es + ",
     "out[4] = -A * (-Phi * Es + ",
     [rates.check_energy_rate_boost]),
    ("volume_rate_sign", "sign of the volume rate",
     "out[5] = wi * wj * ((dv[0] * g[0] + dv[1] * g[1]) + dv[2] * g[2]);",
     "out[5] = -wi * wj * ((dv[0] * g[0] + dv[1] * g[1]) + dv[2] * g[2]);",
     [rates.check_volume_rate_divergence, rates.check_first_law, rates.check_acoustic_pulse]),
    ("volume_rate_no_wj", "volume rate without the source volume",
     "out[5] = wi * wj * ((dv[0] * g[0] + dv[1] * g[1]) + dv[2] * g[2]);",
     "out[5] = wi * ((dv[0] * g[0] + dv[1] * g[1]) + dv[2] * g[2]);",
     [rates.check_volume_rate_divergence, rates.check_first_law]),
    ("pair_weight_half", "pair weight w_i w_j instead of 2 w_i w_j",
     "double A = 2.0 * wi * wj;\n    double Phi",
     "double A = wi * wj;\n    double Phi",
     [rates.check_acoustic_pulse, rates.check_first_law]),
    ("traction_sign", "sign of the deviatoric stress traction",
     "t[a] = ps * g[a] - F * Snbar[a];",
     "t[a] = ps * g[a] + F * Snbar[a];",
     [rates.check_solid_traction, rates.check_elastic_pulse]),
    ("normal_stress_sign", "sign of n.S.n in the solid's Riemann pressure",
     "Pi = pi_ - ((n[0] * ai[0] + n[1] * ai[1]) + n[2] * ai[2]);\n"
     "        Pj = pj - ((n[0] * bj[0] + n[1] * bj[1]) + n[2] * bj[2]);",
     "Pi = pi_ + ((n[0] * ai[0] + n[1] * ai[1]) + n[2] * ai[2]);\n"
     "        Pj = pj + ((n[0] * bj[0] + n[1] * bj[1]) + n[2] * bj[2]);",
     [rates.check_solid_normal_stress_is_pressure]),
    ("gravity_work_dropped", "energy update without the work of gravity",
     "double En = (m * s->E[i] + dt * (r[4] + m * gv)) / mn;",
     "double En = (m * s->E[i] + dt * r[4]) / mn;",
     [rates.check_gravity_work]),
    ("shear_modulus_half", "Jaumann stress rate with G instead of 2G",
     "Sd[a][b] = 2.0 * G * (D[a][b]",
     "Sd[a][b] = G * (D[a][b]",
     [rates.check_elastic_pulse]),
    ("mass_flux_sign", "sign of the Riemann mass flux",
     "out[0] = -A * Phi;",
     "out[0] = A * Phi;",
     [rates.check_energy_rate_boost, phys.test_pair_matches_linear_riemann_closed_form]),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("mid,what,orig,mut,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, source, mid, what, orig, mut, checks):
    assert source.count(orig) == 1, f"mutation {mid}: its text is not (uniquely) in the oracle"
    path = os.path.join(str(tmp_path), f"{mid}.c")
    with open(path, "w") as f:
        f.write(source.replace(orig, mut))
    lib = obuild.build(src=path, out=os.path.join(str(tmp_path), f"lib{mid}.so"))
    with cpu.use_library(lib):
        for chk in checks:
            with pytest.raises(AssertionError):
                chk()
