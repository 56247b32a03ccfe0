"""Pins of the Mie-Gruneisen solid EOS in the oracle (Section IV.A names the
EOS and the cut-off pressure; the form is the linear shock-velocity one),
CPU only.  The pins come from the shock jump conditions and calculus, not
from the formula as coded."""
import math

import numpy as np
import pytest

import sph_synth as S
from oracle import cpu

P = S.c6_hvi(dx=2.5e-4, plate_half=3e-3).params
RHO0, C0, SS, G0, G = P["rho0"], P["c0"], P["mg_s"], P["mg_gamma0"], P["G"]


@pytest.mark.parametrize("up", [50.0, 400.0, 1500.0, 3000.0])
def test_states_on_the_hugoniot(up):
    """A steady shock with particle speed up and shock speed Us = c0 + s up:
    mass and momentum jumps give rho = rho0 Us / (Us - up) and p = rho0 Us up,
    the energy jump e = up^2 / 2.  The EOS must return that p there."""
    us = C0 + SS * up
    rho = RHO0 * us / (us - up)
    p, _ = cpu.eos(P, rho, 0.5 * up * up)
    assert p == pytest.approx(RHO0 * us * up, rel=1e-12)


def test_thermal_term_and_reference_state():
    for e in (0.0, 1e4, 3e5):
        p, _ = cpu.eos(P, RHO0, e)
        assert p == pytest.approx(G0 * RHO0 * e, rel=1e-15, abs=0.0)
    p, c = cpu.eos(P, RHO0, 0.0)
    assert p == 0.0
    assert c == pytest.approx(math.sqrt(C0 * C0 + 4.0 * G / (3.0 * RHO0)), rel=1e-15)


def test_tension_branch_and_cut_off():
    mu = -0.01
    p, c = cpu.eos(P, RHO0 * (1 + mu), 0.0)
    assert p == pytest.approx(RHO0 * C0 * C0 * mu, rel=1e-13)
    assert c == pytest.approx(math.sqrt(C0 * C0 + 4.0 * G / (3.0 * RHO0 * (1 + mu))), rel=1e-13)
    p, _ = cpu.eos(P, RHO0 * 0.95, 0.0)          # rho0 c0^2 (-0.05) = -3.9 GPa, below the cut-off
    assert p == P["p_cut"]


def test_branches_meet_at_the_reference_density():
    for e in (0.0, 2e5):
        lo = cpu.eos(P, RHO0 * (1 - 1e-9), e)
        hi = cpu.eos(P, RHO0 * (1 + 1e-9), e)
        assert hi[0] - lo[0] == pytest.approx(RHO0 * C0 * C0 * 2e-9, rel=1e-4)
        assert hi[1] == pytest.approx(lo[1], rel=1e-8)


@pytest.mark.parametrize("mu,e", [(0.05, 0.0), (0.2, 1e5), (0.45, 8e5), (-0.02, 2e5)])
def test_sound_speed_is_the_isentropic_derivative(mu, e):
    """c^2 - 4G/(3 rho) = dp/drho at fixed e + (p / rho^2) dp/de, both
    derivatives by central differences of the EOS itself."""
    rho = RHO0 * (1 + mu)
    p, c = cpu.eos(P, rho, e)
    dr, de = rho * 1e-6, max(abs(e), 1e4) * 1e-4
    dpdr = (cpu.eos(P, rho + dr, e)[0] - cpu.eos(P, rho - dr, e)[0]) / (2 * dr)
    dpde = (cpu.eos(P, rho, e + de)[0] - cpu.eos(P, rho, e - de)[0]) / (2 * de)
    cb2 = dpdr + max(p, 0.0) * dpde / (rho * rho)
    assert c * c - 4.0 * G / (3.0 * rho) == pytest.approx(cb2, rel=1e-6)


def test_hvi_workload_shape():
    wl = S.c6_hvi()
    t = wl.extra["types"]
    assert 6.4e6 < wl.n < 6.8e6 and 4.5e4 < int(t.sum()) < 6e4
    bead = wl.x[t == 1]
    assert bead[:, 2].min() > 2e-3                # above the plate before impact
    sp = np.linalg.norm(wl.v[t == 1], axis=1)
    assert np.allclose(sp, 4050.0) and np.all(wl.v[t == 0] == 0.0)
    ang = math.degrees(math.acos(-wl.v[t == 1][0, 2] / 4050.0))
    assert ang == pytest.approx(32.0)
