"""Pins of the oracle's energy rate, volume rate, solid traction, gravity work
and wave speeds, each against a property that the physics fixes and that the
oracle's own formulas do not restate (CPU only).

The paper names Gamma-SPH-ALE (Section I) but prints none of its equations,
so the pair terms follow a documented reading; these checks tie that reading
to facts outside it:

* a Galilean boost of the velocities at fixed internal energy changes the
  energy rate by exactly U.(mv)' + |U|^2 m' / 2 (the energy of a moving frame);
* with the Riemann dissipation off and a uniform pressure, the energy rate
  minus the kinetic part v.(mv)' is the pressure work -p w' (first law);
* the volume rate of v = A x on a perfect lattice is w kappa tr(A) (the
  discrete divergence, kappa the lattice sum of (x_j - x_i) grad W);
* the stress traction of a deviatoric stress linear in x is w kappa div(S)
  (momentum balance of a solid at rest);
* along the pair axis a solid's normal stress acts as a pressure -n.sigma.n,
  so its mass flux and normal momentum equal those of a fluid with that
  pressure;
* gravity does the work m g.v in the energy update;
* a small planar pulse travels at the sound speed c0 (fluid) and at the
  longitudinal speed sqrt((K + 4G/3) / rho0) = 6.2 km/s (the cylinder's metal).

Each ``check_*`` function raises AssertionError on failure; the tests call
them on the oracle as built, and ``test_oracle_mutations`` calls them on
copies of the oracle with one term deliberately mistaken.
"""
import json
import os

import numpy as np
import pytest

import sph_synth as S
from oracle import cpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def kappa():
    with open(GOLDEN) as f:
        return json.load(f)["lattice_sums_h1.3"]["sum_xgradW_diag"]


def _cloud(seed, beta=1.0, solid=False):
    """Jittered 7^3 lattice with random velocities, densities and internal
    energies (EOS pressures), sorted into buckets."""
    rng = np.random.default_rng(seed)
    if solid:
        w = S.solid_block(7, seed=seed, s_sigma=1e7)
    else:
        w = S.jittered_lattice(7, seed=seed, jitter=0.3, rho_sigma=0.01, v_sigma=0.5)
    P = dict(w.params, beta=beta)
    s = cpu.State.from_workload(w)
    e = rng.uniform(0.0, 5.0, size=w.n)
    s.E[:] = e + 0.5 * (s.v ** 2).sum(1)
    cpu.prime(P, s)
    srt, _, start = cpu.build_cells(w.grid, s)
    return w, P, srt, start


def _interior(srt, dx, n_side, margin=3):
    ix = np.round(srt.x / dx - 0.5).astype(int)
    return np.all((ix >= margin) & (ix <= n_side - 1 - margin), axis=1)


# ----------------------------------------------------------- energy rate

def check_energy_rate_boost(seed=41, solid=False):
    """v -> v + U at fixed e: (mE)' -> (mE)' + U.(mv)' + |U|^2 m' / 2, per target."""
    w, P, srt, start = _cloud(seed, solid=solid)
    R0 = cpu.interact(P, w.grid, cpu.FORCE, srt, srt, start, True)
    U = np.array([2.5, -1.25, 0.75])
    b = srt.copy()
    b.v += U
    b.E = srt.E + srt.v @ U + 0.5 * U @ U
    R1 = cpu.interact(P, w.grid, cpu.FORCE, b, b, start, True)
    scale = cpu.interact_abs(P, w.grid, cpu.FORCE, b, b, start, True)
    want = R0[:, 4] + R0[:, 1:4] @ U + 0.5 * (U @ U) * R0[:, 0]
    err = np.abs(R1[:, 4] - want)
    assert np.all(err <= 1e-12 * scale[:, 4] + 1e-300), err.max() / scale[:, 4].max()
    # the rates that do not depend on the frame
    assert np.all(np.abs(R1[:, 0] - R0[:, 0]) <= 1e-12 * scale[:, 0])
    assert np.all(np.abs(R1[:, 5] - R0[:, 5]) <= 1e-12 * scale[:, 5])
    # and the test has teeth: the energy rate really moves with the frame
    assert np.abs(R1[:, 4] - R0[:, 4]).max() > 1e-3 * np.abs(R0[:, 4]).max()


def check_first_law(seed=42):
    """beta = 0, uniform p, any velocity field: (mE)' - v.(mv)' = -p w'."""
    w, P, srt, start = _cloud(seed, beta=0.0)
    p = 3.7e4
    srt.p[:] = p
    R = cpu.interact(P, w.grid, cpu.FORCE, srt, srt, start, True)
    scale = cpu.interact_abs(P, w.grid, cpu.FORCE, srt, srt, start, True)
    lhs = R[:, 4] - np.einsum("ij,ij->i", srt.v, R[:, 1:4])
    tol = 1e-12 * (scale[:, 4] + np.abs(srt.v).sum(1) * scale[:, 1:4].max(1) + p * scale[:, 5])
    assert np.all(np.abs(lhs + p * R[:, 5]) <= tol)
    assert np.abs(R[:, 5]).max() > 0.0


# ----------------------------------------------------------- volume rate

def check_volume_rate_divergence():
    """v = A x on a perfect lattice: w' = w kappa tr(A) inside."""
    n_side = 12
    w = S.jittered_lattice(n_side, seed=0, jitter=0.0)
    s = cpu.State.from_workload(w)
    A = np.array([[0.3, -1.0, 0.2], [0.5, -0.7, -0.4], [0.0, 0.7, 1.1]])
    s.v[:] = s.x @ A.T
    s.E[:] = 0.5 * (s.v ** 2).sum(1)
    cpu.prime(w.params, s)
    srt, _, start = cpu.build_cells(w.grid, s)
    R = cpu.interact(w.params, w.grid, cpu.FORCE, srt, srt, start, True)
    inner = _interior(srt, w.extra["dx"], n_side)
    want = srt.w[inner] * kappa() * np.trace(A)
    assert np.allclose(R[inner, 5], want, rtol=1e-9, atol=0.0), np.abs(R[inner, 5] / want - 1).max()
    # a rotation has no divergence
    s.v[:] = s.x @ np.array([[0.0, -1.0, 0.5], [1.0, 0.0, -0.3], [-0.5, 0.3, 0.0]]).T
    s.E[:] = 0.5 * (s.v ** 2).sum(1)
    srt, _, start = cpu.build_cells(w.grid, s)
    R = cpu.interact(w.params, w.grid, cpu.FORCE, srt, srt, start, True)
    assert np.abs(R[inner, 5]).max() <= 1e-9 * abs(want).max()


# ---------------------------------------------------------- solid traction

def _solid_lattice(n_side):
    w = S.solid_block(n_side, seed=0, vz=0.0)
    dx = w.extra["dx"]
    w.x[:] = S._lattice(n_side, n_side, n_side, dx)       # no jitter
    s = cpu.State.from_workload(w)
    s.v[:] = 0.0
    s.E[:] = 0.0
    return w, s, dx


def check_solid_traction(beta=0.0):
    """At rest, p = 0, S deviatoric and linear in x: (mv)' = w kappa div(S) inside."""
    n_side = 12
    w, s, dx = _solid_lattice(n_side)
    P = dict(w.params, beta=beta)
    cpu.prime(P, s)                         # rho = rho0: p = 0
    assert np.all(s.p == 0.0)
    rng = np.random.default_rng(43)
    S0 = np.array([1e7, -4e6, -6e6, 2e6, -3e6, 1e6])
    B = rng.normal(size=(3, 6)) * 1e9        # dS/dx_c for c = 0, 1, 2 (Pa/m)
    B[:, 2] = -(B[:, 0] + B[:, 1])           # traceless
    s.S[:] = S0 + s.x @ B
    srt, _, start = cpu.build_cells(w.grid, s)
    R = cpu.interact(P, w.grid, cpu.FORCE, srt, srt, start, True)
    # div S: (div S)_a = sum_b d S_ab / d x_b, S stored as (xx yy zz xy xz yz)
    full = [[0, 3, 4], [3, 1, 5], [4, 5, 2]]
    div = np.array([sum(B[b, full[a][b]] for b in range(3)) for a in range(3)])
    inner = _interior(srt, dx, n_side)
    want = srt.w[inner, None] * kappa() * div[None, :]
    err = np.abs(R[inner, 1:4] - want).max()
    assert err <= 1e-8 * np.abs(want).max(), err / np.abs(want).max()


def check_solid_normal_stress_is_pressure(seed=44):
    """Along n a solid acts as a fluid of pressure p - n.S.n: equal mass flux
    and equal normal momentum for the same pair (beta = 1)."""
    rng = np.random.default_rng(seed)
    Ps = dict(S.c3_cylinder(dx=1e-3, radius=2e-3, nlayers=1).params, h=1.3e-3)
    full = [[0, 3, 4], [3, 1, 5], [4, 5, 2]]
    for _ in range(100):
        d = rng.normal(size=3)
        d *= rng.uniform(0.2, 1.9) * 1.3e-3 / np.linalg.norm(d)
        n = d / np.linalg.norm(d)
        vi, vj = rng.normal(size=3), rng.normal(size=3)
        Si, Sj = rng.normal(size=6) * 1e8, rng.normal(size=6) * 1e8
        pi, pj = rng.normal() * 1e8, rng.normal() * 1e8
        st = dict(wi=1e-9, wj=1.1e-9, rhoi=2700.0, rhoj=2710.0, ci=6198.0, cj=6198.0, ei=1.0, ej=2.0)
        a = cpu.pair(Ps, d, vi, vj, pi=pi, pj=pj, Si=Si, Sj=Sj, **st)
        Mi = np.array([[Si[k] for k in row] for row in full])
        Mj = np.array([[Sj[k] for k in row] for row in full])
        qi, qj = pi - n @ Mi @ n, pj - n @ Mj @ n
        b = cpu.pair(Ps, d, vi, vj, pi=qi, pj=qj, **st)
        assert abs(a[0] - b[0]) <= 1e-12 * (abs(a[0]) + abs(b[0])) + 1e-300
        an, bn = a[1:4] @ n, b[1:4] @ n
        assert abs(an - bn) <= 1e-10 * (np.abs(a[1:4]).sum() + np.abs(b[1:4]).sum())


# ---------------------------------------------------------------- gravity

def check_gravity_work():
    """One free-flight step: E+ = E + dt g.v (the work of gravity over the step),
    so the internal energy moves only by the O(dt^2) term -dt^2 |g|^2 / 2."""
    w = S.jittered_lattice(4, seed=2, walls=True)
    P = dict(w.params, gravity=[0.3, -0.2, -9.81])
    s = cpu.State.from_workload(w)
    s.E[:] = 3.0 + 0.5 * (s.v ** 2).sum(1)
    cpu.prime(P, s)
    g = np.asarray(P["gravity"])
    E0, v0 = s.E.copy(), s.v.copy()
    dt = 1e-3
    cpu.integrate(P, cpu.MOTION, s, rates=np.zeros((w.n, 6)), dt=dt)
    assert np.allclose(s.E, E0 + dt * (v0 @ g), rtol=1e-15, atol=1e-15)
    e1 = s.E - 0.5 * (s.v ** 2).sum(1)
    assert np.allclose(e1, 3.0 - 0.5 * dt * dt * (g @ g), rtol=0, atol=1e-12)


# ------------------------------------------------------------ wave speeds

def _pulse_speeds(solid, beta=1.0, nx=40, ny=40, sig=4.0, x0=14.0, travel=10.0, core=3,
                  eps=1e-5):
    """Speeds of a right-going planar pulse (Gaussian, width sig dx) along x in
    an nx by ny by ny lattice with free surfaces, divided by the expected wave
    speed c.  The pulse starts as the simple wave of linear acoustics
    (rho' = rho0 eps g, u = c eps g; for the solid also the uniaxial-strain
    deviatoric stress) and runs `travel` dx.  Over the particles within `core`
    dx of the bar's axis, which the release waves from the lateral surfaces
    do not reach in that time, the centroids of u, of rho - rho0 and of the
    normal stress sigma_xx each move at c in linear acoustics; each one's
    speed rests on a different equation (momentum, continuity, the EOS or
    stress rate), so together they pin c^2 and not only one factor of it.
    Returns (speeds of the three centroids / c, c)."""
    dx = 1e-3
    w = S.jittered_lattice(0, seed=0, dx=dx, jitter=0.0, v_sigma=0.0, dims=(nx, ny, ny))
    if solid:
        P = dict(S.c3_cylinder(dx=dx, radius=2 * dx, nlayers=1).params, h=1.3 * dx)
    else:
        P = dict(w.params)
    P.update(beta=beta, wall_mask=0)
    s = cpu.State(w.n, solid=solid)
    s.x[:] = w.x
    s.w[:] = dx ** 3
    s.id[:] = w.id
    g = np.exp(-0.5 * ((w.x[:, 0] / dx - x0) / sig) ** 2)
    rho0 = P["rho0"]
    if solid:
        K, G = P["K"], P["G"]
        c = np.sqrt((K + 4.0 * G / 3.0) / rho0)
        s.S[:, 0] = -4.0 / 3.0 * G * eps * g
        s.S[:, 1] = 2.0 / 3.0 * G * eps * g
        s.S[:, 2] = 2.0 / 3.0 * G * eps * g
    else:
        c = P["c0"]
    s.m[:] = rho0 * (1.0 + eps * g) * dx ** 3
    s.v[:, 0] = c * eps * g
    s.E[:] = 0.5 * (s.v ** 2).sum(1)
    cpu.prime(P, s)
    dt = 0.3 * P["h"] / c
    nst = int(round(travel * dx / c / dt))
    iy = np.round(w.x[:, 1] / dx - 0.5).astype(int)
    iz = np.round(w.x[:, 2] / dx - 0.5).astype(int)
    core_ids = (np.abs(iy - (ny - 1) / 2) < core) & (np.abs(iz - (ny - 1) / 2) < core)

    def centroids(st):
        b = st.by_id()
        x = b.x[core_ids, 0]
        sxx = -b.p[core_ids] + (b.S[core_ids, 0] if solid else 0.0)
        fields = (b.v[core_ids, 0], b.rho[core_ids] - rho0, sxx)
        return np.array([(f * x).sum() / f.sum() for f in fields])

    x_a = centroids(s)
    cpu.run(P, w.grid, s, nst, fixed_dt=dt)
    x_b = centroids(s)
    return (x_b - x_a) / (nst * dt) / c, c


def check_acoustic_pulse():
    """A small planar pulse travels at c0 (the lattice's long-wave factor
    kappa = 0.9935 and the Riemann dissipation keep it within ~2 %)."""
    r1, c = _pulse_speeds(False, beta=1.0)
    assert c == 50.0
    assert np.all(np.abs(r1 - 1.0) < 0.03), r1
    r0, _ = _pulse_speeds(False, beta=0.0)
    assert np.all(np.abs(r0 - 1.0) < 0.015), r0


def check_elastic_pulse():
    """The cylinder's metal carries a small longitudinal pulse at
    sqrt((K + 4G/3) / rho0) = 6.2 km/s."""
    r, c = _pulse_speeds(True, beta=1.0)
    assert abs(c - 6198.0) < 1.0
    assert np.all(np.abs(r - 1.0) < 0.03), r


# ------------------------------------------------------------------ tests

@pytest.mark.parametrize("solid", [False, True])
def test_energy_rate_boost_identity(solid):
    check_energy_rate_boost(solid=solid)


def test_first_law_without_dissipation():
    check_first_law()


def test_volume_rate_is_lattice_divergence():
    check_volume_rate_divergence()


def test_solid_traction_is_stress_divergence():
    check_solid_traction()


def test_solid_normal_stress_acts_as_pressure():
    check_solid_normal_stress_is_pressure()


def test_gravity_work_in_energy():
    check_gravity_work()


def test_acoustic_pulse_travels_at_c0():
    check_acoustic_pulse()


def test_elastic_pulse_travels_at_longitudinal_speed():
    check_elastic_pulse()
