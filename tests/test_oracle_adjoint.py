"""Pins of the reverse-mode reference (oracle/torch_ref.py), CPU only.

The dense PyTorch forward must reproduce the C oracle's steps (two
independent codes of the same reading), and its autograd gradient of the
final kinetic energy must match central finite differences of itself."""
import numpy as np
import pytest
import torch

import sph_synth as S
from oracle import cpu, torch_ref


def small_box(n_side=6, seed=70):
    w = S.jittered_lattice(n_side, seed=seed, dx=2e-3, jitter=0.05, v_sigma=1.0, rho_sigma=0.002)
    w.params["c0"] = 50.0
    return w


def test_dense_forward_matches_c_oracle():
    w = small_box()
    dt, nsteps = 1.4e-5, 4
    s = cpu.State.from_workload(w)
    cpu.run(w.params, w.grid, s, nsteps, fixed_dt=dt)
    ref = s.by_id()
    got = torch_ref.final_state(w, w.params["c0"], dt, nsteps)
    for f, a in (("x", ref.x), ("v", ref.v), ("m", ref.m), ("w", ref.w), ("E", ref.E)):
        err = np.abs(got[f] - a).max() / np.abs(a).max()
        assert err < 1e-13, (f, err)


def test_reverse_mode_matches_central_differences():
    w = small_box(n_side=5, seed=71)
    dt, nsteps, c0 = 1.4e-5, 3, 50.0
    J, gv, gc = torch_ref.gradient(w, c0, dt, nsteps)
    rng = np.random.default_rng(72)
    x0 = torch.tensor(w.x)
    m0 = torch.tensor(w.m)
    w0 = torch.tensor(w.omega)
    e0 = torch.tensor(w.E - 0.5 * (w.v * w.v).sum(1))

    def Jof(v, c):
        with torch.no_grad():
            return float(torch_ref.kinetic_energy_after(x0, torch.tensor(v), m0, w0, e0, w.params, c, dt, nsteps))

    for _ in range(3):
        d = rng.normal(size=w.v.shape)
        eps = 1e-5
        fd = (Jof(w.v + eps * d, c0) - Jof(w.v - eps * d, c0)) / (2 * eps)
        assert fd == pytest.approx(float((gv * d).sum()), rel=1e-7)
    eps = 1e-4 * c0
    fdc = (Jof(w.v, c0 + eps) - Jof(w.v, c0 - eps)) / (2 * eps)
    assert fdc == pytest.approx(gc, rel=1e-6)
    assert gc != 0.0


def test_displacement_gradient_matches_central_differences():
    w = small_box(n_side=5, seed=73)
    dt, nsteps, c0 = 1.4e-5, 4, 50.0
    tag = np.flatnonzero(np.linalg.norm(w.x - w.x.mean(0), axis=1) < 3.0e-3)
    J, gv, gc = torch_ref.gradient_z_displacement(w, c0, dt, nsteps, tag)
    x0, m0, w0 = torch.tensor(w.x), torch.tensor(w.m), torch.tensor(w.omega)
    e0 = torch.tensor(w.E - 0.5 * (w.v * w.v).sum(1))
    t = torch.as_tensor(tag)

    def Jof(v, c):
        with torch.no_grad():
            return float(torch_ref.z_displacement_after(x0, torch.tensor(v), m0, w0, e0, w.params, c, dt, nsteps, t))

    assert abs(J - Jof(w.v, c0)) < 1e-18
    rng = np.random.default_rng(74)
    for _ in range(3):
        d = rng.normal(size=w.v.shape)
        eps = 1e-5
        fd = (Jof(w.v + eps * d, c0) - Jof(w.v - eps * d, c0)) / (2 * eps)
        assert fd == pytest.approx(float((gv * d).sum()), rel=1e-7)
    # displacement of a tagged set grows with its own initial z-velocity:
    # dJ/dv0_z is positive on the tag (about nsteps dt / n_tag) and small elsewhere
    assert gv[tag, 2].min() > 0.5 * nsteps * dt / tag.size
    eps = 1e-4 * c0
    fdc = (Jof(w.v, c0 + eps) - Jof(w.v, c0 - eps)) / (2 * eps)
    assert fdc == pytest.approx(gc, rel=1e-5, abs=1e-14)


def solid_block(seed, s_axial=0.0, rate=0.0, n_side=5):
    """A free J2 block of the cylinder's metal; with s_axial near Y0 and a
    stretch it yields (hardening H = E / 100)."""
    w = S.solid_block(n_side, seed=seed, vz=0.0, s_sigma=2e7, s_axial=s_axial, stretch_rate=rate)
    w.params = dict(w.params, wall_mask=0)
    return w


@pytest.mark.parametrize("plastic", [False, True])
def test_dense_solid_forward_matches_c_oracle(plastic):
    w = solid_block(90 + int(plastic), 270e6 if plastic else 0.0, 2e4 if plastic else 0.0)
    dt, nsteps = 2e-8, 4
    s = cpu.State.from_workload(w)
    cpu.run(w.params, w.grid, s, nsteps, fixed_dt=dt)
    ref = s.by_id()
    got = torch_ref.solid_final_state(w, dt, nsteps)
    for f in ("x", "v", "m", "w", "E", "S", "ep"):
        a = getattr(ref, f)
        err = np.abs(got[f] - a).max() / max(np.abs(a).max(), 1e-300)
        assert err < 1e-13, (f, err)
    assert ((ref.ep > 0).mean() > 0.8) == plastic


@pytest.mark.parametrize("plastic", [False, True])
def test_solid_reverse_mode_matches_central_differences(plastic):
    w = solid_block(92 + int(plastic), 270e6 if plastic else 0.0, 2e4 if plastic else 0.0, n_side=4)
    dt, nsteps = 2e-8, 3
    J, gv, gS = torch_ref.solid_gradient(w, dt, nsteps)
    t = {k: torch.tensor(getattr(w, k)) for k in ("x", "m", "omega", "eps_p")}
    e0 = torch.tensor(w.E - 0.5 * (w.v * w.v).sum(1))

    def Jof(v, Sx):
        with torch.no_grad():
            return float(torch_ref.solid_kinetic_energy_after(t["x"], torch.tensor(v), t["m"], t["omega"], e0,
                                                              torch.tensor(Sx), t["eps_p"], w.params, dt, nsteps))

    rng = np.random.default_rng(94)
    for _ in range(3):
        d = rng.normal(size=w.v.shape)
        eps = 1e-4
        fd = (Jof(w.v + eps * d, w.S) - Jof(w.v - eps * d, w.S)) / (2 * eps)
        assert fd == pytest.approx(float((gv * d).sum()), rel=1e-7)
        dS = rng.normal(size=w.S.shape)
        epsS = 1e2     # Pa, against stresses of 1e7 - 1e8
        fd = (Jof(w.v, w.S + epsS * dS) - Jof(w.v, w.S - epsS * dS)) / (2 * epsS)
        assert fd == pytest.approx(float((gS * dS).sum()), rel=1e-6)
