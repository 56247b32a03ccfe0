"""GPU parity of the hand adjoint (through the C ABI): fluids (one set and
two sets with both local-remote passes) and J2 solids.

* Against reverse mode: the dense float64 PyTorch reference (autograd) on a
  small free box, FP64 form, |dJ/dv0 (GPU) - reference| <= 1e-9 max|ref|
  and dJ/dc0 within 1e-9 relative (both are FP64 evaluations of the same
  function; summation orders differ).
* Against central finite differences on the full 250,047-particle box,
  50 steps, checkpoints every 10: along random directions d,
  |FD - <dJ/dv0, d>| <= 1e-6 |FD| with eps = 1e-4, and likewise for c0.
* The FP32-split form's gradient is reported against the FP64 one.
"""
import numpy as np
import pytest
import torch

import sph_synth as S
from oracle import torch_ref

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_box(n_side=6, seed=80):
    w = S.jittered_lattice(n_side, seed=seed, dx=2e-3, jitter=0.05, v_sigma=1.0, rho_sigma=0.002)
    w.params["c0"] = 50.0
    return w


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_objective_seed_and_input_stage_match_their_definitions(prec):
    """The two ends of a reverse pass against their definitions on a sorted
    random state (ids out of array order, 1,728 particles: several workgroups
    and a ragged one).  sph_objective_adjoint overwrites every cotangent
    field: kinetic energy v-bar = s m v, m-bar = s |v|^2 / 2; tagged mean z
    z-bar = s / ntag on the tagged ids (ids at or above the tag table's
    length untagged); everything else 0.  Both are FP64 arithmetic rounded
    once, equal to NumPy's evaluation in the same order.  The INPUT_VELOCITY
    stage adds E-bar v to v-bar, within two roundings of the form's
    precision of |v-bar| + |E-bar v| (the kernel may fuse the multiply-add);
    E-bar is left as it was."""
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.adjoint import Cotangent
    from paper_2310_03596_amd.sim import Sim
    from paper_2310_03596_amd.state import stream_handle
    wl = small_box(12, seed=81)
    n = wl.n
    print(f"[objective seed] n={n} prec={prec}", flush=True)
    sim = Sim(wl, prec)
    sim.build()
    torch.cuda.synchronize()
    h = sim.A.host()
    assert not np.array_equal(h["id"], np.arange(n))
    nd = np.float64 if prec == FP64 else np.float32
    st = stream_handle()
    s = -1.75
    bar = Cotangent(n, prec, "cuda", solid=True)
    def poison():
        for t in (bar.x, bar.v, bar.m, bar.w, bar.E, bar.rho, bar.p, bar.c, bar.e, bar.S, bar.ep):
            t.fill_(7.0)

    poison()
    L.sph_objective_adjoint(L.SPH_OBJ_KINETIC_ENERGY, sim.A.struct(), None, 0, 0, s, bar.struct(), st)
    torch.cuda.synchronize()
    v, m = h["v"].astype(np.float64), h["m"].astype(np.float64)
    assert np.array_equal(bar.v.cpu().numpy().T, ((s * m)[:, None] * v).astype(nd))
    assert np.array_equal(bar.m.cpu().numpy(), (s * 0.5 * ((v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1])
                                                            + v[:, 2] * v[:, 2])).astype(nd))
    for t in (bar.x, bar.w, bar.E, bar.rho, bar.p, bar.c, bar.e, bar.S, bar.ep):
        assert not t.cpu().numpy().any()
    # tagged mean z, with a tag table shorter than the ids: ids 400 and n - 1 fall outside it
    tag_ids = np.array([3, 17, 399, 400, n - 1])
    flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    flags[torch.as_tensor(tag_ids, device="cuda")] = 1
    poison()
    L.sph_objective_adjoint(L.SPH_OBJ_TAGGED_MEAN_Z, sim.A.struct(), flags.data_ptr(), 400, 3, s, bar.struct(), st)
    torch.cuda.synchronize()
    hit = np.isin(h["id"], tag_ids[:3])
    assert hit.sum() == 3
    assert np.array_equal(bar.x[2].cpu().numpy(), np.where(hit, s / 3, 0.0).astype(nd))
    for t in (bar.x[:2], bar.v, bar.m, bar.w, bar.E, bar.rho, bar.p, bar.c, bar.e, bar.S, bar.ep):
        assert not t.cpu().numpy().any()
    # the input-velocity stage
    g = torch.Generator(device="cpu").manual_seed(82)
    vb0 = torch.randn((3, n), generator=g, dtype=torch.float64).to(bar.v.dtype)
    Eb0 = torch.randn(n, generator=g, dtype=torch.float64).to(bar.E.dtype)
    bar.v.copy_(vb0)
    bar.E.copy_(Eb0)
    L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_INPUT_VELOCITY, sim.A.struct(), None, None, bar.struct(), None,
                            None, None, 0, st)
    torch.cuda.synchronize()
    vb, Eb = vb0.double().numpy(), Eb0.double().numpy()
    got = bar.v.double().cpu().numpy()
    prod = Eb[None, :] * v.T
    bound = 2 * np.finfo(nd).eps * (np.abs(vb) + np.abs(prod))
    assert (np.abs(got - (vb + prod)) <= bound).all()
    assert np.array_equal(bar.E.cpu().numpy(), Eb0.numpy())


def _rollout(w, prec, nsteps, ckpt, dt):
    from paper_2310_03596_amd.adjoint import KineticEnergyRollout
    return KineticEnergyRollout(w, prec, nsteps, ckpt, dt)


@pytest.mark.parametrize("nsteps,ckpt", [(5, 2), (6, 6), (4, 1)])
def test_adjoint_matches_reverse_mode(nsteps, ckpt):
    w = small_box()
    dt = 1.4e-5
    print(f"[adjoint vs reverse mode] n={w.n} steps={nsteps} ckpt={ckpt}", flush=True)
    J_ref, gv_ref, gc_ref = torch_ref.gradient(w, w.params["c0"], dt, nsteps)
    ro = _rollout(w, FP64, nsteps, ckpt, dt)
    J = ro.forward(w.v, w.params["c0"])
    gv, gc = ro.backward(1.0)
    assert J == pytest.approx(J_ref, rel=1e-13)
    assert np.abs(gv - gv_ref).max() <= 1e-9 * np.abs(gv_ref).max()
    assert gc == pytest.approx(gc_ref, rel=1e-9)


def test_adjoint_through_autograd_function():
    from paper_2310_03596_amd.adjoint import KineticEnergy
    w = small_box(n_side=5, seed=81)
    ro = _rollout(w, FP64, 3, 2, 1.4e-5)
    v0 = torch.tensor(w.v, dtype=torch.float64, requires_grad=True)
    c0 = torch.tensor(w.params["c0"], dtype=torch.float64, requires_grad=True)
    J = KineticEnergy.apply(v0, c0, ro)
    J.backward()
    _, gv_ref, gc_ref = torch_ref.gradient(w, w.params["c0"], 1.4e-5, 3)
    assert np.abs(v0.grad.numpy() - gv_ref).max() <= 1e-9 * np.abs(gv_ref).max()
    assert float(c0.grad) == pytest.approx(gc_ref, rel=1e-9)


def test_fp32_adjoint_close_to_fp64():
    w = small_box(n_side=8, seed=82)
    ro64 = _rollout(w, FP64, 6, 3, 1.4e-5)
    ro64.forward(w.v, 50.0)
    g64, c64 = ro64.backward(1.0)
    ro32 = _rollout(w, FP32, 6, 3, 1.4e-5)
    ro32.forward(w.v, 50.0)
    g32, c32 = ro32.backward(1.0)
    rel = np.abs(g32 - g64).max() / np.abs(g64).max()
    print(f"FP32 adjoint vs FP64: max rel {rel:.3e}, c0 {abs(c32 - c64) / abs(c64):.3e}")
    assert rel < 1e-3
    assert abs(c32 - c64) <= 1e-2 * abs(c64)


def test_adjoint_matches_central_differences_full_box():
    w = S.c5_box()
    dt, nsteps, ckpt = w.extra["dt"], w.extra["steps"], w.extra["ckpt"]
    c0 = w.params["c0"]
    print(f"[adjoint vs FD] n={w.n} steps={nsteps} ckpt={ckpt}", flush=True)
    ro = _rollout(w, FP64, nsteps, ckpt, dt)
    ro.forward(w.v, c0)
    gv, gc = ro.backward(1.0)
    rng = np.random.default_rng(5)
    eps = 1e-4
    worst = 0.0
    for k in range(64):
        d = rng.normal(size=w.v.shape)
        jp = _rollout(w, FP64, nsteps, nsteps, dt).forward(w.v + eps * d, c0)
        jm = _rollout(w, FP64, nsteps, nsteps, dt).forward(w.v - eps * d, c0)
        fd = (jp - jm) / (2 * eps)
        ad = float((gv * d).sum())
        rel = abs(fd - ad) / abs(fd)
        worst = max(worst, rel)
        if k % 16 == 0:
            print(f"direction {k}: FD {fd:.12e} adjoint {ad:.12e} rel {rel:.2e}", flush=True)
        assert rel <= 1e-6, (k, fd, ad)
    print(f"64 directions: worst relative difference {worst:.3e}", flush=True)
    h = 1e-4 * c0
    fdc = (_rollout(w, FP64, nsteps, nsteps, dt).forward(w.v, c0 + h)
           - _rollout(w, FP64, nsteps, nsteps, dt).forward(w.v, c0 - h)) / (2 * h)
    print(f"c0: FD {fdc:.12e} adjoint {gc:.12e}", flush=True)
    assert abs(fdc - gc) <= 1e-6 * abs(fdc)


def _tag_sphere(w, radius):
    c = 0.5 * (w.x.min(0) + w.x.max(0))
    return np.flatnonzero(np.linalg.norm(w.x - c, axis=1) < radius)


def test_displacement_adjoint_matches_reverse_mode():
    """Mean z-displacement of a tagged sphere: GPU adjoint (FP64) against the
    dense reverse-mode reference."""
    w = small_box(n_side=6, seed=83)
    dt, nsteps = 1.4e-5, 5
    tag = _tag_sphere(w, 3.5e-3)
    print(f"[displacement adjoint vs reverse mode] n={w.n} tagged={tag.size}", flush=True)
    J_ref, gv_ref, gc_ref = torch_ref.gradient_z_displacement(w, w.params["c0"], dt, nsteps, tag)
    from paper_2310_03596_amd.adjoint import KineticEnergyRollout
    ro = KineticEnergyRollout(w, FP64, nsteps, 2, dt, tag_ids=w.id[tag])
    J = ro.forward(w.v, w.params["c0"])
    gv, gc = ro.backward(1.0)
    assert J == pytest.approx(J_ref, rel=1e-11, abs=1e-18)
    assert np.abs(gv - gv_ref).max() <= 1e-9 * np.abs(gv_ref).max()
    assert abs(gc - gc_ref) <= 1e-8 * abs(gc_ref) + 1e-12 * np.abs(gv_ref).max()


def test_displacement_adjoint_matches_central_differences_full_box():
    """250,047 particles, 50 steps, checkpoints every 10; tag: the sphere of
    radius 10 dx at the box centre."""
    from paper_2310_03596_amd.adjoint import KineticEnergyRollout
    w = S.c5_box()
    dt, nsteps, ckpt = w.extra["dt"], w.extra["steps"], w.extra["ckpt"]
    c0 = w.params["c0"]
    tag = _tag_sphere(w, 10 * w.extra.get("dx", 2e-3))
    print(f"[displacement adjoint vs FD] n={w.n} tagged={tag.size}", flush=True)
    ro = KineticEnergyRollout(w, FP64, nsteps, ckpt, dt, tag_ids=w.id[tag])
    ro.forward(w.v, c0)
    gv, gc = ro.backward(1.0)
    rng = np.random.default_rng(6)
    eps = 1e-4

    def J(v, c):
        return KineticEnergyRollout(w, FP64, nsteps, nsteps, dt, tag_ids=w.id[tag]).forward(v, c)

    worst = 0.0
    for k in range(16):
        d = rng.normal(size=w.v.shape)
        fd = (J(w.v + eps * d, c0) - J(w.v - eps * d, c0)) / (2 * eps)
        ad = float((gv * d).sum())
        worst = max(worst, abs(fd - ad) / abs(fd))
        assert abs(fd - ad) <= 1e-6 * abs(fd), (k, fd, ad)
    print(f"16 directions: worst relative difference {worst:.3e}", flush=True)
    h = 1e-4 * c0
    fdc = (J(w.v, c0 + h) - J(w.v, c0 - h)) / (2 * h)
    print(f"c0: FD {fdc:.12e} adjoint {gc:.12e}", flush=True)
    assert abs(fdc - gc) <= 1e-6 * abs(fdc)


def test_fp32_adjoint_full_box_error():
    """The adjoint configuration as prescribed (250,047 particles, 50 FP32
    steps, checkpoints every 10): the FP32-split gradient against the FP64
    adjoint (max-norm and RMS, relative) and, along 8 random directions,
    against central differences of the FP64 forward."""
    w = S.c5_box()
    dt, nsteps, ckpt = w.extra["dt"], w.extra["steps"], w.extra["ckpt"]
    c0 = w.params["c0"]
    print(f"[FP32 adjoint full box] n={w.n} steps={nsteps} ckpt={ckpt}", flush=True)
    out = {}
    for prec in (FP64, FP32):
        ro = _rollout(w, prec, nsteps, ckpt, dt)
        ro.forward(w.v, c0)
        out[prec] = ro.backward(1.0)
        del ro
    g64, c64 = out[FP64]
    g32, c32 = out[FP32]
    rel_max = np.abs(g32 - g64).max() / np.abs(g64).max()
    rel_rms = np.sqrt(np.mean((g32 - g64) ** 2) / np.mean(g64 ** 2))
    rel_c0 = abs(c32 - c64) / abs(c64)
    rng = np.random.default_rng(7)
    eps = 1e-4
    worst = 0.0
    for _ in range(8):
        d = rng.normal(size=w.v.shape)
        fd = (_rollout(w, FP64, nsteps, nsteps, dt).forward(w.v + eps * d, c0)
              - _rollout(w, FP64, nsteps, nsteps, dt).forward(w.v - eps * d, c0)) / (2 * eps)
        worst = max(worst, abs(fd - float((g32 * d).sum())) / abs(fd))
    print(f"FP32 adjoint vs FP64 adjoint: max-norm {rel_max:.3e}, RMS {rel_rms:.3e}, c0 {rel_c0:.3e}; "
          f"vs central differences along 8 directions: worst {worst:.3e}", flush=True)
    assert rel_max < 5e-2 and rel_rms < 1e-2 and rel_c0 < 1e-2 and worst < 1e-2


@pytest.mark.parametrize("layout", ["random", "slab"])
def test_two_set_adjoint_matches_reverse_mode_on_the_union(layout):
    """Two sets stepping as two GPUs' shares (local-local and local-remote
    passes, steps e and f), FP64: the hand adjoint of the two-set rollout,
    including the reverse of both local-remote passes, equals the reverse-mode
    gradient of one dense rollout over the union of the sets."""
    from paper_2310_03596_amd.adjoint import TwoSetKineticEnergyRollout
    w = small_box(n_side=7, seed=84)
    owner = (np.random.default_rng(85).random(w.n) < 0.5) if layout == "random" else w.x[:, 0] > np.median(w.x[:, 0])
    dt, nsteps = 1.4e-5, 4
    print(f"[two-set adjoint] n={w.n} layout={layout} set B={int(owner.sum())}", flush=True)
    J_ref, gv_ref, gc_ref = torch_ref.gradient(w, w.params["c0"], dt, nsteps)
    ro = TwoSetKineticEnergyRollout(w, owner, FP64, nsteps, 2, dt)
    J = ro.forward(w.v, w.params["c0"])
    nb = ro.ts.nb.cpu().numpy()
    assert nb.min() > 0            # both local-remote passes had targets
    gv, gc = ro.backward(1.0)
    assert J == pytest.approx(J_ref, rel=1e-13)
    assert np.abs(gv - gv_ref).max() <= 1e-9 * np.abs(gv_ref).max()
    assert gc == pytest.approx(gc_ref, rel=1e-9)


def test_interact_adjoint_splits_into_its_two_cotangents():
    """The local-remote reverse with both cotangents equals the sum of the
    call with the targets' cotangent alone and the call with the sources'
    alone (the form a GPU uses when the remote rates are not differentiated,
    and the one that gives the received particles' cotangent)."""
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.adjoint import Cotangent
    from paper_2310_03596_amd.sim import SharePass
    from paper_2310_03596_amd.state import Rates, cells_struct, stream_handle
    loc, rem = S.c4_share("mixed", seed=86, nx=24, ny=12, nz=12, split_ix=18)
    sp = SharePass(loc, rem, FP64)
    sp.build()
    sp.mark()
    rng = np.random.default_rng(87)
    rl, rr = Rates(sp.nl, FP64, False, "cuda"), Rates(sp.nr, FP64, False, "cuda")
    rl.hi.copy_(torch.from_numpy(rng.normal(size=(6, sp.nl))))
    rr.hi.copy_(torch.from_numpy(rng.normal(size=(6, sp.nr))))
    ws_bytes = L.sph_workspace_size(sp.grid, max(sp.nl, sp.nr), FP64, L.SPH_SOLID_J2)
    ws = torch.zeros(ws_bytes, dtype=torch.uint8, device="cuda")
    st = stream_handle()
    outs = []
    for rt, rs in ((rl, rr), (rl, None), (None, rr)):
        b = Cotangent(sp.nl, FP64, "cuda")
        L.sph_interact_adjoint(sp.params, sp.grid, L.SPH_PASS_FORCE, sp.LB.struct(), sp.bidx.data_ptr(), sp.nb.data_ptr(),
                               sp.RB.struct(), cells_struct(sp.rstart, sp.nc), None if rt is None else rt.struct(),
                               None if rs is None else rs.struct(), b.struct(), ws.data_ptr(), ws_bytes, st)
        torch.cuda.synchronize()
        outs.append(torch.cat([b.x, b.v, b.w[None], b.rho[None], b.p[None], b.c[None], b.e[None]]).cpu().numpy())
    both, only_t, only_s = outs
    scale = np.abs(both).max(axis=1, keepdims=True) + 1e-300
    assert np.abs(both - (only_t + only_s)).max(axis=1, keepdims=True).max() <= (1e-12 * scale).max()
    assert np.abs(only_t).max() > 0 and np.abs(only_s).max() > 0
    # targets off the boundary list have no remote pairs: nothing accumulated there
    nb = int(sp.nb.cpu()[0])
    off = np.setdiff1d(np.arange(sp.nl), sp.bidx.cpu().numpy()[:nb])
    assert not np.abs(both[:, off]).any()


def solid_block(seed, s_axial=0.0, rate=0.0, n_side=5):
    """A free J2 block of the cylinder's metal (linear EOS, H = E / 100); with
    s_axial near Y0 and a stretch it yields within a step."""
    w = S.solid_block(n_side, seed=seed, vz=0.0, s_sigma=2e7, s_axial=s_axial, stretch_rate=rate)
    w.params = dict(w.params, wall_mask=0)
    return w


@pytest.mark.parametrize("plastic", [False, True], ids=["elastic", "plastic"])
def test_solid_adjoint_matches_reverse_mode(plastic):
    """Solid steps (GRADIENT pass, stress stage, FORCE pass, update), FP64:
    dJ/dv0 and dJ/dS0 of the final kinetic energy against the dense
    reverse-mode reference."""
    from paper_2310_03596_amd.adjoint import SolidKineticEnergyRollout
    w = solid_block(95 + int(plastic), 270e6 if plastic else 0.0, 2e4 if plastic else 0.0)
    dt, nsteps = 2e-8, 4
    print(f"[solid adjoint vs reverse mode] n={w.n} plastic={plastic}", flush=True)
    J_ref, gv_ref, gS_ref = torch_ref.solid_gradient(w, dt, nsteps)
    ro = SolidKineticEnergyRollout(w, FP64, nsteps, 2, dt)
    J = ro.forward(w.v)
    gv, gS = ro.backward(1.0)
    ev = np.abs(gv - gv_ref).max() / np.abs(gv_ref).max()
    eS = np.abs(gS - gS_ref).max() / np.abs(gS_ref).max()
    print(f"max-norm error: dJ/dv0 {ev:.3e}, dJ/dS0 {eS:.3e}", flush=True)
    assert J == pytest.approx(J_ref, rel=1e-12)
    assert ev <= 1e-9 and eS <= 1e-9


def test_solid_adjoint_matches_central_differences():
    """A 12^3 block that yields during the run, 10 steps with checkpoints every
    4, FP64: directional derivatives along random directions in v0 and S0
    against central differences; FP32-split gradient reported against FP64.
    A central difference resolves the derivative no finer than one rounding
    unit of J over |J(+) - J(-)|: the S0 step (1e3 Pa, 4e-6 of the deviator's
    size) keeps that floor near 1e-7 of the derivative for these directions,
    and the bound adds 4 rounding units of J to the 1e-6 relative one."""
    from paper_2310_03596_amd.adjoint import SolidKineticEnergyRollout
    w = solid_block(97, 270e6, 2e4, n_side=12)
    dt, nsteps = 2e-8, 10
    print(f"[solid adjoint vs FD] n={w.n} steps={nsteps}", flush=True)
    ro = SolidKineticEnergyRollout(w, FP64, nsteps, 4, dt)
    ro.forward(w.v)
    gv, gS = ro.backward(1.0)
    assert (ro.final.ep.cpu().numpy() > 0).mean() > 0.5

    def J(v, Sx):
        return SolidKineticEnergyRollout(w, FP64, nsteps, nsteps, dt).forward(v, Sx)

    rng = np.random.default_rng(98)
    worst = 0.0
    for k in range(6):
        d = rng.normal(size=w.v.shape)
        jp, jm = J(w.v + 1e-4 * d, w.S), J(w.v - 1e-4 * d, w.S)
        fd = (jp - jm) / 2e-4
        rel = abs(fd - float((gv * d).sum())) / abs(fd)
        floor = 4 * np.spacing(max(abs(jp), abs(jm))) / abs(jp - jm)
        dS = rng.normal(size=w.S.shape)
        jp, jm = J(w.v, w.S + 1e3 * dS), J(w.v, w.S - 1e3 * dS)
        fdS = (jp - jm) / 2e3
        relS = abs(fdS - float((gS * dS).sum())) / abs(fdS)
        floorS = 4 * np.spacing(max(abs(jp), abs(jm))) / abs(jp - jm)
        worst = max(worst, rel, relS)
        print(f"direction {k}: v0 rel {rel:.2e} (floor {floor:.1e}), S0 rel {relS:.2e} (floor {floorS:.1e})",
              flush=True)
        assert rel <= 1e-6 + floor and relS <= 1e-6 + floorS, (k, rel, relS)
    print(f"worst relative difference {worst:.3e}", flush=True)
    ro32 = SolidKineticEnergyRollout(w, FP32, nsteps, 4, dt)
    ro32.forward(w.v)
    g32, gS32 = ro32.backward(1.0)
    print(f"FP32-split solid adjoint vs FP64: dJ/dv0 {np.abs(g32 - gv).max() / np.abs(gv).max():.3e}, "
          f"dJ/dS0 {np.abs(gS32 - gS).max() / np.abs(gS).max():.3e}", flush=True)
    assert np.abs(g32 - gv).max() <= 1e-2 * np.abs(gv).max()
