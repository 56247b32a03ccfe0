"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances
  * Integer outputs (hash, permutation, bucket table, ids, communication
    hash, boundary list and count): bit-exact.
  * Pair sums are compared against B, the per-target sum of the oracle's
    magnitude bound of each term (every input in absolute value, every
    difference as a sum, |n_k| -> 1: forward error analysis bounds the
    rounding of a ~30-operation term by ~30 u B, and a relative perturbation
    of positions or velocities by the same fraction of B), and B_peak, the
    same sum with every pair at the kernel's peak strength F_max / F (near the
    support edge F ~ (2 - q)^2, so a one-ulp change of q is a large relative
    change of a vanishing term but a tiny one of the term at full strength).
  * FP64 form: |gpu - oracle| <= 1e-13 B + 1e-14 B_peak (u = 1.1e-16; FMA
    contraction on one side only).
  * FP32-split form on the same (float-rounded) inputs: |gpu - oracle| <=
    2e-5 B + 2e-6 B_peak (u = 6e-8 over ~30 operations is ~2e-6 B; positions
    enter through float offsets, a relative error ~2e-7 of the bucket side,
    so q moves by ~2e-7 and F by at most ~6e-7 F_max; a pair within that of
    r = 2h may be counted on one side only; the compensated sum adds one
    rounding of the result).
  * One whole step: FP64 form within 1e-12 of the oracle per field (max
    norm relative to the field's max); FP32-split form within 2e-5.
"""
import numpy as np
import pytest
import torch

import sph_synth as S
from oracle import cpu
from tests import brute
from tests.gpu_helpers import (assert_within, dense_cell_cloud, field_errors, oracle_state, pressure_scale,
                               rate_bound)

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
PRECS = [pytest.param(FP64, id="fp64"), pytest.param(FP32, id="fp32split")]
TOL_STEP = {FP64: 1e-12, FP32: 2e-5}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_03596_amd import _lib
    _lib.load()


def _sim(wl, prec, **kw):
    from paper_2310_03596_amd.sim import Sim
    return Sim(wl, prec, **kw)


def _clamped_cloud():
    w = S.random_cloud(700, seed=51, h=0.05)
    w.x[:40] -= 0.3            # outside the grid on the low side
    w.x[40:80] += 0.3          # and on the high side
    return w


def _faces():
    w = S.random_cloud(400, seed=52, h=0.05, box=0.5)
    L = w.grid["cell"]
    w.x[:, 0] = (np.arange(w.n) % 4) * L
    w.x[1::3, 1] = np.nextafter(w.x[1::3, 0], np.inf)
    w.x[2::3, 1] = np.nextafter(w.x[2::3, 0], -np.inf)
    w.x = np.clip(w.x, 0.0, None)
    return w


def _coincident():
    """A fifth of the particles sit exactly on another one (different velocity
    and density): such a pair has no direction and, with F(0) = 0, adds
    nothing; the pair body must produce exact zeros there, not NaN."""
    w = S.random_cloud(1200, seed=56, h=0.05, rho_sigma=0.01)
    rng = np.random.default_rng(58)
    src = rng.choice(w.n, size=240, replace=False)
    dst = rng.choice(np.setdiff1d(np.arange(w.n), src), size=240, replace=False)
    w.x[dst] = w.x[src]
    return w


def _far_origin():
    """A lattice 2 km from the coordinate origin (the grid moves with it): the
    FP64 form's filter works on FP64 differences rounded to float, with a
    margin that grows with the frame's distance from the origin."""
    w = S.jittered_lattice(10, seed=57, rho_sigma=0.01)
    shift = np.array([1000.0, -2000.0, 500.0])
    w.x = w.x + shift
    g = dict(w.grid)
    g["origin"] = [float(o + d) for o, d in zip(g["origin"], shift)]
    w.grid = g
    return w


def _exact_edge():
    """Pairs exactly at r = 2h and r = h: h = 1/16 and a lattice of spacing
    1/8 = 2h (with a second lattice shifted by h along x), so every
    difference, offset and squared distance is exact in both forms and the
    strict predicate r^2 < (2h)^2 leaves the pairs at r = 2h out."""
    h = 0.0625
    w = S.random_cloud(2 * 6 ** 3, seed=59, h=h, box=0.75, rho_sigma=0.01)
    g = np.arange(6) * (2 * h) + 2 * h
    a = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    b = a + np.array([h, 0.0, 0.0])
    w.x = np.concatenate([a, b])
    return w


CASES = {
    "one": lambda: S.random_cloud(1, seed=50, h=0.05),
    "cloud2049": lambda: S.random_cloud(2049, seed=53, h=0.04, rho_sigma=0.01),
    "cube8000": lambda: S.c1_cube(),
    "faces": _faces,
    "clamped": _clamped_cloud,
    "dense": lambda: dense_cell_cloud(1500, seed=54),
    "lattice12": lambda: S.jittered_lattice(12, seed=55, rho_sigma=0.01),
    "far_origin": _far_origin,
    "coincident": _coincident,
    "exact_edge": _exact_edge,
}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(CASES))
def test_build_cells_bit_exact(case, prec):
    wl = CASES[case]()
    print(f"[build_cells] case={case} prec={prec} n={wl.n}", flush=True)
    sim = _sim(wl, prec)
    sim.build()
    torch.cuda.synchronize()
    h = sim.A.host()
    s = cpu.State.from_workload(wl)
    o, operm, ostart = cpu.build_cells(wl.grid, s)
    assert np.array_equal(sim.perm.cpu().numpy().view(np.uint32), operm)
    assert np.array_equal(h["hash"], o.hash)
    assert np.array_equal(h["id"], o.id)
    assert np.array_equal(sim.start.cpu().numpy().view(np.uint32), ostart)
    assert np.array_equal(h["x"], o.x)
    assert np.array_equal(h["E"], o.E)
    if prec == FP64:
        assert np.array_equal(h["v"], o.v) and np.array_equal(h["m"], o.m)
    else:
        assert np.array_equal(h["v"], o.v.astype(np.float32).astype(np.float64))
        # offsets from the bucket corner, rounded once to float
        n = np.asarray(wl.grid["dims"])
        c = np.stack([o.hash % n[0], (o.hash // n[0]) % n[1], o.hash // (n[0] * n[1])], axis=1)
        ref = (o.x - np.asarray(wl.grid["origin"])) - c * wl.grid["cell"]
        assert np.array_equal(h["off"], ref.astype(np.float32).astype(np.float64))


def _sparse(n, seed, clumps=False):
    """n particles in the unit box with h = 0.003: a grid of 4.6 million
    buckets, almost all empty.  Placed at random, the empty runs between
    occupied buckets are thousands long (with 800 particles more of them
    exceed 4096 buckets than the bucket table's list of long runs holds, so
    its workgroup fallback runs too); in two clumps at opposite corners, one
    run spans almost the whole grid."""
    w = S.random_cloud(n, seed=seed, h=0.003, rho_sigma=0.01)
    if clumps:
        half = n // 2
        w.x[:half] *= 0.05
        w.x[half:] = 0.95 + 0.05 * w.x[half:]
    return w


SPARSE = {
    "sparse800": lambda: _sparse(800, 60),
    "sparse3000": lambda: _sparse(3000, 61),
    "clumps": lambda: _sparse(1000, 62, clumps=True),
}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(SPARSE))
def test_bucket_table_long_empty_runs(case, prec):
    wl = SPARSE[case]()
    nc = int(np.prod(wl.grid["dims"]))
    print(f"[build_cells sparse] case={case} prec={prec} n={wl.n} buckets={nc}", flush=True)
    sim = _sim(wl, prec)
    sim.start.fill_(-1)   # every entry must be written
    sim.build()
    torch.cuda.synchronize()
    h = sim.A.host()
    s = cpu.State.from_workload(wl)
    o, operm, ostart = cpu.build_cells(wl.grid, s)
    assert np.array_equal(sim.perm.cpu().numpy().view(np.uint32), operm)
    assert np.array_equal(h["hash"], o.hash)
    assert np.array_equal(sim.start.cpu().numpy().view(np.uint32), ostart)
    runs = np.diff(np.concatenate([[-1], np.unique(o.hash), [nc]])) - 1
    print(f"  empty runs over 4096 buckets: {(runs > 4096).sum()}, longest {runs.max()}", flush=True)


@pytest.mark.parametrize("prec", PRECS)
def test_bucket_table_of_no_particles(prec):
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.state import Particles, cells_struct, grid_struct, ncells, stream_handle
    wl = S.random_cloud(10, seed=63, h=0.01)
    nc = ncells(wl.grid)
    a, b = Particles(0, prec, False), Particles(0, prec, False)
    start = torch.full((nc + 1,), 7, dtype=torch.int32, device="cuda")
    gs = grid_struct(wl.grid)
    wsb = L.sph_workspace_size(gs, 0, prec, L.SPH_FLUID_TAIT)
    ws = torch.zeros(max(wsb, 1), dtype=torch.uint8, device="cuda")
    rc = L.sph_build_cells(gs, a.struct(), b.struct(), None, cells_struct(start, nc), ws.data_ptr(), wsb,
                           stream_handle())
    assert rc == 0
    torch.cuda.synchronize()
    assert int(start.abs().sum()) == 0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(CASES))
def test_force_pass_matches_oracle(case, prec):
    wl = CASES[case]()
    print(f"[force] case={case} prec={prec} n={wl.n}", flush=True)
    sim = _sim(wl, prec)
    sim.build()
    sim.interact()
    torch.cuda.synchronize()
    h = sim.A.host()
    st = oracle_state(h, False)
    start = cpu.cell_start(st.hash, cpu.ncells(wl.grid))
    assert np.array_equal(sim.start.cpu().numpy().view(np.uint32), start)
    ref = cpu.interact(wl.params, wl.grid, cpu.FORCE, st, st, start, True)
    bound = rate_bound(wl.params, wl.grid, cpu.FORCE, st, st, start, True, prec)
    got = sim.rates.force().T.cpu().numpy()
    assert_within(got, ref, bound, f"{case} rates")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["cloud2049", "dense"])
def test_force_pass_continues_its_sums(case, prec):
    """zero_first = 0 on a pass over every target (the FP64 form's
    matrix-filter kernel, the FP32 form's VALU filter): the second pass adds
    its terms to the sums the first left, so the rates are twice the
    oracle's, within twice the one-pass bound."""
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.state import stream_handle
    wl = CASES[case]()
    print(f"[force continue] case={case} prec={prec} n={wl.n}", flush=True)
    sim = _sim(wl, prec)
    sim.build()
    sim.interact()
    a = sim.A.struct()
    L.sph_interact(sim.params, sim.grid, L.SPH_PASS_FORCE, a, None, None, a, sim.cells, 0, sim.rates.struct(),
                   sim.ws.data_ptr(), sim.ws_bytes, stream_handle())
    torch.cuda.synchronize()
    st = oracle_state(sim.A.host(), False)
    start = cpu.cell_start(st.hash, cpu.ncells(wl.grid))
    ref = cpu.interact(wl.params, wl.grid, cpu.FORCE, st, st, start, True)
    bound = rate_bound(wl.params, wl.grid, cpu.FORCE, st, st, start, True, prec)
    assert_within(sim.rates.force().T.cpu().numpy(), 2.0 * ref, 2.0 * bound, f"{case} rates after two passes")


@pytest.mark.parametrize("prec", PRECS)
def test_force_pass_conserves(prec):
    wl = S.jittered_lattice(14, seed=56, jitter=0.3, rho_sigma=0.02, v_sigma=1.0)
    sim = _sim(wl, prec)
    sim.build()
    sim.interact()
    torch.cuda.synchronize()
    got = sim.rates.force().T.cpu().numpy()
    st = oracle_state(sim.A.host(), False)
    start = cpu.cell_start(st.hash, cpu.ncells(wl.grid))
    scale = cpu.interact_abs(wl.params, wl.grid, cpu.FORCE, st, st, start, True).sum(0)
    tot = got.sum(0)
    lim = 1e-12 if prec == FP64 else 2e-6
    for k in range(5):
        assert abs(tot[k]) <= lim * scale[k], (k, tot[k], scale[k])


@pytest.mark.parametrize("prec", PRECS)
def test_gradient_pass_matches_oracle(prec):
    wl = S.solid_block(8, seed=57, s_sigma=1e7)
    sim = _sim(wl, prec)
    sim.build()
    sim.interact(pass_=1)
    torch.cuda.synchronize()
    st = oracle_state(sim.A.host(), True)
    start = cpu.cell_start(st.hash, cpu.ncells(wl.grid))
    ref = cpu.interact(wl.params, wl.grid, cpu.GRADIENT, st, st, start, True)
    bound = rate_bound(wl.params, wl.grid, cpu.GRADIENT, st, st, start, True, prec)
    got = sim.rates.grad().T.cpu().numpy()
    assert_within(got, ref, bound, "velocity gradient")


@pytest.mark.parametrize("prec", PRECS)
def test_solid_force_pass_matches_oracle(prec):
    wl = S.solid_block(8, seed=58, s_sigma=1e8)
    sim = _sim(wl, prec)
    sim.build()
    sim.interact()
    torch.cuda.synchronize()
    st = oracle_state(sim.A.host(), True)
    start = cpu.cell_start(st.hash, cpu.ncells(wl.grid))
    ref = cpu.interact(wl.params, wl.grid, cpu.FORCE, st, st, start, True)
    bound = rate_bound(wl.params, wl.grid, cpu.FORCE, st, st, start, True, prec)
    got = sim.rates.force().T.cpu().numpy()
    assert_within(got, ref, bound, "solid rates")


def _step_vs_oracle(wl, prec, nsteps, tol):
    """Run nsteps on the GPU; before each, run the oracle one step from the
    GPU's own state with the GPU's dt and compare in array order."""
    sim = _sim(wl, prec)
    solid = wl.S is not None
    worst = {}
    for k in range(nsteps):
        torch.cuda.synchronize()
        h0 = sim.A.host()
        dt = float(sim.diag[sim.cur, 0].cpu()) if sim.fixed is None else float(sim.fixed.cpu())
        st = oracle_state(h0, solid)
        dts, odiag = cpu.run(wl.params, wl.grid, st, 1, dts_in=np.array([dt]))
        sim.step()
        torch.cuda.synchronize()
        h1 = sim.A.host()
        assert np.array_equal(h1["id"], st.id), f"step {k}: permutation differs"
        fields = ("x", "v", "m", "w", "rho", "p", "c", "E") + (("S", "ep") if solid else ())
        sc = {"p": np.abs(st.p).max() + pressure_scale(wl.params)}
        if solid:
            sc["S"] = np.abs(st.S).max() + wl.params["G"] * 1e-3
            sc["ep"] = max(np.abs(st.ep).max(), 1e-6)
        err = field_errors(h1, st, fields, sc)
        for f, e in err.items():
            worst[f] = max(worst.get(f, 0.0), e)
            assert e <= tol, f"step {k} field {f}: rel err {e:.3e} > {tol}"
        gd = sim.diagnostics()
        assert gd[0] == pytest.approx(odiag[0], rel=tol * 10)
    return worst


@pytest.mark.parametrize("prec", PRECS)
def test_cube_steps_match_oracle_each_step(prec):
    worst = _step_vs_oracle(S.c1_cube(), prec, 10, TOL_STEP[prec])
    print("worst per-field error over 10 steps:", worst)


@pytest.mark.parametrize("prec", PRECS)
def test_solid_steps_match_oracle_each_step(prec):
    wl = S.solid_block(8, seed=59)
    worst = _step_vs_oracle(wl, prec, 3, TOL_STEP[prec])
    print("solid worst per-field error:", worst)


@pytest.mark.parametrize("prec", PRECS)
def test_solid_block_yields_with_hardening(prec):
    """A block at 0.9 of the yield stress under an isochoric stretch that
    raises its deviator by about 100 MPa a step: the interior goes plastic in
    the first step, so the radial return with linear hardening (the
    cylinder's H = E / 100) decides S and the plastic strain at every step."""
    wl = S.solid_block(8, seed=62, vz=0.0, s_sigma=1e6, s_axial=270e6, stretch_rate=2e4)
    assert wl.params["H"] == pytest.approx(70e9 / 100)
    worst = _step_vs_oracle(wl, prec, 3, TOL_STEP[prec])
    print("yielding block worst per-field error:", worst)
    # the same three steps went plastic (inside at the first step, the
    # surface, where the stretch is resolved only in part, soon after)
    sim = _sim(wl, prec)
    sim.run(3)
    torch.cuda.synchronize()
    ep = sim.A.host()["ep"]
    assert (ep > 0).mean() > 0.5 and ep.max() > 1e-3, ((ep > 0).mean(), ep.max())


@pytest.mark.parametrize("prec", PRECS)
def test_gravity_walls_step(prec):
    wl = S.c2_column(nx=10, ny=8, nz=20, dx=5.4e-3, box=(0.1, 0.05, 0.12))
    _step_vs_oracle(wl, prec, 4, TOL_STEP[prec])


def test_steps_are_deterministic():
    outs = []
    for _ in range(2):
        sim = _sim(S.c1_cube(), FP32)
        for _k in range(5):
            sim.step()
        torch.cuda.synchronize()
        outs.append(sim.A.host())
    for f in outs[0]:
        assert np.array_equal(outs[0][f], outs[1][f]), f


@pytest.mark.parametrize("layout", ["slab", "mixed"])
@pytest.mark.parametrize("prec", PRECS)
def test_share_pass_matches_oracle(layout, prec):
    from paper_2310_03596_amd.sim import SharePass
    loc, rem = S.c4_share(layout, seed=60, nx=40, ny=18, nz=16, split_ix=30)
    print(f"[share] layout={layout} prec={prec} local={loc.n} remote={rem.n}", flush=True)
    sp = SharePass(loc, rem, prec)
    sp.run()
    torch.cuda.synchronize()
    hl, hr = sp.LB.host(), sp.RB.host()
    nb = int(sp.nb.cpu()[0])
    sl, sr = oracle_state(hl, False), oracle_state(hr, False)
    lstart = cpu.cell_start(sl.hash, cpu.ncells(loc.grid))
    rstart = cpu.cell_start(sr.hash, cpu.ncells(loc.grid))
    assert np.array_equal(sp.rstart.cpu().numpy().view(np.uint32), rstart)
    comm, bidx = cpu.mark_boundary(loc.grid, sl.hash, rstart)
    assert nb == bidx.size
    assert np.array_equal(sp.comm.cpu().numpy().view(np.uint32), comm)
    assert np.array_equal(sp.bidx.cpu().numpy().view(np.uint32)[:nb], bidx)
    flags = brute.boundary_flags(loc.grid, sl.x, sr.x)
    assert np.array_equal(np.flatnonzero(flags), bidx)
    # packed payload = boundary particles, bit for bit
    hp = sp.payload.host()
    for f in ("x", "v", "m", "w", "rho", "p", "c", "E", "id", "hash"):
        assert np.array_equal(hp[f][:nb], hl[f][bidx]), f
    # LL then LR accumulate the same sums as the oracle's two passes
    ref = cpu.interact(loc.params, loc.grid, cpu.FORCE, sl, sl, lstart, True)
    ref = cpu.interact(loc.params, loc.grid, cpu.FORCE, sl, sr, rstart, False, rates=ref, tidx=bidx)
    bound = rate_bound(loc.params, loc.grid, cpu.FORCE, sl, sl, lstart, True, prec)
    bound += rate_bound(loc.params, loc.grid, cpu.FORCE, sl, sr, rstart, False, prec)
    got = sp.rates.force().T.cpu().numpy()
    assert_within(got, ref, bound, f"share {layout}")
    # the decomposition loses no pair: LL + LR equal one pass over the union of
    # the two arrays (Section II, steps e and f), matched by particle id
    u = cpu.State(sl.n + sr.n)
    for f in ("x", "v", "m", "w", "rho", "p", "c", "E", "id"):
        getattr(u, f)[...] = np.concatenate([getattr(sl, f), getattr(sr, f)])
    us, _, ustart = cpu.build_cells(loc.grid, u)
    uref = cpu.interact(loc.params, loc.grid, cpu.FORCE, us, us, ustart, True)
    ubound = rate_bound(loc.params, loc.grid, cpu.FORCE, us, us, ustart, True, prec)
    row = {int(i): k for k, i in enumerate(us.id)}
    sel = np.array([row[int(i)] for i in sl.id])
    assert_within(got, uref[sel], ubound[sel], f"share {layout} vs union")
    # particles with no remote bucket nearby have no remote neighbour
    pi, pj = cpu.neighbors(loc.params, loc.grid, sl, sr, rstart, False)
    assert set(np.unique(pi).tolist()) <= set(bidx.tolist())


def test_boundary_capacity_overflow_reports_true_count():
    """A boundary list shorter than the flagged set: the list holds the first
    cap indices, the count its consumers read is cap, and the flagged count
    is the true one; packing and a local-remote pass from the short list
    read only its entries."""
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.sim import SharePass
    from paper_2310_03596_amd.state import cells_struct, stream_handle
    loc, rem = S.c4_share("mixed", seed=61, nx=30, ny=12, nz=12, split_ix=24)
    sp = SharePass(loc, rem, FP32)
    sp.build()
    cap = 17
    sentinel = torch.full((sp.nl,), -7, dtype=torch.int32, device="cuda")
    nflag = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.sph_mark_boundary(sp.grid, sp.LB.struct(), cells_struct(sp.rstart, sp.nc), sp.comm.data_ptr(),
                        sentinel.data_ptr(), cap, sp.nb.data_ptr(), nflag.data_ptr(), sp.ws.data_ptr(), sp.ws_bytes,
                        stream_handle())
    torch.cuda.synchronize()
    comm = sp.comm.cpu().numpy().view(np.uint32)
    flagged = np.flatnonzero(comm != cpu.ncells(loc.grid))
    assert int(nflag.cpu()[0]) == flagged.size > cap
    assert int(sp.nb.cpu()[0]) == cap
    got = sentinel.cpu().numpy()
    assert np.all(got[cap:] == -7)
    assert np.array_equal(got[:cap], flagged[:cap])
    # consumers of the short list: a list of exactly cap entries (the rest of
    # the buffer poisoned with indices past the array) packs and interacts
    # like the first cap flagged particles
    short = torch.full((sp.nl,), -1, dtype=torch.int32, device="cuda")   # 0xFFFFFFFF: no particle
    short[:cap] = sentinel[:cap]
    sp.bidx.copy_(short)
    sp.pack()
    torch.cuda.synchronize()
    pay = sp.payload.host()
    hl = sp.LB.host()
    assert np.array_equal(pay["id"][:cap], hl["id"][flagged[:cap]])
    _, _, c_short, k_short = sp.census()
    listed = flagged[:cap]
    rest = np.setdiff1d(np.arange(sp.nl), listed)
    assert not c_short[rest].any() and not k_short[rest].any()
    sp.mark()    # the whole list (capacity: every local particle)
    _, _, c_full, k_full = sp.census()
    assert c_full[listed].sum() > 0
    assert np.array_equal(c_short[listed], c_full[listed]) and np.array_equal(k_short[listed], k_full[listed])
