"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments on the host before anything
is enqueued (no compute call runs here)."""
import ctypes as C
import os
import re

import pytest

from paper_2310_03596_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")

FAKE = 0x1000   # never dereferenced: every call below fails validation first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("sph_build_cells", "sph_mark_boundary", "sph_interact", "sph_integrate",
                 "sph_interact_adjoint"):
        assert must in names
    assert set(names) == set(L.EXPORTS)


def test_binding_wraps_every_export():
    # sph_last_error is read by the wrappers themselves: a failed call raises
    # SphError with its message
    for name in L.EXPORTS:
        if name != "sph_last_error":
            assert callable(getattr(L, name, None)), name


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert "gfx950" in L.sph_version()


def _grid(dims=(4, 4, 4), cell=1.0):
    g = L.SphGrid()
    for d in range(3):
        g.origin[d] = 0.0
        g.dims[d] = dims[d]
    g.cell = cell
    return g


def _params(h=0.5, prec=L.SPH_FP64):
    p = L.SphParams()
    p.h, p.rho0, p.c0, p.gamma, p.cfl, p.beta = h, 1000.0, 50.0, 7.0, 0.3, 1.0
    p.prec = prec
    return p


def _particles(n, prec=L.SPH_FP64, full=True):
    s = L.SphParticles()
    s.n, s.prec = n, prec
    if full:
        for d in range(3):
            s.x[d] = s.v[d] = s.off[d] = FAKE
        for f in ("hash", "id", "m", "omega", "rho", "p", "c", "e", "E"):
            setattr(s, f, FAKE)
    return s


def _last():
    return L.load().sph_last_error().decode()


def test_workspace_size_grows_with_n():
    g = _grid()
    a, b = L.sph_workspace_size(g, 1000, 0, 0), L.sph_workspace_size(g, 100000, 0, 0)
    assert 0 < a < b
    assert L.sph_workspace_size(g, 0, 0, 0) > 0
    # FP64 and solid records are larger
    assert L.sph_workspace_size(g, 1000, 1, 0) < a < L.sph_workspace_size(g, 1000, 0, 1)


def test_build_cells_rejects_bad_arguments():
    lib = L.load()
    g = _grid()
    cells = L.SphCells(FAKE, 64, 0)
    a, b = _particles(10), _particles(10)
    b.x[0] = 0x2000
    ws = L.sph_workspace_size(g, 10, 0, 0)
    # grid too large for 32-bit hashes
    big = _grid(dims=(1 << 11, 1 << 11, 1 << 10))
    assert lib.sph_build_cells(C.byref(big), C.byref(a), C.byref(b), FAKE, cells, FAKE, ws, None) == L.SPH_ERR_ARG
    assert "2^32" in _last()
    # bucket count mismatch
    bad = L.SphCells(FAKE, 63, 0)
    assert lib.sph_build_cells(C.byref(g), C.byref(a), C.byref(b), FAKE, bad, FAKE, ws, None) == L.SPH_ERR_ARG
    # missing field
    c = _particles(10)
    c.rho = None
    assert lib.sph_build_cells(C.byref(g), C.byref(c), C.byref(b), FAKE, cells, FAKE, ws, None) == L.SPH_ERR_ARG
    assert "required field" in _last()
    # in/out overlap
    assert lib.sph_build_cells(C.byref(g), C.byref(a), C.byref(a), FAKE, cells, FAKE, ws, None) == L.SPH_ERR_ARG
    # workspace too small
    assert (lib.sph_build_cells(C.byref(g), C.byref(a), C.byref(b), FAKE, cells, FAKE, 64, None)
            == L.SPH_ERR_WORKSPACE)
    assert lib.sph_build_cells(C.byref(g), C.byref(a), C.byref(b), FAKE, cells, None, ws, None) == L.SPH_ERR_WORKSPACE
    # n mismatch
    d = _particles(11)
    assert lib.sph_build_cells(C.byref(g), C.byref(a), C.byref(d), FAKE, cells, FAKE, ws, None) == L.SPH_ERR_ARG
    # zero-size bucket
    z = _grid(cell=0.0)
    assert lib.sph_build_cells(C.byref(z), C.byref(a), C.byref(b), FAKE, cells, FAKE, ws, None) == L.SPH_ERR_ARG


def test_interact_rejects_bad_arguments():
    lib = L.load()
    g = _grid()
    cells = L.SphCells(FAKE, 64, 0)
    p = _particles(10)
    r = L.SphRates()
    for k in range(6):
        r.hi[k] = FAKE
    # bucket smaller than the support 2h
    assert lib.sph_interact(C.byref(_params(h=0.6)), C.byref(g), 0, C.byref(p), None, None, C.byref(p), cells, 1,
                            C.byref(r), FAKE, 1 << 30, None) == L.SPH_ERR_ARG
    assert "smaller than the support" in _last()
    # precision mismatch
    assert lib.sph_interact(C.byref(_params(prec=L.SPH_FP32_SPLIT)), C.byref(g), 0, C.byref(p), None, None,
                            C.byref(p), cells, 1, C.byref(r), FAKE, 1 << 30, None) == L.SPH_ERR_ARG
    # FP32 split needs the compensation buffers and offsets
    q = _particles(10, L.SPH_FP32_SPLIT)
    assert lib.sph_interact(C.byref(_params(prec=L.SPH_FP32_SPLIT)), C.byref(g), 0, C.byref(q), None, None,
                            C.byref(q), cells, 1, C.byref(r), FAKE, 1 << 30, None) == L.SPH_ERR_ARG
    assert "lo" in _last()
    # target list without a device count
    assert lib.sph_interact(C.byref(_params()), C.byref(g), 0, C.byref(p), FAKE, None, C.byref(p), cells, 0,
                            C.byref(r), FAKE, 1 << 30, None) == L.SPH_ERR_ARG
    # unknown pass
    assert lib.sph_interact(C.byref(_params()), C.byref(g), 7, C.byref(p), None, None, C.byref(p), cells, 1,
                            C.byref(r), FAKE, 1 << 30, None) == L.SPH_ERR_ARG
    # solid FORCE pass needs the stress fields
    ps = _params()
    ps.material, ps.K, ps.G = L.SPH_SOLID_J2, 1e9, 1e9
    assert lib.sph_interact(C.byref(ps), C.byref(g), 0, C.byref(p), None, None, C.byref(p), cells, 1, C.byref(r),
                            FAKE, 1 << 30, None) == L.SPH_ERR_ARG
    assert "S[0]" in _last()
    # pair records are addressed with 32-bit byte offsets: fewer than 2^27 sources, in both forms
    for prec in (L.SPH_FP64, L.SPH_FP32_SPLIT):
        t, big = _particles(10, prec), _particles(1 << 27, prec)
        if prec == L.SPH_FP32_SPLIT:
            for k in range(6):
                r.lo[k] = FAKE
        assert lib.sph_interact(C.byref(_params(prec=prec)), C.byref(g), 0, C.byref(t), None, None, C.byref(big),
                                cells, 1, C.byref(r), FAKE, 1 << 62, None) == L.SPH_ERR_ARG
        assert "must be below 134217728" in _last()


def test_neighbor_census_rejects_bad_arguments():
    lib = L.load()
    g = _grid()
    cells = L.SphCells(FAKE, 64, 0)
    p = _particles(10)

    def census(params, pass_, t, s, count, csum, tidx=None, nt=None, cl=cells):
        return lib.sph_neighbor_census(C.byref(params), C.byref(g), pass_, C.byref(t), tidx, nt, C.byref(s), cl,
                                       count, csum, FAKE, 1 << 40, None)

    assert census(_params(h=0.6), 0, p, p, FAKE, FAKE) == L.SPH_ERR_ARG
    assert "smaller than the support" in _last()
    assert census(_params(), 5, p, p, FAKE, FAKE) == L.SPH_ERR_ARG
    assert "unknown pass" in _last()
    assert census(_params(), 0, p, p, None, FAKE) == L.SPH_ERR_ARG
    assert "count_out" in _last()
    assert census(_params(), 0, p, p, FAKE, None) == L.SPH_ERR_ARG
    assert census(_params(), 0, p, p, FAKE, FAKE, tidx=FAKE) == L.SPH_ERR_ARG
    assert census(_params(), 0, p, p, FAKE, FAKE, cl=L.SphCells(FAKE, 63, 0)) == L.SPH_ERR_ARG
    assert census(_params(prec=L.SPH_FP32_SPLIT), 0, p, p, FAKE, FAKE) == L.SPH_ERR_ARG
    ps = _params()
    ps.material, ps.K, ps.G = L.SPH_SOLID_J2, 1e9, 1e9
    assert census(ps, 0, p, p, FAKE, FAKE) == L.SPH_ERR_ARG
    assert "S[0]" in _last()
    big = _particles(1 << 27)
    assert census(_params(), 0, p, big, FAKE, FAKE) == L.SPH_ERR_ARG
    assert "must be below 134217728" in _last()
    # no targets: nothing to do, even without outputs
    assert census(_params(), 0, _particles(0), p, None, None) == L.SPH_OK


def test_mark_boundary_noalloc_rejects_bad_arguments():
    lib = L.load()
    g = _grid()
    cells = L.SphCells(FAKE, 64, 0)

    def mark(p, cl=cells, comm=FAKE, bidx=FAKE, cap=10, nb=FAKE):
        return lib.sph_mark_boundary_noalloc(C.byref(g), C.byref(p), cl, comm, bidx, cap, nb, None, None)

    # beyond the fixed block-count array: a clear error, before anything runs
    assert mark(_particles((1 << 26) + 1)) == L.SPH_ERR_ARG
    assert "exceeds the 67108864 particles" in _last()
    p = _particles(10)
    assert mark(p, cl=L.SphCells(FAKE, 63, 0)) == L.SPH_ERR_ARG
    assert mark(p, nb=None) == L.SPH_ERR_ARG
    assert mark(p, comm=None) == L.SPH_ERR_ARG
    assert mark(p, bidx=None) == L.SPH_ERR_ARG
    q = _particles(10)
    q.hash = None
    assert mark(q) == L.SPH_ERR_ARG


def test_pair_events_need_both_handles():
    lib = L.load()
    assert lib.sph_set_pair_events(FAKE, None) == L.SPH_ERR_ARG
    assert "both events" in _last()
    assert lib.sph_set_pair_events(None, FAKE) == L.SPH_ERR_ARG
    assert lib.sph_set_pair_events(None, None) == 0   # off: nothing is recorded


def test_passes_over_one_array_need_one_size():
    """A pass whose targets and sources share their hash array is a pass over
    one array (the local-local pass): their sizes must agree."""
    lib = L.load()
    g = _grid()
    cells = L.SphCells(FAKE, 64, 0)
    t, s = _particles(10), _particles(12)
    r = L.SphRates()
    for k in range(6):
        r.hi[k] = FAKE
    assert lib.sph_interact(C.byref(_params()), C.byref(g), 0, C.byref(t), None, None, C.byref(s), cells, 1,
                            C.byref(r), FAKE, 1 << 40, None) == L.SPH_ERR_ARG
    assert "share their hash array" in _last()
    assert lib.sph_count_pairs(C.byref(_params()), C.byref(g), C.byref(t), None, None, C.byref(s), cells, FAKE,
                               None) == L.SPH_ERR_ARG
    assert lib.sph_neighbor_census(C.byref(_params()), C.byref(g), 0, C.byref(t), None, None, C.byref(s), cells, FAKE,
                                   FAKE, FAKE, 1 << 40, None) == L.SPH_ERR_ARG
    full = L.SphAdjoint()
    for d in range(3):
        full.x[d] = full.v[d] = FAKE
    for f in ("m", "omega", "E", "rho", "p", "c", "e"):
        setattr(full, f, FAKE)
    assert lib.sph_interact_adjoint(C.byref(_params()), C.byref(g), 0, C.byref(t), None, None, C.byref(s), cells,
                                    C.byref(r), C.byref(r), C.byref(full), FAKE, 1 << 40, None) == L.SPH_ERR_ARG


def test_integrate_and_adjoint_reject_bad_arguments():
    lib = L.load()
    p = _particles(10)
    ws = L.sph_workspace_size(_grid(), 10, 0, 0)
    # stress stage on a fluid
    assert lib.sph_integrate(C.byref(_params()), L.SPH_STAGE_STRESS, C.byref(p), None, FAKE, None, None, 0,
                             None) == L.SPH_ERR_ARG
    # motion without dt
    r = L.SphRates()
    for k in range(6):
        r.hi[k] = FAKE
    assert lib.sph_integrate(C.byref(_params()), L.SPH_STAGE_MOTION, C.byref(p), C.byref(r), None, FAKE, FAKE, ws,
                             None) == L.SPH_ERR_ARG
    # eos without diagnostics buffer
    assert lib.sph_integrate(C.byref(_params()), L.SPH_STAGE_EOS, C.byref(p), None, None, None, FAKE, ws,
                             None) == L.SPH_ERR_ARG
    # adjoint: walls are not differentiated
    pw = _params()
    pw.wall_mask = 1
    bar = L.SphAdjoint()
    assert lib.sph_integrate_adjoint(C.byref(pw), L.SPH_STAGE_MOTION, C.byref(p), C.byref(r), FAKE, C.byref(bar),
                                     C.byref(r), None, None, 0, None) == L.SPH_ERR_UNSUPPORTED
    # adjoint of a solid
    ps = _params()
    ps.material, ps.K, ps.G = L.SPH_SOLID_J2, 1e9, 1e9
    cl = L.SphCells(FAKE, 64, 0)

    def iadj(params, t, s, rt, rs, b, tidx=None, nt=None):
        return lib.sph_interact_adjoint(C.byref(params), C.byref(_grid()), 0, C.byref(t), tidx, nt, C.byref(s), cl,
                                        None if rt is None else C.byref(rt), None if rs is None else C.byref(rs),
                                        C.byref(b), FAKE, 1 << 40, None)

    # the solid reverse needs the stress fields and takes the linear EOS only
    full0 = L.SphAdjoint()
    for d in range(3):
        full0.x[d] = full0.v[d] = FAKE
    for f in ("m", "omega", "E", "rho", "p", "c", "e"):
        setattr(full0, f, FAKE)
    assert iadj(ps, p, p, r, r, full0) == L.SPH_ERR_ARG
    assert "S[0]" in _last()
    pm = _params()
    pm.material, pm.eos, pm.c0, pm.G, pm.mg_s = L.SPH_SOLID_J2, L.SPH_EOS_MIE_GRUNEISEN, 5000.0, 1e9, 1.3
    assert iadj(pm, p, p, r, r, full0) == L.SPH_ERR_UNSUPPORTED
    assert lib.sph_integrate_adjoint(C.byref(pm), L.SPH_STAGE_MOTION, C.byref(p), C.byref(r), FAKE, C.byref(full0),
                                     C.byref(r), None, None, 0, None) == L.SPH_ERR_UNSUPPORTED
    # the stress stage's reverse is for solids, and needs the stress cotangents
    assert lib.sph_integrate_adjoint(C.byref(_params()), L.SPH_STAGE_STRESS, C.byref(p), C.byref(r), FAKE,
                                     C.byref(full0), C.byref(r), None, None, 0, None) == L.SPH_ERR_ARG
    # the GRADIENT reverse reads the velocity-gradient cotangents
    assert lib.sph_interact_adjoint(C.byref(ps), C.byref(_grid()), 1, C.byref(p), None, None, C.byref(p), cl,
                                    C.byref(r), None, C.byref(full0), FAKE, 1 << 40, None) == L.SPH_ERR_ARG
    assert "Lhi[0]" in _last()
    full = L.SphAdjoint()
    for d in range(3):
        full.x[d] = full.v[d] = FAKE
    for f in ("m", "omega", "E", "rho", "p", "c", "e"):
        setattr(full, f, FAKE)
    # neither rate cotangent given
    assert iadj(_params(), p, p, None, None, full) == L.SPH_ERR_ARG
    assert "no rate cotangents" in _last()
    # a target list needs its device count; the state cotangent needs its fields
    assert iadj(_params(), p, p, r, None, full, tidx=FAKE) == L.SPH_ERR_ARG
    assert iadj(_params(), p, p, None, r, bar) == L.SPH_ERR_ARG
    half = L.SphRates()
    half.hi[0] = FAKE
    assert iadj(_params(), p, p, r, half, full) == L.SPH_ERR_ARG
    assert "rates_bar_sources.hi[1]" in _last()
    assert iadj(_params(), p, _particles(1 << 27), None, r, full) == L.SPH_ERR_ARG
    assert "must be below 134217728" in _last()


def test_objective_adjoint_rejects_bad_arguments():
    lib = L.load()
    p = _particles(10)
    full = L.SphAdjoint()
    for d in range(3):
        full.x[d] = full.v[d] = FAKE
    for f in ("m", "omega", "E", "rho", "p", "c", "e"):
        setattr(full, f, FAKE)
    KE, TZ = L.SPH_OBJ_KINETIC_ENERGY, L.SPH_OBJ_TAGGED_MEAN_Z

    def seed(obj, q=p, tag=None, tag_len=0, ntag=0, scale=1.0, b=full):
        return lib.sph_objective_adjoint(obj, C.byref(q), tag, tag_len, ntag, scale,
                                         None if b is None else C.byref(b), None)

    assert seed(7) == L.SPH_ERR_ARG
    assert "unknown objective" in _last()
    assert seed(KE, b=None) == L.SPH_ERR_ARG
    assert seed(KE, scale=float("nan")) == L.SPH_ERR_ARG
    assert seed(KE, b=L.SphAdjoint()) == L.SPH_ERR_ARG
    assert "bar.v or bar.m" in _last()
    q = _particles(10)
    q.m = None
    assert seed(KE, q) == L.SPH_ERR_ARG
    assert seed(TZ, tag=FAKE, tag_len=10, ntag=0) == L.SPH_ERR_ARG
    assert "ntag = 0" in _last()
    assert seed(TZ, tag=None, tag_len=10, ntag=2) == L.SPH_ERR_ARG
    q = _particles(10)
    q.id = None
    assert seed(TZ, q, FAKE, 10, 2) == L.SPH_ERR_ARG
    # no particles: nothing to do
    assert seed(KE, _particles(0, full=False)) == L.SPH_OK
    # the input-velocity stage reads bar.v and bar.E; unknown stages are refused
    assert lib.sph_integrate_adjoint(C.byref(_params()), L.SPH_STAGE_INPUT_VELOCITY, C.byref(p), None, None,
                                     C.byref(L.SphAdjoint()), None, None, None, 0, None) == L.SPH_ERR_ARG
    assert lib.sph_integrate_adjoint(C.byref(_params()), 9, C.byref(p), None, None, C.byref(full), None, None,
                                     None, 0, None) == L.SPH_ERR_ARG
    assert "unknown adjoint stage" in _last()


def test_zero_particles_is_a_noop():
    lib = L.load()
    g = _grid()
    cells = L.SphCells(FAKE, 64, 0)
    p = _particles(0, full=False)
    r = L.SphRates()
    for k in range(6):
        r.hi[k] = FAKE
    assert lib.sph_interact(C.byref(_params()), C.byref(g), 0, C.byref(p), None, None, C.byref(p), cells, 1,
                            C.byref(r), FAKE, 1 << 30, None) == L.SPH_OK
    out = L.SphParticles()
    out.n = 5
    assert lib.sph_pack_boundary(C.byref(p), None, None, C.byref(L.SphParticles()), None) == L.SPH_OK
    assert lib.sph_permute_adjoint(0, 0, None, None, None, None) == L.SPH_OK


def test_balancing_entry_points_reject_bad_arguments():
    lib = L.load()
    ARG, WS = L.SPH_ERR_ARG, L.SPH_ERR_WORKSPACE
    p = _particles(10)
    n_ws = L.sph_workspace_size(_grid(), 10, 0, 0)
    assert lib.sph_centroid(None, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_centroid(C.byref(p), None, FAKE, n_ws, None) == ARG
    assert lib.sph_centroid(C.byref(p), FAKE, FAKE, 64, None) == WS and "workspace" in _last()
    for hmax in (0, 1 << 20):
        assert lib.sph_balance_hash(C.byref(p), FAKE, FAKE, hmax, FAKE, FAKE, FAKE, n_ws, None) == ARG
        assert "hmax" in _last()
    assert lib.sph_balance_hash(C.byref(p), None, FAKE, 1000, FAKE, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_balance_hash(C.byref(p), FAKE, FAKE, 1000, None, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_balance_select(10, FAKE, 1000, None, FAKE, FAKE, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_balance_select(10, None, 1000, FAKE, FAKE, FAKE, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_balance_select(10, FAKE, 1000, FAKE, FAKE, FAKE, FAKE, None, n_ws, None) == WS
    q = _particles(10, prec=L.SPH_FP32_SPLIT)
    assert lib.sph_swap(C.byref(p), FAKE, C.byref(q), FAKE, FAKE, 10, None) == ARG and "precision" in _last()
    assert lib.sph_swap(C.byref(p), None, C.byref(p), FAKE, FAKE, 10, None) == ARG
    assert lib.sph_swap(C.byref(p), None, C.byref(p), None, None, 0, None) == L.SPH_OK   # nothing to do


def test_type_balancing_entry_points_reject_bad_arguments():
    lib = L.load()
    ARG, WS = L.SPH_ERR_ARG, L.SPH_ERR_WORKSPACE
    p = _particles(10)
    n_ws = L.sph_workspace_size(_grid(), 10, 0, 0)
    for nt in (0, L.SPH_MAX_TYPES + 1):
        assert lib.sph_centroid_types(C.byref(p), FAKE, nt, 0.1, FAKE, FAKE, n_ws, None) == ARG
        assert "ntypes" in _last()
        assert lib.sph_balance_hash_types(C.byref(p), FAKE, nt, FAKE, FAKE, 1000, FAKE, FAKE, FAKE, n_ws,
                                          None) == ARG
        assert lib.sph_balance_select_types(10, FAKE, nt, FAKE, 1000, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, n_ws,
                                            None) == ARG
    for alpha in (-0.1, 1.5, float("nan")):
        assert lib.sph_centroid_types(C.byref(p), FAKE, 2, alpha, FAKE, FAKE, n_ws, None) == ARG
        assert "alpha" in _last()
    assert lib.sph_centroid_types(C.byref(p), None, 2, 0.1, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_centroid_types(C.byref(p), FAKE, 2, 0.1, None, FAKE, n_ws, None) == ARG
    assert lib.sph_centroid_types(C.byref(p), FAKE, 2, 0.1, FAKE, FAKE, 64, None) == WS
    assert lib.sph_balance_hash_types(C.byref(p), FAKE, 2, FAKE, FAKE, 0, FAKE, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_balance_hash_types(C.byref(p), None, 2, FAKE, FAKE, 1000, FAKE, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_balance_hash_types(C.byref(p), FAKE, 2, FAKE, None, 1000, FAKE, FAKE, FAKE, n_ws, None) == ARG
    assert lib.sph_balance_select_types(10, FAKE, 2, FAKE, 1000, FAKE, FAKE, FAKE, FAKE, None, FAKE, n_ws,
                                        None) == ARG
    assert lib.sph_balance_select_types(10, None, 2, FAKE, 1000, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, n_ws,
                                        None) == ARG
    assert lib.sph_balance_select_types(10, FAKE, 2, FAKE, 1000, FAKE, FAKE, FAKE, FAKE, FAKE, None, n_ws,
                                        None) == WS
