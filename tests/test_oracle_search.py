"""Pins of the oracle's bucket hash, stable sort, cell table, neighbour set and
communication hash against brute force and closed forms (CPU only)."""
import numpy as np
import pytest

import sph_synth as S
from oracle import cpu
from tests import brute


def _cases():
    yield S.random_cloud(600, seed=11, h=0.04)
    yield S.jittered_lattice(9, seed=12)
    w = S.random_cloud(400, seed=13, h=0.05, box=0.5)
    # positions exactly on bucket faces and one ulp either side
    L = w.grid["cell"]
    k = np.arange(w.n) % 4
    w.x[:, 0] = k * L
    w.x[1::3, 1] = np.nextafter(w.x[1::3, 0], np.inf)
    w.x[2::3, 1] = np.nextafter(w.x[2::3, 0], -np.inf)
    w.x = np.clip(w.x, 0.0, None)
    yield w


@pytest.mark.parametrize("wl", list(_cases()), ids=["cloud", "lattice", "faces"])
def test_hash_is_containing_bucket(wl):
    """Section I: hash = bucket containing the particle (x-fastest linear index)."""
    h = cpu.hash_cells(wl.grid, wl.x)
    n = np.asarray(wl.grid["dims"])
    c = np.stack([h % n[0], (h // n[0]) % n[1], h // (n[0] * n[1])], axis=1).astype(np.int64)
    o = np.asarray(wl.grid["origin"])
    L = wl.grid["cell"]
    # containment: o + c L <= x < o + (c + 1) L for interior particles (by FP64 division)
    t = (wl.x - o) / L
    assert np.all(c <= np.maximum(t, 0))
    inside = (t < n)
    assert np.all(t[inside] < c[inside] + 1)
    assert np.all(c < n) and np.all(c >= 0)


def test_hash_clamps_outside_particles():
    wl = S.random_cloud(64, seed=3, h=0.1)
    wl.x[:8] = -5.0
    wl.x[8:16] = 7.0
    h = cpu.hash_cells(wl.grid, wl.x)
    n = wl.grid["dims"]
    assert np.all(h[:8] == 0)
    assert np.all(h[8:16] == (n[0] - 1) + n[0] * ((n[1] - 1) + n[1] * (n[2] - 1)))


def test_sort_matches_numpy_stable_argsort():
    """Stable radix sort by hash: same permutation as a library stable sort."""
    rng = np.random.default_rng(7)
    for nkeys in (1, 5, 512, 1 << 18):
        key = rng.integers(0, nkeys, size=20000).astype(np.uint32)
        perm = cpu.sort_perm(key, nkeys)
        assert np.array_equal(perm, np.argsort(key, kind="stable").astype(np.uint32))
    assert cpu.sort_perm(np.zeros(0, np.uint32), 4).shape == (0,)


def test_cell_start_table():
    rng = np.random.default_rng(8)
    nc = 300
    key = np.sort(rng.integers(0, nc, size=5000)).astype(np.uint32)
    start = cpu.cell_start(key, nc)
    assert start[0] == 0 and start[nc] == key.shape[0]
    for c in range(nc):
        assert np.all(key[start[c]:start[c + 1]] == c)
    assert np.array_equal(start[:-1], np.searchsorted(key, np.arange(nc), side="left"))


@pytest.mark.parametrize("wl", list(_cases()), ids=["cloud", "lattice", "faces"])
def test_neighbor_set_matches_brute_force(wl):
    """Bucket search over the 27 buckets finds exactly {j != i : r < 2h}."""
    s = cpu.State.from_workload(wl)
    srt, perm, start = cpu.build_cells(wl.grid, s)
    pi, pj = cpu.neighbors(wl.params, wl.grid, srt, srt, start, True)
    got = set(zip(pi.tolist(), pj.tolist()))
    ref = brute.neighbor_pairs(srt.x, srt.x, wl.params["h"], True)
    assert got == ref
    assert len(got) == len(pi)          # no pair visited twice
    # visiting order is ascending sorted index per target
    for i in np.unique(pi)[:50]:
        js = pj[pi == i]
        assert np.all(np.diff(js.astype(np.int64)) > 0)


def test_neighbor_count_on_lattice():
    """Perfect lattice with h = 1.3 dx: 80 neighbours inside 2h (shells r^2 = 1..6)."""
    wl = S.jittered_lattice(12, seed=0, jitter=0.0)
    s = cpu.State.from_workload(wl)
    srt, perm, start = cpu.build_cells(wl.grid, s)
    pi, pj = cpu.neighbors(wl.params, wl.grid, srt, srt, start, True)
    cnt = np.bincount(pi, minlength=wl.n)
    ix = np.round(srt.x / wl.extra["dx"] - 0.5).astype(int)
    interior = np.all((ix >= 3) & (ix <= 8), axis=1)
    assert np.all(cnt[interior] == 80)


def test_remote_pass_neighbors():
    wl = S.random_cloud(500, seed=21, h=0.05)
    rem = S.random_cloud(300, seed=22, h=0.05)
    s = cpu.State.from_workload(wl)
    r = cpu.State.from_workload(rem)
    srt, _, _ = cpu.build_cells(wl.grid, s)
    rs, _, rstart = cpu.build_cells(wl.grid, r)
    pi, pj = cpu.neighbors(wl.params, wl.grid, srt, rs, rstart, False)
    assert set(zip(pi.tolist(), pj.tolist())) == brute.neighbor_pairs(srt.x, rs.x, 0.05, False)


@pytest.mark.parametrize("layout", ["slab", "mixed"])
def test_mark_matches_brute_force(layout):
    """Section II step c: comm hash = hash if remote particles are in the bucket
    or the surrounding buckets, else G = ncells; B lists flagged particles in order."""
    loc, rem = S.c4_share(layout, seed=40, nx=30, ny=14, nz=12, split_ix=22)
    s = cpu.State.from_workload(loc)
    r = cpu.State.from_workload(rem)
    srt, _, _ = cpu.build_cells(loc.grid, s)
    rs, _, rstart = cpu.build_cells(loc.grid, r)
    comm, bidx = cpu.mark_boundary(loc.grid, srt.hash, rstart)
    flags = brute.boundary_flags(loc.grid, srt.x, rs.x)
    G = cpu.ncells(loc.grid)
    assert np.array_equal(comm != G, flags)
    assert np.array_equal(comm[flags], srt.hash[flags])
    assert np.array_equal(bidx, np.flatnonzero(flags).astype(np.uint32))
    # a stable sort by comm hash puts exactly B first, in sorted order
    perm = np.argsort(comm, kind="stable")
    assert np.array_equal(perm[: bidx.size], bidx)


def test_mark_slab_closed_form():
    """Slab split at lattice column s with L = 2.6 dx: exactly the two local columns
    ix in {s-2, s-1} share or touch the first remote bucket (closed form 2 ny nz)."""
    ny, nz = 20, 16
    loc, rem = S.c4_share("slab", seed=41, nx=60, ny=ny, nz=nz, split_ix=50)
    s = cpu.State.from_workload(loc)
    r = cpu.State.from_workload(rem)
    srt, _, _ = cpu.build_cells(loc.grid, s)
    rs, _, rstart = cpu.build_cells(loc.grid, r)
    comm, bidx = cpu.mark_boundary(loc.grid, srt.hash, rstart)
    # remote x >= 50.45 dx -> bucket floor(50.45 / 2.6) = 19 spans [49.4, 52.0) dx;
    # local bucket 18 spans [46.8, 49.4): columns 47 (47.5 +- 0.05) and 48.  Bucket 19 holds
    # local column 49.  So flagged = columns 47, 48, 49 -> 3 ny nz.
    assert bidx.size == 3 * ny * nz
    ix = np.round(srt.x[bidx, 0] / 1e-3 - 0.5).astype(int)
    assert set(ix.tolist()) == {47, 48, 49}


@pytest.mark.slow
def test_mark_full_share_slab_count():
    """The 8M + 2M slab share: remote starts at column 200 (bucket 77, [200.2, 202.8) dx);
    local bucket 76 = [197.6, 200.2) dx holds columns 198, 199 -> n_B = 2 * 200 * 200."""
    loc, rem = S.c4_share("slab")
    s = cpu.State.from_workload(loc)
    r = cpu.State.from_workload(rem)
    lh = cpu.hash_cells(loc.grid, s.x)
    perm = cpu.sort_perm(lh, cpu.ncells(loc.grid))
    rh = np.sort(cpu.hash_cells(loc.grid, r.x))
    rstart = cpu.cell_start(rh, cpu.ncells(loc.grid))
    comm, bidx = cpu.mark_boundary(loc.grid, lh[perm], rstart)
    assert bidx.size == 80000
