"""Pins of the balancing heuristic in the oracle (Section III.A), CPU only."""
import math

import numpy as np
import pytest

import sph_synth as S
from oracle import cpu


def _cloud(points, masses=None):
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    s = cpu.State(points.shape[0])
    s.x[:] = points
    s.m[:] = 1.0 if masses is None else masses
    s.w[:] = 1.0
    s.id[:] = np.arange(points.shape[0], dtype=np.uint32)
    return s


def test_centroid_closed_forms():
    cg, m = cpu.centroid(_cloud([[0, 0, 0], [4, 0, 0]], masses=[1.0, 3.0]))
    assert np.array_equal(cg, [3.0, 0.0, 0.0]) and m == 4.0
    # a symmetric lattice about (0.5, 0.25, -2): its centre exactly
    g = (np.arange(8) - 3.5) * 0.125
    pts = np.stack(np.meshgrid(g + 0.5, g + 0.25, g - 2.0, indexing="ij"), -1).reshape(-1, 3)
    cg, m = cpu.centroid(_cloud(pts))
    assert np.abs(cg - [0.5, 0.25, -2.0]).max() < 1e-15 and m == 512.0


def test_balance_hash_on_the_line():
    # Cg_A = 0, Cg_B = (2, 0, 0): midpoint 1, half distance 1
    pts = [[0.5, 0, 0], [1.0, 0, 0], [1.25, 0, 0], [1.25 + 1e-4, 0, 0], [1.5, 7, -3], [2.0, 0, 0],
           [5.0, 1, 1], [-3.0, 0, 0], [1.0 + 1e-9, 0, 0]]
    h, npos = cpu.balance_hash(_cloud(pts), [0, 0, 0], [2, 0, 0])
    assert h.tolist() == [0, 0, 250, 251, 500, 1000, 1000, 0, 1]
    assert npos == 6


def test_balance_hash_diagonal_and_degenerate():
    # towards (1, 1, 0): the projection of (x, y) past the midpoint (0.5, 0.5)
    # is ((x + y) - 1) / sqrt 2 over a half distance sqrt(2) / 2
    pts = [[0.75, 0.75, 3.0], [1.0, 0.5, 0.0], [0.5, 0.5, 0.0], [0.9, 0.9, -1.0]]
    h, _ = cpu.balance_hash(_cloud(pts), [0, 0, 0], [1, 1, 0])
    assert h.tolist() == [500, 500, 0, 800]
    h, npos = cpu.balance_hash(_cloud(pts), [1, 2, 3], [1, 2, 3])
    assert h.tolist() == [0, 0, 0, 0] and npos == 0


def test_balance_hash_within_one_of_the_square_root_form():
    rng = np.random.default_rng(40)
    pts = rng.uniform(-1, 3, size=(2000, 3))
    a, b = np.array([0.1, -0.2, 0.3]), np.array([1.7, 0.4, 1.1])
    h, npos = cpu.balance_hash(_cloud(pts), a, b)
    e = b - a
    d = math.sqrt(float(e @ e))
    s = (pts - 0.5 * (a + b)) @ e / d
    ref = np.where(s <= 0, 0, np.where(s >= d / 2, 1000, np.ceil(1000 * s / (d / 2))))
    assert np.abs(h.astype(np.int64) - ref.astype(np.int64)).max() <= 1
    assert npos == int((h > 0).sum())


def test_balance_select_matches_sorted():
    rng = np.random.default_rng(41)
    h = rng.integers(0, 1001, size=500).astype(np.uint32)
    h[rng.integers(0, 500, size=200)] = 0
    for k in (0, 1, 17, 300):
        sel = cpu.balance_select(h, k)
        ref = sorted(range(500), key=lambda i: (-int(h[i]), i))[:k]
        assert sel.tolist() == ref


def test_swap_exchanges_selected_particles():
    wa, wb = S.c1_cube(n_side=6), S.c1_cube(n_side=5, seed=2)
    a, b = cpu.State.from_workload(wa), cpu.State.from_workload(wb)
    b.id[:] += 10000
    a0, b0 = a.copy(), b.copy()
    sa = np.array([3, 0, 7], dtype=np.uint32)
    sb = np.array([1, 10, 2], dtype=np.uint32)
    cpu.swap(a, sa, b, sb)
    assert a.n == a0.n and b.n == b0.n
    for i, j in zip(sa, sb):
        assert a.id[i] == b0.id[j] and b.id[j] == a0.id[i]
        assert np.array_equal(a.x[i], b0.x[j]) and np.array_equal(b.v[j], a0.v[i])
        assert a.E[i] == b0.E[j] and b.m[j] == a0.m[i]
    keep = np.setdiff1d(np.arange(a.n), sa)
    assert np.array_equal(a.x[keep], a0.x[keep])
    assert sorted(np.concatenate([a.id, b.id]).tolist()) == sorted(np.concatenate([a0.id, b0.id]).tolist())


def _round(a, b, grid):
    ca, _ = cpu.centroid(a)
    cb, _ = cpu.centroid(b)
    ha, na = cpu.balance_hash(a, ca, cb)
    hb, nb = cpu.balance_hash(b, cb, ca)
    k = min(na, nb)
    cpu.swap(a, cpu.balance_select(ha, k), b, cpu.balance_select(hb, k))
    return k


def _boundary_count(a, b, grid):
    oa, _, _ = cpu.build_cells(grid, a)
    ob, _, sb = cpu.build_cells(grid, b)
    _, bidx = cpu.mark_boundary(grid, oa.hash, sb)
    return bidx.size


def test_swapping_separates_two_mixed_clouds():
    """Two GPUs holding randomly mixed halves of a lattice: repeated balancing
    keeps both counts and shrinks the exchange set towards a surface."""
    wl = S.jittered_lattice(16, seed=42, dx=1e-3)
    rng = np.random.default_rng(43)
    own = rng.permutation(wl.n) < wl.n // 2
    full = cpu.State.from_workload(wl)
    a, b = cpu.State(int(own.sum())), cpu.State(int((~own).sum()))
    for dst, m in ((a, own), (b, ~own)):
        for f in ("x", "v", "m", "w", "rho", "p", "c", "E", "id"):
            getattr(dst, f)[...] = getattr(full, f)[m]
    n0 = (a.n, b.n)
    before = _boundary_count(a, b, wl.grid)
    swaps = [_round(a, b, wl.grid) for _ in range(30)]
    after = _boundary_count(a, b, wl.grid)
    assert (a.n, b.n) == n0
    assert swaps[0] > 0
    assert after < 0.5 * before, (before, after, swaps)
