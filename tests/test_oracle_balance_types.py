"""Pins of the per-type balancing in the oracle (Section III.B), CPU only.

Each type is balanced with the single-type rule of Section III.A (pinned in
test_oracle_balance.py) towards the biased centre
Cg'_t = alpha Cg_all + (1 - alpha) Cg_t, alpha = 0.1.
"""
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


def _cube(centre, k=4, step=0.125):
    g = (np.arange(k) - (k - 1) / 2) * step
    return np.stack(np.meshgrid(g + centre[0], g + centre[1], g + centre[2], indexing="ij"), -1).reshape(-1, 3)


def test_biased_centres_closed_form():
    # type 0: a symmetric cube about (0, 0, 0), unit masses; type 1: one about
    # (1, 2, -1) with masses 3.  Cg_all = (3 * 64 * c1) / (64 + 3 * 64) = 3 c1 / 4.
    p0, p1 = _cube((0.0, 0.0, 0.0)), _cube((1.0, 2.0, -1.0))
    s = _cloud(np.concatenate([p0, p1]), np.concatenate([np.ones(64), np.full(64, 3.0)]))
    types = np.repeat([0, 1], 64)
    rec = cpu.centroid_types(s, types, 2)
    c1 = np.array([1.0, 2.0, -1.0])
    call = 0.75 * c1
    assert np.abs(rec[2, :3] - call).max() < 1e-14 and rec[2, 3] == 256.0
    assert np.abs(rec[0, :3] - 0.1 * call).max() < 1e-14 and rec[0, 3] == 64.0
    assert np.abs(rec[1, :3] - (0.1 * call + 0.9 * c1)).max() < 1e-14 and rec[1, 3] == 192.0
    # without bias the records are the plain per-type centres
    rec0 = cpu.centroid_types(s, types, 2, alpha=0.0)
    assert np.abs(rec0[0, :3]).max() < 1e-15 and np.abs(rec0[1, :3] - c1).max() < 1e-14


def test_one_type_is_the_single_type_rule():
    rng = np.random.default_rng(70)
    s = _cloud(rng.uniform(-1, 2, size=(3000, 3)), rng.uniform(0.5, 2.0, size=3000))
    types = np.zeros(s.n, dtype=np.uint8)
    cg, m = cpu.centroid(s)
    rec = cpu.centroid_types(s, types, 1, alpha=0.0)
    assert np.array_equal(rec[0, :3], cg) and rec[0, 3] == m and np.array_equal(rec[1, :3], cg)
    own, other = rec[:1], np.array([[1.5, 0.2, 0.9, 0.0]])
    h, npos = cpu.balance_hash_types(s, types, 1, own, other)
    h1, n1 = cpu.balance_hash(s, own[0, :3], other[0, :3])
    assert np.array_equal(h, h1) and npos.tolist() == [n1]
    sel, k, off = cpu.balance_select_types(h, types, 1, [n1], [n1 // 3])
    assert k.tolist() == [n1 // 3] and off.tolist() == [0, n1 // 3]
    assert np.array_equal(sel, cpu.balance_select(h, n1 // 3))


def test_bias_moves_the_hash():
    # Along x: A holds type 0 at x = 0 and type 1 at x = 1 (equal masses), so
    # Cg_all(A) = 0.5 and Cg'_1(A) = 0.05 + 0.9 = 0.95; the other side's biased
    # centre for type 1 is put at 2.95.  Midpoint 1.95, half distance 1, so a
    # type-1 particle at x has hash ceil(1000 (x - 1.95)) between the two.
    a = _cloud(np.concatenate([_cube((0.0, 0.0, 0.0)), _cube((1.0, 0.0, 0.0))]))
    types = np.repeat([0, 1], 64).astype(np.uint8)
    rec = cpu.centroid_types(a, types, 2)
    assert abs(rec[1, 0] - 0.95) < 1e-15 and abs(rec[0, 0] - 0.05) < 1e-15
    other = rec.copy()
    other[1, :3] = [2.95, 0.0, 0.0]
    probe = _cloud([[2.2504, 0.0, 0.0], [1.9, 0.0, 0.0], [3.5, 0.0, 0.0]])
    h, npos = cpu.balance_hash_types(probe, np.array([1, 1, 1]), 2, rec, other)
    assert h.tolist() == [301, 0, 1000] and npos.tolist() == [0, 2]
    # the unbiased type-1 centre (1.0, midpoint 1.975) gives another hash
    rec0 = cpu.centroid_types(a, types, 2, alpha=0.0)
    other0 = rec0.copy()
    other0[1, :3] = [2.95, 0.0, 0.0]
    h0, _ = cpu.balance_hash_types(probe, np.array([1, 1, 1]), 2, rec0, other0)
    assert h0[0] != h[0]


def test_invalid_labels_take_no_part():
    rng = np.random.default_rng(71)
    s = _cloud(rng.uniform(0, 1, size=(500, 3)))
    types = rng.integers(0, 2, size=500).astype(np.uint8)
    bad = rng.random(500) < 0.2
    t2 = types.copy()
    t2[bad] = 7
    rec_all = cpu.centroid_types(s, t2, 2)
    keep = ~bad
    sub = _cloud(s.x[keep])
    assert np.array_equal(rec_all, cpu.centroid_types(sub, types[keep], 2))
    other = rec_all + np.array([0.3, 0.0, 0.0, 0.0])
    h, npos = cpu.balance_hash_types(s, t2, 2, rec_all, other)
    assert (h[bad] == 0).all()
    sel, k, off = cpu.balance_select_types(h, t2, 2, npos, npos)
    assert not np.isin(sel, np.nonzero(bad)[0]).any() and off[-1] == npos.sum()


def test_select_types_brute_force():
    rng = np.random.default_rng(72)
    n = 400
    types = rng.integers(0, 4, size=n).astype(np.uint8)
    h = rng.integers(0, 1001, size=n).astype(np.uint32)
    h[rng.random(n) < 0.4] = 0
    npos = np.array([(h[types == t] > 0).sum() for t in range(3)])
    other = np.array([5, 1000, 0])
    sel, k, off = cpu.balance_select_types(h, types, 3, npos, other)
    ref, ks = [], []
    for t in range(3):
        idx = [i for i in range(n) if types[i] == t]
        kt = min(int(npos[t]), int(other[t]), len(idx))
        ref += sorted(idx, key=lambda i: (-int(h[i]), i))[:kt]
        ks.append(kt)
    assert sel.tolist() == ref and k.tolist() == ks and off.tolist() == [0, ks[0], ks[0] + ks[1], sum(ks)]


def test_empty_type_swaps_nothing():
    rng = np.random.default_rng(73)
    s = _cloud(rng.uniform(0, 1, size=(200, 3)))
    types = np.zeros(200, dtype=np.uint8)   # type 1 absent here
    rec = cpu.centroid_types(s, types, 2)
    assert rec[1].tolist() == [0.0, 0.0, 0.0, 0.0]
    _, npos = cpu.balance_hash_types(s, types, 2, rec, rec + 0.5)
    _, k, _ = cpu.balance_select_types(np.zeros(200, np.uint32), types, 2, npos, [10, 10])
    assert k[1] == 0


def _round_types(a, ta, b, tb, ntypes):
    ra, rb = cpu.centroid_types(a, ta, ntypes), cpu.centroid_types(b, tb, ntypes)
    ha, na = cpu.balance_hash_types(a, ta, ntypes, ra, rb)
    hb, nb = cpu.balance_hash_types(b, tb, ntypes, rb, ra)
    sa, ka, oa = cpu.balance_select_types(ha, ta, ntypes, na, nb)
    sb, kb, ob = cpu.balance_select_types(hb, tb, ntypes, nb, na)
    assert np.array_equal(ka, kb) and np.array_equal(oa, ob)
    assert np.array_equal(ta[sa], tb[sb])   # every pair is of one type
    cpu.swap(a, sa, b, sb)
    return int(oa[-1])


def test_rounds_keep_type_counts_and_separate_types():
    """Two GPUs holding randomly mixed halves of a two-type lattice (a bead of
    type 1 inside type 0): rounds keep every type's count on each side and
    shrink each type's exchange set."""
    wl = S.jittered_lattice(14, seed=74, dx=1e-3)
    full = cpu.State.from_workload(wl)
    c = full.x.mean(0)
    t_full = (np.linalg.norm(full.x - c, axis=1) < 4e-3).astype(np.uint8)
    own = np.random.default_rng(75).permutation(wl.n) < wl.n // 2
    a, b = cpu.State(int(own.sum())), cpu.State(int((~own).sum()))
    for dst, m in ((a, own), (b, ~own)):
        for f in ("x", "v", "m", "w", "rho", "p", "c", "E", "id"):
            getattr(dst, f)[...] = getattr(full, f)[m]
    ta, tb = t_full[own], t_full[~own]
    counts0 = [np.bincount(ta, minlength=2).tolist(), np.bincount(tb, minlength=2).tolist()]

    def boundary(t):
        ma, mb = ta == t, tb == t
        pa, pb = cpu.State(int(ma.sum())), cpu.State(int(mb.sum()))
        pa.x[:], pb.x[:] = a.x[ma], b.x[mb]
        oa, _, _ = cpu.build_cells(wl.grid, pa)
        _, _, sb = cpu.build_cells(wl.grid, pb)
        return cpu.mark_boundary(wl.grid, oa.hash, sb)[1].size

    before = [boundary(t) for t in (0, 1)]
    swaps = [_round_types(a, ta, b, tb, 2) for _ in range(25)]
    after = [boundary(t) for t in (0, 1)]
    # the types ride with their particles: the labels did not move, so the
    # per-side type counts can only stay if every pair was of one type
    assert [np.bincount(ta, minlength=2).tolist(), np.bincount(tb, minlength=2).tolist()] == counts0
    assert swaps[0] > 0
    assert after[0] < 0.5 * before[0] and after[1] < before[1], (before, after)
    ids = np.concatenate([a.id, b.id])
    assert np.array_equal(np.sort(ids), np.sort(full.id))
