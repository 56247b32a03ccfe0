"""GPU parity of the particle-swapping heuristic (Section III.A) through the
C ABI, against the oracle.

* Centres of gravity: FP64 sums in another order than the oracle's, so
  |gpu - oracle| <= 1e-13 max|x| per component and 1e-13 relative in mass.
* Balancing hashes: integers decided in FP64 from the same centres (the
  oracle is given the device's centres): bit-exact, and so are the positive
  counts, the selections (a stable sort) and the swapped arrays.
"""
import numpy as np
import pytest
import torch

import sph_synth as S
from oracle import cpu

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair(layout="mixed", nx=40, ny=20, nz=20, split=30, seed=4):
    return S.c4_share(layout, seed=seed, nx=nx, ny=ny, nz=nz, split_ix=split)


def _state(h):
    s = cpu.State(h["x"].shape[0])
    for f in ("x", "v", "m", "w", "rho", "p", "c", "E", "id", "hash"):
        getattr(s, f)[...] = h[f]
    return s


def _check_round(bp, prec):
    """Run one round step by step, comparing every stage with the oracle."""
    ha, hb = bp.A.host(), bp.B.host()
    sa, sb = _state(ha), _state(hb)
    bp.centroids()
    torch.cuda.synchronize()
    cg = bp.cg.cpu().numpy()
    for q, s in enumerate((sa, sb)):
        ref, m = cpu.centroid(s)
        scale = np.abs(s.x).max() if s.n else 1.0
        assert np.abs(cg[q, :3] - ref).max() <= 1e-13 * scale
        assert cg[q, 3] == pytest.approx(m, rel=1e-13)
    bp.hashes()
    torch.cuda.synchronize()
    npos = bp.npos.cpu().numpy()
    bh = [bp.bh[0].cpu().numpy().view(np.uint32)[:sa.n], bp.bh[1].cpu().numpy().view(np.uint32)[:sb.n]]
    ref_h = []
    for q, s in enumerate((sa, sb)):
        h, n = cpu.balance_hash(s, cg[q, :3], cg[1 - q, :3], bp.hmax)
        assert np.array_equal(bh[q], h), f"balancing hash of set {q}"
        assert npos[q] == n
        ref_h.append(h)
    bp.selections()
    torch.cuda.synchronize()
    k = int(min(npos[0], npos[1], sa.n, sb.n))
    kk = bp.k.cpu().numpy()
    assert kk[0] == k and kk[1] == k
    sel = []
    for q in range(2):
        got = bp.sel[q].cpu().numpy().view(np.uint32)[:k]
        assert np.array_equal(got, cpu.balance_select(ref_h[q], k, bp.hmax)), f"selection of set {q}"
        sel.append(got)
    bp.swap()
    torch.cuda.synchronize()
    cpu.swap(sa, sel[0], sb, sel[1])
    for s, p in ((sa, bp.A), (sb, bp.B)):
        h = p.host()
        assert np.array_equal(h["id"], s.id)
        assert np.array_equal(h["x"], s.x)
        for f in ("v", "m", "w", "rho", "E"):
            assert np.array_equal(h[f], getattr(s, f)), f
    return k


@pytest.mark.parametrize("prec", [FP32, FP64])
@pytest.mark.parametrize("layout", ["mixed", "slab"])
def test_round_matches_oracle(prec, layout):
    from paper_2310_03596_amd.balance import BalancePair
    a, b = _pair(layout)
    print(f"[balance] {layout} prec={prec} A={a.n} B={b.n}", flush=True)
    bp = BalancePair(a, b, prec)
    k = _check_round(bp, prec)
    if layout == "mixed":
        assert k > 0
    k2 = _check_round(bp, prec)   # a second round on the swapped sets
    assert k2 <= max(k, 1) * 2


def test_identical_centres_swap_nothing():
    from paper_2310_03596_amd.balance import BalancePair
    w = S.jittered_lattice(8, seed=60, dx=1e-3)
    bp = BalancePair(w, w, FP64)
    h0 = bp.A.host()
    bp.round()
    torch.cuda.synchronize()
    assert bp.k.cpu().numpy().tolist() == [0, 0]
    assert bp.npos.cpu().numpy().tolist() == [0, 0]
    assert np.array_equal(bp.A.host()["x"], h0["x"])


def test_rounds_separate_mixed_sets():
    """Repeated rounds keep both counts and shrink the exchange set."""
    from paper_2310_03596_amd.balance import BalancePair
    a, b = _pair("mixed", nx=24, ny=24, nz=24, split=12, seed=44)
    bp = BalancePair(a, b, FP32)

    def boundary():
        sa, sb = _state(bp.A.host()), _state(bp.B.host())
        oa, _, _ = cpu.build_cells(a.grid, sa)
        _, _, st = cpu.build_cells(a.grid, sb)
        return cpu.mark_boundary(a.grid, oa.hash, st)[1].size

    before = boundary()
    for _ in range(30):
        bp.round()
    torch.cuda.synchronize()
    after = boundary()
    print(f"boundary particles {before} -> {after}", flush=True)
    assert (bp.A.n, bp.B.n) == (a.n, b.n)
    assert after < 0.5 * before
    ids = np.concatenate([bp.A.host()["id"], bp.B.host()["id"]])
    assert np.array_equal(np.sort(ids), np.sort(np.concatenate([a.id, b.id])))


def test_full_size_round_mixed():
    """8,000,000 + 2,000,000 particles (one GPU's share and its partner's),
    FP32 split: hashes, counts and selections whole, swap on a sample."""
    from paper_2310_03596_amd.balance import BalancePair
    a, b = S.c4_share("mixed")
    print(f"[balance full] A={a.n} B={b.n}", flush=True)
    bp = BalancePair(a, b, FP32)
    xa, xb = a.x.copy(), b.x.copy()
    sa, sb = cpu.State(a.n), cpu.State(b.n)
    sa.x[:], sb.x[:] = xa, xb
    sa.m[:], sb.m[:] = a.m.astype(np.float32), b.m.astype(np.float32)
    bp.centroids()
    bp.hashes()
    bp.selections()
    torch.cuda.synchronize()
    cg = bp.cg.cpu().numpy()
    npos = bp.npos.cpu().numpy()
    bh = []
    for q, s in enumerate((sa, sb)):
        ref, m = cpu.centroid(s)
        assert np.abs(cg[q, :3] - ref).max() <= 1e-13 * np.abs(s.x).max()
        h, n = cpu.balance_hash(s, cg[q, :3], cg[1 - q, :3], bp.hmax)
        got = bp.bh[q].cpu().numpy().view(np.uint32)[:s.n]
        assert np.array_equal(got, h)
        assert npos[q] == n
        bh.append(h)
    k = int(min(npos))
    assert k > 0
    sel = [bp.sel[q].cpu().numpy().view(np.uint32)[:k] for q in range(2)]
    for q in range(2):
        assert np.array_equal(sel[q], cpu.balance_select(bh[q], k, bp.hmax))
    bp.swap()
    torch.cuda.synchronize()
    ha, hb = bp.A.host(), bp.B.host()
    rng = np.random.default_rng(95)
    t = rng.choice(k, size=min(k, 4096), replace=False)
    assert np.array_equal(ha["x"][sel[0][t]], xb[sel[1][t]])
    assert np.array_equal(hb["x"][sel[1][t]], xa[sel[0][t]])
    assert np.array_equal(ha["id"][sel[0][t]], b.id[sel[1][t]])
