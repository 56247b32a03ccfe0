"""GPU parity of the per-type balancing (Section III.B) through the C ABI,
against the oracle.

* Centres: FP64 sums in another order than the oracle's, so
  |gpu - oracle| <= 1e-13 max|x| per component and 1e-13 relative in mass.
* Hashes: integers decided in FP64 from the same centres (the oracle is given
  the device's centres): bit-exact, and so are the per-type positive counts,
  the per-type selections and offsets (a stable sort) and the swapped arrays.
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


def _state(h):
    s = cpu.State(h["x"].shape[0])
    for f in ("x", "v", "m", "w", "rho", "p", "c", "E", "id", "hash"):
        getattr(s, f)[...] = h[f]
    return s


def _labels(wl, seed, p_third):
    lo = np.asarray(wl.grid["origin"], dtype=np.float64)
    hi = lo + np.asarray(wl.grid["dims"]) * wl.grid["cell"]
    c = lo + 0.7 * (hi - lo)
    return S.particle_types(wl.x, c, 0.25 * float((hi - lo).min()), seed=seed, p_third=p_third)


def _check_round(bp, ta, tb):
    nt = bp.ntypes
    sa, sb = _state(bp.A.host()), _state(bp.B.host())
    bp.centroids()
    torch.cuda.synchronize()
    cg = bp.cg.cpu().numpy()
    for q, (s, t) in enumerate(((sa, ta), (sb, tb))):
        ref = cpu.centroid_types(s, t, nt, bp.alpha)
        scale = np.abs(s.x).max() if s.n else 1.0
        assert np.abs(cg[q, :, :3] - ref[:, :3]).max() <= 1e-13 * scale
        assert np.allclose(cg[q, :, 3], ref[:, 3], rtol=1e-13, atol=0)
    bp.hashes()
    torch.cuda.synchronize()
    npos = bp.npos.cpu().numpy()
    bh = [bp.bh[0].cpu().numpy().view(np.uint32)[:sa.n], bp.bh[1].cpu().numpy().view(np.uint32)[:sb.n]]
    refn = []
    for q, (s, t) in enumerate(((sa, ta), (sb, tb))):
        h, n = cpu.balance_hash_types(s, t, nt, cg[q], cg[1 - q], bp.hmax)
        assert np.array_equal(bh[q], h), f"balancing hashes of set {q}"
        assert npos[q].tolist() == n.tolist()
        refn.append(n)
    bp.selections()
    torch.cuda.synchronize()
    sel = []
    for q, t in enumerate((ta, tb)):
        ref, k, off = cpu.balance_select_types(bh[q], t, nt, refn[q], refn[1 - q], bp.hmax)
        assert bp.k[q].cpu().numpy().tolist() == k.tolist()
        assert bp.off[q].cpu().numpy().tolist() == off.tolist()
        got = bp.sel[q].cpu().numpy().view(np.uint32)[:off[-1]]
        assert np.array_equal(got, ref), f"selection of set {q}"
        sel.append(got)
    assert np.array_equal(ta[sel[0]], tb[sel[1]])
    bp.swap()
    torch.cuda.synchronize()
    cpu.swap(sa, sel[0], sb, sel[1])
    for s, p in ((sa, bp.A), (sb, bp.B)):
        h = p.host()
        assert np.array_equal(h["id"], s.id)
        assert np.array_equal(h["x"], s.x)
        for f in ("v", "m", "w", "rho", "E"):
            assert np.array_equal(h[f], getattr(s, f)), f
    return int(bp.off[0, nt].cpu())


@pytest.mark.parametrize("prec", [FP32, FP64])
@pytest.mark.parametrize("ntypes,p_third", [(2, 0.0), (3, 0.1)])
def test_round_matches_oracle(prec, ntypes, p_third):
    from paper_2310_03596_amd.balance import BalanceTypesPair
    a, b = S.c4_share("mixed", seed=8, nx=40, ny=20, nz=20, split_ix=30)
    ta, tb = _labels(a, 80, p_third), _labels(b, 81, p_third)
    print(f"[balance types] prec={prec} ntypes={ntypes} A={a.n} B={b.n}", flush=True)
    bp = BalanceTypesPair(a, b, ta, tb, ntypes, prec)
    k = _check_round(bp, ta, tb)
    assert k > 0
    _check_round(bp, ta, tb)   # a second round on the swapped sets


def test_invalid_labels_and_absent_type():
    """Labels of ntypes or more take no part; a type absent from one side
    swaps nothing."""
    from paper_2310_03596_amd.balance import BalanceTypesPair
    a, b = S.c4_share("mixed", seed=9, nx=30, ny=20, nz=16, split_ix=22)
    rng = np.random.default_rng(82)
    ta = rng.integers(0, 2, size=a.n).astype(np.uint8)
    tb = np.zeros(b.n, dtype=np.uint8)            # type 1 absent from B
    ta[rng.random(a.n) < 0.1] = 200                # not a valid type
    bp = BalanceTypesPair(a, b, ta, tb, 3, FP32)
    _check_round(bp, ta, tb)
    assert bp.k[0, 1].item() == 0 and bp.k[0, 2].item() == 0


def test_one_type_without_bias_is_the_single_type_round():
    from paper_2310_03596_amd.balance import BalancePair, BalanceTypesPair
    a, b = S.c4_share("mixed", seed=10, nx=40, ny=20, nz=20, split_ix=30)
    one = BalancePair(a, b, FP32)
    typ = BalanceTypesPair(a, b, np.zeros(a.n, np.uint8), np.zeros(b.n, np.uint8), 1, FP32, alpha=0.0)
    for bp in (one, typ):
        bp.centroids()
    torch.cuda.synchronize()
    c1, ct = one.cg.cpu().numpy(), typ.cg.cpu().numpy()
    assert np.abs(ct[:, 0, :3] - c1[:, :3]).max() <= 1e-13 * np.abs(a.x).max()
    typ.cg[:, 0, :] = one.cg            # same centres: identical integer decisions
    for bp in (one, typ):
        bp.hashes()
        bp.selections()
    torch.cuda.synchronize()
    for q in range(2):
        assert torch.equal(one.bh[q], typ.bh[q])
        k = int(one.k[q].item())
        assert int(typ.off[q, 1].item()) == k
        assert torch.equal(one.sel[q][:k], typ.sel[q][:k])


def test_full_size_round_two_types():
    """8,000,000 + 2,000,000 particles with a bead of type 1, FP32 split:
    centres, hashes, counts and selections whole, the swap on a sample."""
    from paper_2310_03596_amd.balance import BalanceTypesPair
    a, b = S.c4_share("mixed")
    ta, tb = _labels(a, 83, 0.0), _labels(b, 84, 0.0)
    print(f"[balance types full] A={a.n} B={b.n} bead A={int(ta.sum())} B={int(tb.sum())}", flush=True)
    bp = BalanceTypesPair(a, b, ta, tb, 2, FP32)
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
    for q, (s, t) in enumerate(((sa, ta), (sb, tb))):
        ref = cpu.centroid_types(s, t, 2, bp.alpha)
        assert np.abs(cg[q, :, :3] - ref[:, :3]).max() <= 1e-13 * np.abs(s.x).max()
        h, n = cpu.balance_hash_types(s, t, 2, cg[q], cg[1 - q], bp.hmax)
        got = bp.bh[q].cpu().numpy().view(np.uint32)[:s.n]
        assert np.array_equal(got, h)
        assert npos[q].tolist() == n.tolist()
        bh.append(h)
    sel = []
    for q, t in enumerate((ta, tb)):
        ref, k, off = cpu.balance_select_types(bh[q], t, 2, npos[q], npos[1 - q], bp.hmax)
        assert bp.off[q].cpu().numpy().tolist() == off.tolist()
        got = bp.sel[q].cpu().numpy().view(np.uint32)[:off[-1]]
        assert np.array_equal(got, ref)
        sel.append(got)
    assert sel[0].size > 0 and (bp.k[0].cpu().numpy() > 0).all()
    bp.swap()
    torch.cuda.synchronize()
    ha = bp.A.host()
    rng = np.random.default_rng(96)
    t = rng.choice(sel[0].size, size=min(sel[0].size, 4096), replace=False)
    assert np.array_equal(ha["x"][sel[0][t]], xb[sel[1][t]])
    assert np.array_equal(ta[sel[0]], tb[sel[1]])
