"""Neighbour sets of the production pair kernel (Section I: a particle's
neighbours lie in its own bucket or the 26 around it), through
``sph_neighbor_census``: the same staging, wavefront mapping, filter, hit
lists and predicate as the FORCE and GRADIENT passes, reporting per target
the number of sources evaluated and a checksum of their ids.

Expected sets come from the definition {j : r_ij < 2h} evaluated in FP64
(tests/census.py; pinned on the CPU against the O(N^2) brute force and the
oracle's bucket search), the pairs at r = 0 included (they are evaluated and
add exactly zero).

* FP64 form: count and checksum equal for every target (bit-exact sets).
* FP32-split form: every pair with |r / 2h - 1| >= 1e-6 in the set exactly as
  in FP64; pairs closer than that to the support edge may fall either way,
  and their number is reported (their terms are ~(2 - q)^2 ~ 1e-12 of a
  full-strength term).
"""
import numpy as np
import pytest
import torch

import sph_synth as S
from tests.census import expected, match, mix64, sum64
from tests.test_gpu_parity import CASES

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
PRECS = [pytest.param(FP64, id="fp64"), pytest.param(FP32, id="fp32split")]
WINDOW = {FP64: 0.0, FP32: 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_03596_amd import _lib
    _lib.load()


def check_census(cnt, chk, targets, x_t, x_s, id_s, h, prec, what):
    """Compare the device census of `targets` (indices into cnt/chk; x_t their
    positions) with the expected sets among sources x_s (ids id_s).  Returns
    the number of pairs near r = 2h on which the FP32 form differs."""
    ex = expected(x_t, x_s, h, WINDOW[prec])
    bad, differ = [], 0
    for k, i in enumerate(targets):
        core = id_s[ex.core[k]]
        if prec == FP64:
            ok = int(cnt[i]) == core.size and int(chk[i]) == sum64(mix64(core))
            if not ok:
                bad.append((int(i), int(cnt[i]), core.size))
        else:
            m = match(int(cnt[i]), int(chk[i]), core, id_s[ex.amb[k]], ex.amb_in[k])
            if m is None:
                bad.append((int(i), int(cnt[i]), core.size, ex.amb[k].size))
            else:
                differ += m
    assert not bad, f"{what}: {len(bad)} targets with a different neighbour set, first {bad[:5]}"
    print(f"{what}: {len(targets)} targets, FP32 pairs differing within 1e-6 of r = 2h: {differ}", flush=True)
    return differ


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(CASES))
def test_force_pass_neighbour_sets(case, prec):
    """Local-local FORCE pass of a fluid (row-aligned wavefronts)."""
    from paper_2310_03596_amd.sim import Sim
    wl = CASES[case]()
    print(f"[census] case={case} prec={prec} n={wl.n}", flush=True)
    sim = Sim(wl, prec)
    sim.build()
    cnt, chk = sim.census()
    h = sim.A.host()
    check_census(cnt, chk, np.arange(wl.n), h["x"], h["x"], h["id"], wl.params["h"], prec, case)


@pytest.mark.parametrize("prec", PRECS)
def test_solid_passes_neighbour_sets(prec):
    """GRADIENT and solid FORCE passes (64 consecutive targets per
    wavefront, grouped by bucket row), on a jittered block."""
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.sim import Sim
    wl = S.solid_block(9, seed=73, s_sigma=1e7)
    sim = Sim(wl, prec)
    sim.build()
    h = sim.A.host()
    for pass_ in (L.SPH_PASS_GRADIENT, L.SPH_PASS_FORCE):
        cnt, chk = sim.census(pass_)
        check_census(cnt, chk, np.arange(wl.n), h["x"], h["x"], h["id"], wl.params["h"], prec, f"solid pass {pass_}")


@pytest.mark.parametrize("layout", ["slab", "mixed"])
@pytest.mark.parametrize("prec", PRECS)
def test_share_passes_neighbour_sets(layout, prec):
    """Local-local pass over every local particle and local-remote pass over
    the boundary list (a target list) against the separate remote array."""
    from paper_2310_03596_amd.sim import SharePass
    loc, rem = S.c4_share(layout, seed=74, nx=40, ny=18, nz=16, split_ix=30)
    sp = SharePass(loc, rem, prec)
    sp.build()
    sp.mark()
    c_ll, s_ll, c_lr, s_lr = sp.census()
    hl, hr = sp.LB.host(), sp.RB.host()
    nb = int(sp.nb.cpu()[0])
    bidx = sp.bidx.cpu().numpy().view(np.uint32)[:nb]
    h = loc.params["h"]
    check_census(c_ll, s_ll, np.arange(loc.n), hl["x"], hl["x"], hl["id"], h, prec, f"{layout} local-local")
    check_census(c_lr, s_lr, bidx, hl["x"][bidx], hr["x"], hr["id"], h, prec, f"{layout} local-remote")
    # particles off the list have no remote neighbour, and the list pass left them alone
    off = np.setdiff1d(np.arange(loc.n), bidx)
    ex = expected(hl["x"][off], hr["x"], h)
    assert all(c.size == 0 for c in ex.core)
    assert not c_lr[off].any()


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_column_full_size_neighbour_sets(prec):
    """The 810,448-particle column in the benchmark's launch configuration:
    every target's count adds up to the pair count (each particle also
    evaluates itself), and 4,096 sampled targets have the expected sets."""
    from paper_2310_03596_amd.sim import Sim
    wl = S.c2_column()
    print(f"[census column full] n={wl.n} prec={prec}", flush=True)
    sim = Sim(wl, prec)
    sim.build()
    cnt, chk = sim.census()
    _, pairs = sim.count_pairs()
    assert int(cnt.astype(np.int64).sum()) == pairs + wl.n
    h = sim.A.host()
    rng = np.random.default_rng(95)
    t = np.sort(rng.choice(wl.n, size=4096, replace=False))
    check_census(cnt, chk, t, h["x"][t], h["x"], h["id"], wl.params["h"], prec, "column sample")
