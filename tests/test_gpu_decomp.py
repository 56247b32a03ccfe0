"""Two particle sets stepping as two GPUs' shares of one decomposition
(Section II a-g) with swaps of the balancing heuristic in between (Section
III.A), on one device, through the C ABI.

* The split changes no physics: two sets with local-local plus
  local-remote passes, balanced every few steps, end where one set holding
  every particle ends, particle by particle (matched by id), within the
  one-step tolerances (the pair sums only add in another order).
* Balancing shrinks the exchange set of a random split of the column
  workload (the behaviour of the paper's Fig. 2), and keeps a slab split's
  from growing.
"""
import numpy as np
import pytest
import torch

import sph_synth as S
from paper_2310_03596_amd import SPH_FP32_SPLIT, SPH_FP64
from paper_2310_03596_amd.decomp import TwoSets
from paper_2310_03596_amd.sim import Sim

pytestmark = pytest.mark.gpu

TOL = {SPH_FP64: 1e-12, SPH_FP32_SPLIT: 2e-5}


def _by_id(h):
    order = np.argsort(h["id"], kind="stable")
    return {f: v[order] for f, v in h.items()}


@pytest.mark.parametrize("prec", [SPH_FP64, SPH_FP32_SPLIT])
def test_two_sets_match_one_set(prec):
    wl = S.jittered_lattice(16, seed=90, rho_sigma=0.01, walls=True)
    owner = np.random.default_rng(91).random(wl.n) < 0.5
    one = Sim(wl, prec)
    torch.cuda.synchronize()
    dt = 0.5 * float(one.diag[one.cur, 0].cpu())
    one.fixed = torch.full((1,), dt, dtype=torch.float64, device=one.ws.device)
    two = TwoSets(wl, owner, prec, fixed_dt=dt, period=3)
    print(f"[decomp] prec={prec} n={wl.n} sets={two.sides[0].n}+{two.sides[1].n} dt={dt:.3e}", flush=True)
    for _ in range(8):
        one.step()
        two.step()
    torch.cuda.synchronize()
    a, b = _by_id(one.A.host()), two.host()
    assert np.array_equal(a["id"], b["id"])
    assert two.sides[0].n + two.sides[1].n == wl.n
    for f in ("x", "v", "m", "w", "rho", "p", "E"):
        ref = np.asarray(a[f], dtype=np.float64)
        err = np.abs(np.asarray(b[f], dtype=np.float64) - ref).max() / np.abs(ref).max()
        assert err <= TOL[prec], (f, err)


def test_balancing_shrinks_the_exchange_set():
    wl = S.c2_column()
    rng = np.random.default_rng(92)
    mixed = TwoSets(wl, rng.random(wl.n) < 0.5, SPH_FP32_SPLIT, period=1)
    mixed.step()
    f0 = mixed.exchange_fraction()
    for _ in range(30):
        mixed.step()
    f30 = mixed.exchange_fraction()
    slab = TwoSets(wl, wl.x[:, 0] > np.median(wl.x[:, 0]), SPH_FP32_SPLIT, period=1)
    fs = []
    for _ in range(10):
        slab.step()
        fs.append(slab.exchange_fraction())
    print(f"[decomp] mixed: {f0:.3f} -> {f30:.3f} after 30 rounds; slab: {fs[0]:.4f} .. {max(fs):.4f}", flush=True)
    # a random split exchanges almost every particle; thirty rounds leave a
    # thin layer (5.4 % measured)
    assert f0 > 0.9
    assert f30 < 0.1
    # a slab split at the median x exchanges the particles of about three
    # bucket columns of the 28 across the column (10.8 % measured), and
    # balancing does not let that grow
    assert fs[0] < 0.15 and max(fs) <= 1.05 * fs[0]
