"""GPU parity of the hypervelocity-impact workload (Section IV.A): a J2
solid in the perfectly plastic limit with the Mie-Gruneisen EOS and spall
cut-off, through the C ABI.

* Small case (plate 6 x 6 x 2 mm, bead of 912 particles, 250 um lattice):
  every step against the oracle run one step from the GPU's own state with
  the GPU's dt, per field within the tolerances of the other step tests.
* Full size (6.67 M particles, the paper's count): after three steps, the
  EOS on a sample of particles and the FORCE pass on a sample of targets,
  from the device state.
"""
import numpy as np
import pytest
import torch

import sph_synth as S
from oracle import cpu
from tests.gpu_helpers import assert_within, oracle_state, rate_bound
from tests.test_gpu_parity import TOL_STEP, _step_vs_oracle

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_hvi_steps_match_oracle_each_step(prec):
    wl = S.c6_hvi(dx=2.5e-4, plate_half=3e-3)
    print(f"[hvi small] n={wl.n} prec={prec}", flush=True)
    worst = _step_vs_oracle(wl, prec, 6, TOL_STEP[prec])
    print("hvi worst per-field error:", worst)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [FP32, FP64])
def test_hvi_full_size_sampled(prec):
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.sim import Sim
    wl = S.c6_hvi()
    print(f"[hvi full] n={wl.n} prec={prec}", flush=True)
    sim = Sim(wl, prec)
    for _ in range(3):
        sim.step()
    sim.build()
    torch.cuda.synchronize()
    h = sim.A.host()
    rng = np.random.default_rng(97)
    # the impact zone (bead and the plate under it) and uniform picks
    bead = h["id"] >= wl.n - int(wl.extra["types"].sum())     # the bead's ids come last
    centre = h["x"][bead].mean(0)
    near = np.flatnonzero(np.linalg.norm(h["x"] - centre, axis=1) < 2e-3)
    tidx = np.unique(np.concatenate([rng.choice(near, size=min(1024, near.size), replace=False),
                                     rng.choice(wl.n, size=1024, replace=False)])).astype(np.uint32)
    # EOS from the stored state
    pe, ce = np.empty(tidx.size), np.empty(tidx.size)
    for k, i in enumerate(tidx):
        pe[k], ce[k] = cpu.eos(wl.params, h["m"][i] / h["w"][i], h["e"][i])
    ps = wl.params["rho0"] * wl.params["c0"] ** 2
    tol = 2e-6 if prec == FP32 else 1e-12
    assert np.abs(h["p"][tidx] - pe).max() <= tol * ps
    assert np.abs(h["c"][tidx] - ce).max() <= tol * ce.max()
    assert (h["p"][tidx] >= wl.params["p_cut"]).all()
    assert np.abs(h["p"][near]).max() > 1e8      # the shock has formed
    # FORCE pass on the sample
    sim.interact()
    torch.cuda.synchronize()
    st = oracle_state(sim.A.host(), True)
    start = cpu.cell_start(st.hash, cpu.ncells(wl.grid))
    ref = cpu.interact(wl.params, wl.grid, cpu.FORCE, st, st, start, True, tidx=tidx)[tidx]
    b = rate_bound(wl.params, wl.grid, cpu.FORCE, st, st, start, True, prec, tidx=tidx)[tidx]
    assert_within(sim.rates.force().T.cpu().numpy()[tidx], ref, b, "hvi FORCE (sample)")
    assert L.SPH_EOS_MIE_GRUNEISEN == wl.params["eos"]
