"""Run-time guards of the device path, through the C ABI.

* The update's diagnostics count the particles whose stored fields are not
  finite (slot 7), so a blow-up is seen without reading the state back: zero
  over a clean run, and at least the seeded particle after a NaN velocity.
* Checkpoint and resume: a run saved after k steps, loaded into a fresh
  simulation and continued, ends bit for bit where the uninterrupted run ends
  (the library keeps no state between calls besides the caller's buffers).
"""
import numpy as np
import pytest
import torch

import sph_synth as S

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
PRECS = [pytest.param(FP64, id="fp64"), pytest.param(FP32, id="fp32split")]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", PRECS)
def test_non_finite_count(prec):
    from paper_2310_03596_amd.sim import Sim
    wl = S.c1_cube(n_side=10)
    sim = Sim(wl, prec)
    for _ in range(5):
        sim.step()
        assert sim.diagnostics()[7] == 0
    bad = S.c1_cube(n_side=10)
    bad.v[17, 1] = np.nan
    bad.E[17] = np.nan
    sim = Sim(bad, prec)
    assert sim.diagnostics()[7] == 1          # the initial EOS stage sees the one particle
    sim.step()
    d = sim.diagnostics()
    print("non-finite particles after one step:", d[7])
    assert d[7] >= 1 and np.isfinite(d[0])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["column", "solid"])
def test_resume_is_bitwise(case, prec, tmp_path):
    from paper_2310_03596_amd.sim import Sim
    if case == "column":
        wl = S.c2_column(nx=10, ny=8, nz=20, dx=5.4e-3, box=(0.1, 0.05, 0.12))
    else:
        wl = S.solid_block(8, seed=63, vz=-50.0, s_sigma=1e7)
    whole = Sim(wl, prec)
    whole.run(12)
    first = Sim(wl, prec)
    first.run(5)
    path = str(tmp_path / "ckpt.npz")
    first.save(path)
    del first
    resumed = Sim(wl, prec)
    resumed.load(path)
    resumed.run(7)
    torch.cuda.synchronize()
    a, b = whole.A.host(), resumed.A.host()
    for f in a:
        assert np.array_equal(a[f], b[f], equal_nan=False), f
    assert np.array_equal(whole.diagnostics(), resumed.diagnostics())
    assert resumed.steps_done == 12
