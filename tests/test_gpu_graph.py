"""A captured step loop (paper_2310_03596_amd.graph.StepGraph) replays the
library's steps bit for bit: every replay is checked against the same steps
run eagerly on a second simulation, with eager work and synchronisations
between the replays (fluid cube with box walls and a dt that changes every
step; a solid block with its two interaction loops)."""
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
@pytest.mark.parametrize("case", ["cube", "solid"])
def test_step_graph_replays_match_eager_steps(case, prec):
    from paper_2310_03596_amd.graph import StepGraph
    from paper_2310_03596_amd.sim import Sim
    wl = S.c1_cube() if case == "cube" else S.solid_block(8, seed=64, s_sigma=1e7)
    eager, cap = Sim(wl, prec), Sim(wl, prec)
    g = StepGraph(cap, steps=4)
    for rep in range(3):
        eager.run(4)
        g.replay()
        torch.cuda.synchronize()
        a, b = eager.A.host(), cap.A.host()
        for f in a:
            assert np.array_equal(a[f], b[f]), (rep, f)
        assert np.array_equal(eager.diagnostics(), cap.diagnostics()), rep
        assert cap.steps_done == eager.steps_done == 4 * (rep + 1)


def test_step_graph_needs_an_even_count():
    from paper_2310_03596_amd.graph import StepGraph
    from paper_2310_03596_amd.sim import Sim
    sim = Sim(S.c1_cube(n_side=6), FP32)
    with pytest.raises(ValueError):
        StepGraph(sim, steps=3)
