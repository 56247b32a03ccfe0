"""The measurement hook (sph_set_pair_events): the events the library records
around the pair kernel of a FORCE call bracket that kernel inside the call,
so the interval they give is positive and shorter than the whole call's
(which also stages the source records), and turning the hook off leaves
caller-recorded events alone."""
import pytest
import torch

import sph_synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_03596_amd import _lib
    _lib.load()


def test_pair_events_bracket_the_pair_kernel_inside_the_call():
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.sim import Sim
    print("[pair events] lattice 24^3, FP32 split", flush=True)
    sim = Sim(S.jittered_lattice(24, seed=64, rho_sigma=0.01), 1)
    sim.build()
    outer = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    inner = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for ev in inner:
        ev.record()   # created by torch, recorded again by the library below
    torch.cuda.synchronize()
    for _ in range(3):
        outer[0].record()
        assert L.sph_set_pair_events(inner[0].cuda_event, inner[1].cuda_event) == 0
        sim.interact()
        assert L.sph_set_pair_events(None, None) == 0
        outer[1].record()
        torch.cuda.synchronize()
        whole, kernel = outer[0].elapsed_time(outer[1]), inner[0].elapsed_time(inner[1])
        print(f"  call {whole:.4f} ms, pair kernel {kernel:.4f} ms", flush=True)
        assert 0.0 < kernel < whole
    # off: a later call does not touch the events
    sim.interact()
    torch.cuda.synchronize()
    assert inner[0].elapsed_time(inner[1]) == pytest.approx(kernel)
