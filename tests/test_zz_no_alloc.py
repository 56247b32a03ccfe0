"""sph_mark_boundary_noalloc (step c with no workspace argument, for callers
that cannot allocate) against sph_mark_boundary through the C ABI: two calls
in a row on one GPU, the second on a smaller share with a boundary capacity
below its count; communication hashes, boundary lists and counts bit-exact."""
import numpy as np
import pytest
import torch

import sph_synth as S

pytestmark = pytest.mark.gpu

FP32 = 1


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_noalloc_mark_equals_workspace_mark():
    from paper_2310_03596_amd import _lib as L
    from paper_2310_03596_amd.sim import SharePass
    from paper_2310_03596_amd.state import cells_struct, stream_handle
    shares = [("mixed", dict(seed=75, nx=40, ny=18, nz=16, split_ix=30), None),
              ("slab", dict(seed=76, nx=30, ny=12, nz=12, split_ix=24), 0.5)]
    sizes = []
    for layout, kw, cap_frac in shares:
        loc, rem = S.c4_share(layout, **kw)
        print(f"[noalloc] layout={layout} local={loc.n} remote={rem.n}", flush=True)
        sp = SharePass(loc, rem, FP32)
        sp.build()
        sp.mark()
        torch.cuda.synchronize()
        nb_ref = int(sp.nb.cpu()[0])
        comm_ref = sp.comm.cpu().numpy().view(np.uint32).copy()
        bidx_ref = sp.bidx.cpu().numpy().view(np.uint32)[:nb_ref].copy()
        assert nb_ref > 0
        cap = sp.nl if cap_frac is None else int(nb_ref * cap_frac)
        comm = torch.full((sp.nl,), -5, dtype=torch.int32, device="cuda")
        bidx = torch.full((sp.nl,), -5, dtype=torch.int32, device="cuda")
        nb = torch.full((1,), -5, dtype=torch.int32, device="cuda")
        nflag = torch.full((1,), -5, dtype=torch.int32, device="cuda")
        L.sph_mark_boundary_noalloc(sp.grid, sp.LB.struct(), cells_struct(sp.rstart, sp.nc), comm.data_ptr(),
                                    bidx.data_ptr(), cap, nb.data_ptr(), nflag.data_ptr(), stream_handle())
        torch.cuda.synchronize()
        assert int(nflag.cpu()[0]) == nb_ref            # the true count, also past the capacity
        assert int(nb.cpu()[0]) == min(cap, nb_ref)     # the entries written
        assert np.array_equal(comm.cpu().numpy().view(np.uint32), comm_ref)
        got = bidx.cpu().numpy()
        k = min(cap, nb_ref)
        assert np.array_equal(got[:k].view(np.uint32), bidx_ref[:k])
        assert np.all(got[k:] == -5)                    # nothing written past min(count, capacity)
        sizes.append(loc.n)
        del sp
    assert sizes[1] < sizes[0]
