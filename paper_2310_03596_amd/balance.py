"""One round of the particle-swapping heuristic between two GPUs' particle
sets (Section III.A; per particle type with biased centres, Section III.B),
held as two arrays on one device.

Every step runs in libsph; this module only owns the buffers and sequences
the calls: both centres of gravity, both balancing hashes (each towards the
other's centre) with their positive counts, both selections of
k = min(n+_A, n+_B) particles, and the pairwise swap.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .state import Particles, grid_struct, stream_handle

HMAX = 1000   # maximum swapping hash (the paper: "typically 1000")
ALPHA = 0.1   # bias of a type's centre towards the centre of all types (Section III.B)


class BalancePair:
    """Two particle sets A and B (e.g. the shares of two GPUs) on one device."""

    def __init__(self, wl_a, wl_b, prec: int, device="cuda", hmax: int = HMAX):
        self._setup(Particles.upload(wl_a, prec, device), Particles.upload(wl_b, prec, device), wl_a.grid,
                    prec, device, hmax)

    @classmethod
    def of(cls, A: Particles, B: Particles, grid: dict, prec: int, hmax: int = HMAX) -> "BalancePair":
        """A pair over two existing particle arrays (swaps happen in place)."""
        self = cls.__new__(cls)
        self._setup(A, B, grid, prec, A.device, hmax)
        return self

    def _setup(self, A, B, grid, prec, device, hmax):
        self.prec, self.hmax = prec, hmax
        self.A, self.B = A, B
        n = max(self.A.n, self.B.n, 1)
        self.ws_bytes = L.sph_workspace_size(grid_struct(grid), n, prec,
                                             L.SPH_SOLID_J2 if A.solid else L.SPH_FLUID_TAIT)
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.cg = torch.zeros((2, 4), dtype=torch.float64, device=device)
        self.bh = [torch.zeros(max(self.A.n, 1), **i32), torch.zeros(max(self.B.n, 1), **i32)]
        self.sel = [torch.zeros(max(self.A.n, 1), **i32), torch.zeros(max(self.B.n, 1), **i32)]
        self.npos = torch.zeros(2, **i32)
        self.k = torch.zeros(2, **i32)

    def centroids(self):
        st = stream_handle()
        for q, p in enumerate((self.A, self.B)):
            L.sph_centroid(p.struct(), self.cg[q].data_ptr(), self.ws.data_ptr(), self.ws_bytes, st)

    def hashes(self):
        st = stream_handle()
        for q, p in enumerate((self.A, self.B)):
            L.sph_balance_hash(p.struct(), self.cg[q].data_ptr(), self.cg[1 - q].data_ptr(), self.hmax,
                               self.bh[q].data_ptr(), self.npos[q:q + 1].data_ptr(), self.ws.data_ptr(),
                               self.ws_bytes, st)

    def selections(self):
        st = stream_handle()
        for q, p in enumerate((self.A, self.B)):
            L.sph_balance_select(p.n, self.bh[q].data_ptr(), self.hmax, self.npos[q:q + 1].data_ptr(),
                                 self.npos[1 - q:2 - q].data_ptr(), self.sel[q].data_ptr(),
                                 self.k[q:q + 1].data_ptr(), self.ws.data_ptr(), self.ws_bytes, st)

    def swap(self):
        L.sph_swap(self.A.struct(), self.sel[0].data_ptr(), self.B.struct(), self.sel[1].data_ptr(),
                   self.k[0:1].data_ptr(), min(self.A.n, self.B.n), stream_handle())

    def round(self):
        """Enqueue one full round; returns nothing (k stays on the device)."""
        self.centroids()
        self.hashes()
        self.selections()
        self.swap()


class BalanceTypesPair(BalancePair):
    """Two particle sets with a type label per particle (u8, below ntypes):
    every type is balanced on its own towards biased centres
    Cg'_t = alpha Cg_all + (1 - alpha) Cg_t (Section III.B).  Pairs exchange
    particles of one type, so the labels stay where they are."""

    def __init__(self, wl_a, wl_b, types_a, types_b, ntypes: int, prec: int, device="cuda", hmax: int = HMAX,
                 alpha: float = ALPHA):
        super().__init__(wl_a, wl_b, prec, device, hmax)
        self.ntypes, self.alpha = ntypes, alpha
        u8 = dict(dtype=torch.uint8, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.types = []
        for t, p in ((types_a, self.A), (types_b, self.B)):
            buf = torch.zeros(max(p.n, 1), **u8)
            buf[:p.n] = torch.as_tensor(t, dtype=torch.uint8)
            self.types.append(buf)
        self.cg = torch.zeros((2, ntypes + 1, 4), dtype=torch.float64, device=device)
        self.npos = torch.zeros((2, ntypes), **i32)
        self.k = torch.zeros((2, ntypes), **i32)
        self.off = torch.zeros((2, ntypes + 1), **i32)

    def centroids(self):
        st = stream_handle()
        for q, p in enumerate((self.A, self.B)):
            L.sph_centroid_types(p.struct(), self.types[q].data_ptr(), self.ntypes, self.alpha,
                                 self.cg[q].data_ptr(), self.ws.data_ptr(), self.ws_bytes, st)

    def hashes(self):
        st = stream_handle()
        for q, p in enumerate((self.A, self.B)):
            L.sph_balance_hash_types(p.struct(), self.types[q].data_ptr(), self.ntypes, self.cg[q].data_ptr(),
                                     self.cg[1 - q].data_ptr(), self.hmax, self.bh[q].data_ptr(),
                                     self.npos[q].data_ptr(), self.ws.data_ptr(), self.ws_bytes, st)

    def selections(self):
        st = stream_handle()
        for q, p in enumerate((self.A, self.B)):
            L.sph_balance_select_types(p.n, self.types[q].data_ptr(), self.ntypes, self.bh[q].data_ptr(),
                                       self.hmax, self.npos[q].data_ptr(), self.npos[1 - q].data_ptr(),
                                       self.sel[q].data_ptr(), self.k[q].data_ptr(), self.off[q].data_ptr(),
                                       self.ws.data_ptr(), self.ws_bytes, st)

    def swap(self):
        L.sph_swap(self.A.struct(), self.sel[0].data_ptr(), self.B.struct(), self.sel[1].data_ptr(),
                   self.off[0][self.ntypes:].data_ptr(), min(self.A.n, self.B.n), stream_handle())
