"""Two particle sets on one device stepping as the shares of two GPUs in the
particle decomposition of Section II, with the swapping heuristic of
Section III.A every `period` steps (the paper balances every 20 integration
loops).

A step, for each set X with the other set Y:
  a  hash, sort and bucket table of X (`sph_build_cells`);
  b  Y's bucket table stands in for the hashes the other GPU would send;
  c  communication hash of X against Y's table and compaction of X's
     boundary list (`sph_mark_boundary`);
  d  on two GPUs the boundary payload would travel here; on one device the
     local-remote pass reads Y's sorted array directly;
  e  local-local FORCE pass over X;
  f  local-remote FORCE pass of X's boundary particles against Y,
     continuing the sums of e;
  g  explicit update of X.
The time step is fixed, or the smaller of the two sets' next dt (the
all-reduce a multi-GPU run makes).  Every step of the path runs in libsph;
this module only owns buffers and sequences calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .balance import HMAX, BalancePair
from .sim import Sim
from .state import stream_handle


def split_workload(wl, owner: np.ndarray):
    """The two sub-workloads of wl: particles with owner False, then True."""
    owner = np.asarray(owner, dtype=bool)
    return wl.subset(~owner), wl.subset(owner)


class TwoSets:
    """Sets A and B (two GPUs' shares of one fluid workload) on one device."""

    def __init__(self, wl, owner: np.ndarray, prec: int, device="cuda", fixed_dt: float | None = None,
                 period: int = 20, hmax: int = HMAX):
        wa, wb = split_workload(wl, owner)
        self.sides = [Sim(wa, prec, device, fixed_dt=fixed_dt), Sim(wb, prec, device, fixed_dt=fixed_dt)]
        self.prec, self.period, self.hmax, self.grid_dict = prec, period, hmax, wl.grid
        self.n = wl.n
        s0 = self.sides[0]
        self.params, self.grid, self.nc = s0.params, s0.grid, s0.nc
        # one workspace for every call (sized for the larger set: a local-remote
        # pass stages the other set's particles)
        nmax = max(wa.n, wb.n, 1)
        self.ws_bytes = L.sph_workspace_size(self.grid, nmax, prec, L.SPH_FLUID_TAIT)
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.comm = [torch.zeros(max(s.n, 1), **i32) for s in self.sides]
        self.bidx = [torch.zeros(max(s.n, 1), **i32) for s in self.sides]
        self.nb = torch.zeros(2, **i32)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.steps_done = 0

    def _dt_ptr(self):
        a, b = self.sides
        if a.fixed is not None:
            return a.fixed.data_ptr()
        # the smaller of the two sets' next dt (on two GPUs: an all-reduce)
        torch.minimum(a.diag[a.cur, 0:1], b.diag[b.cur, 0:1], out=self.dt)
        return self.dt.data_ptr()

    def step(self):
        dtp = self._dt_ptr()
        self.rates_pass()
        self.update(dtp)
        self.steps_done += 1
        if self.period and self.steps_done % self.period == 0:
            self.balance()

    def rates_pass(self):
        """Steps a-f for both sets: sort and table, marking, local-local and
        local-remote FORCE passes (the sorted states and rates stay in the
        sets until update)."""
        st = stream_handle()
        for s in self.sides:
            s.build()
        ws, wsb = self.ws.data_ptr(), self.ws_bytes
        for q, (X, Y) in enumerate(self.pairs()):
            L.sph_mark_boundary(self.grid, X.A.struct(), Y.cells, self.comm[q].data_ptr(), self.bidx[q].data_ptr(),
                                X.n, self.nb[q:q + 1].data_ptr(), None, ws, wsb, st)
        for q, (X, Y) in enumerate(self.pairs()):
            a, r = X.A.struct(), X.rates.struct()
            L.sph_interact(self.params, self.grid, L.SPH_PASS_FORCE, a, None, None, a, X.cells, 1, r, ws, wsb, st)
            L.sph_interact(self.params, self.grid, L.SPH_PASS_FORCE, a, self.bidx[q].data_ptr(),
                           self.nb[q:q + 1].data_ptr(), Y.A.struct(), Y.cells, 0, r, ws, wsb, st)

    def update(self, dtp):
        """Step g for both sets with the time step at dtp (device)."""
        st = stream_handle()
        for X in self.sides:
            nxt = 1 - X.cur
            L.sph_integrate(self.params, L.SPH_STAGE_MOTION, X.A.struct(), X.rates.struct(), dtp,
                            X.diag[nxt].data_ptr(), self.ws.data_ptr(), self.ws_bytes, st)
            X.cur = nxt

    def pairs(self):
        """(own set, other set) for both sets."""
        return ((self.sides[0], self.sides[1]), (self.sides[1], self.sides[0]))

    def balance(self):
        """One round of the swapping heuristic between the two sets (in place)."""
        a, b = self.sides
        BalancePair.of(a.A, b.A, self.grid_dict, self.prec, self.hmax).round()

    def exchange_fraction(self) -> float:
        """Boundary particles of both sets (the exchange set of the last step) over all particles."""
        return float(self.nb.sum().cpu()) / self.n

    def host(self) -> dict:
        """Both sets' fields, concatenated and ordered by particle id."""
        hs = [s.A.host() for s in self.sides]
        out = {f: np.concatenate([h[f] for h in hs]) for f in hs[0]}
        order = np.argsort(out["id"], kind="stable")
        return {f: v[order] for f, v in out.items()}
