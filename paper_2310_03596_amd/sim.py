"""Step driver: sequences the libsph calls of one GPU's share of a step.

Fluid step (Section II, steps a, e, g): build_cells -> FORCE pass -> MOTION.
Solid step (two interaction loops per iteration, Section II note):
build_cells -> GRADIENT pass -> STRESS stage -> FORCE pass -> MOTION.
Share step (steps a, c, d packing, e, f): see ``SharePass``.
All work is enqueued on the current stream; dt, boundary counts and
diagnostics stay on the device.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .state import Particles, Rates, cells_struct, grid_struct, ncells, params_struct, stream_handle


class Sim:
    def __init__(self, wl, prec: int, device="cuda", fixed_dt: float | None = None):
        self.wl = wl
        self.prec = prec
        self.solid = wl.S is not None
        self.grid = grid_struct(wl.grid)
        self.params = params_struct(wl.params, prec)
        self.nc = ncells(wl.grid)
        self.n = wl.n
        self.A = Particles.upload(wl, prec, device)
        self.B = Particles(self.n, prec, self.solid, device)
        self.perm = torch.zeros(self.n, dtype=torch.int32, device=device)
        self.start = torch.zeros(self.nc + 1, dtype=torch.int32, device=device)
        self.ws_bytes = L.sph_workspace_size(self.grid, self.n, prec, int(wl.params["material"]))
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=device)
        self.rates = Rates(self.n, prec, self.solid, device)
        self.diag = torch.zeros((2, 8), dtype=torch.float64, device=device)
        self.cur = 0
        self.fixed = None
        if fixed_dt is not None:
            self.fixed = torch.full((1,), float(fixed_dt), dtype=torch.float64, device=device)
        self.steps_done = 0
        s = self.A.struct()
        L.sph_integrate(self.params, L.SPH_STAGE_EOS, s, None, None, self.diag[0].data_ptr(),
                        self.ws.data_ptr(), self.ws_bytes, stream_handle())

    @property
    def cells(self):
        return cells_struct(self.start, self.nc)

    def build(self):
        """Step a + bucket sort: A (any order) -> B (hash order), then swap."""
        a, b = self.A.struct(), self.B.struct()
        L.sph_build_cells(self.grid, a, b, self.perm.data_ptr(), self.cells, self.ws.data_ptr(), self.ws_bytes,
                          stream_handle())
        self.A, self.B = self.B, self.A

    def interact(self, pass_=L.SPH_PASS_FORCE):
        a = self.A.struct()
        r = self.rates.struct()
        L.sph_interact(self.params, self.grid, pass_, a, None, None, a, self.cells, 1, r, self.ws.data_ptr(),
                       self.ws_bytes, stream_handle())

    def dt_ptr(self, dt_ptr=None):
        if dt_ptr is not None:
            return dt_ptr
        if self.fixed is not None:
            return self.fixed.data_ptr()
        return self.diag[self.cur].data_ptr()    # [0] = next dt of the previous update

    def step(self, dt_ptr=None, force_events=None):
        """One whole step.  force_events: optional (start, end) torch CUDA
        events (timing enabled) that the FORCE call records around its pair
        kernel alone (sph_set_pair_events)."""
        dtp = self.dt_ptr(dt_ptr)
        self.build()
        a = self.A.struct()
        r = self.rates.struct()
        st = stream_handle()
        if self.solid:
            L.sph_interact(self.params, self.grid, L.SPH_PASS_GRADIENT, a, None, None, a, self.cells, 1, r,
                           self.ws.data_ptr(), self.ws_bytes, st)
            L.sph_integrate(self.params, L.SPH_STAGE_STRESS, a, r, dtp, None, None, 0, st)
        if force_events is not None:
            for ev in force_events:
                if not ev.cuda_event:   # torch creates an event at its first record
                    ev.record()
            L.sph_set_pair_events(force_events[0].cuda_event, force_events[1].cuda_event)
        L.sph_interact(self.params, self.grid, L.SPH_PASS_FORCE, a, None, None, a, self.cells, 1, r,
                       self.ws.data_ptr(), self.ws_bytes, st)
        if force_events is not None:
            L.sph_set_pair_events(None, None)
        nxt = 1 - self.cur
        L.sph_integrate(self.params, L.SPH_STAGE_MOTION, a, r, dtp, self.diag[nxt].data_ptr(), self.ws.data_ptr(),
                        self.ws_bytes, st)
        self.cur = nxt
        self.steps_done += 1

    def run(self, nsteps: int, dts: np.ndarray | None = None):
        """nsteps steps; dts (optional) replays a given dt schedule."""
        dts_dev = None
        if dts is not None:
            dts_dev = torch.as_tensor(np.asarray(dts, dtype=np.float64), device=self.A.x.device)
        for k in range(nsteps):
            self.step(None if dts_dev is None else dts_dev[k].data_ptr())
        return dts_dev

    def count_pairs(self) -> tuple[int, int]:
        """(candidates, pairs within 2h) of the FORCE pass on the current state."""
        c = torch.zeros(2, dtype=torch.int64, device=self.A.x.device)
        a = self.A.struct()
        L.sph_count_pairs(self.params, self.grid, a, None, None, a, self.cells, c.data_ptr(), stream_handle())
        torch.cuda.synchronize()
        v = c.cpu().numpy()
        return int(v[0]), int(v[1])

    def census(self, pass_=L.SPH_PASS_FORCE) -> tuple[np.ndarray, np.ndarray]:
        """Per particle of the current (sorted) state: number of sources the
        pass evaluates and the mixed-id checksum of their ids."""
        dev = self.A.x.device
        cnt = torch.zeros(self.n, dtype=torch.int32, device=dev)
        chk = torch.zeros(self.n, dtype=torch.int64, device=dev)
        a = self.A.struct()
        L.sph_neighbor_census(self.params, self.grid, pass_, a, None, None, a, self.cells, cnt.data_ptr(),
                              chk.data_ptr(), self.ws.data_ptr(), self.ws_bytes, stream_handle())
        torch.cuda.synchronize()
        return cnt.cpu().numpy().view(np.uint32), chk.cpu().numpy().view(np.uint64)

    def diagnostics(self) -> np.ndarray:
        """[next dt, M, Px, Py, Pz, sum m E, kinetic energy, non-finite count]."""
        return self.diag[self.cur, :8].cpu().numpy()

    def save(self, path: str):
        """Checkpoint: the particle state in its current array order (one
        device-to-host copy of the state's single allocation), the
        diagnostics record that holds the next dt, and the step count."""
        torch.cuda.synchronize()
        np.savez(path, state=self.A._buf.cpu().numpy(), diag=self.diag[self.cur].cpu().numpy(),
                 steps=np.array([self.steps_done], dtype=np.int64),
                 shape=np.array([self.n, self.prec, int(self.solid)], dtype=np.int64))

    def load(self, path: str):
        """Resume from a checkpoint of a Sim of the same workload and form:
        the next steps are those the saved run would have taken, bit for bit."""
        with np.load(path, allow_pickle=False) as z:
            shape = z["shape"].tolist()
            if shape != [self.n, self.prec, int(self.solid)]:
                raise ValueError(f"checkpoint of (n, prec, solid) = {shape}, this run has "
                                 f"{[self.n, self.prec, int(self.solid)]}")
            self.A._buf.copy_(torch.from_numpy(z["state"]))
            self.diag[self.cur].copy_(torch.from_numpy(z["diag"]))
            self.steps_done = int(z["steps"][0])
        torch.cuda.synchronize()

    def state_by_id(self) -> dict:
        h = self.A.host()
        order = np.argsort(h["id"], kind="stable")
        return {k: v[order] for k, v in h.items()}


class SharePass:
    """One GPU's share of a particle-decomposition pass set (Section II a-f).

    Local and remote particles are kept in separate arrays on the same grid.
    ``run()`` enqueues: build_cells on both arrays (step a and the one-GPU
    stand-in for receiving hashes, step b), communication hash and boundary
    compaction (step c), packing of the boundary payload (step d), the
    local-local FORCE pass (step e) and the local-remote FORCE pass over the
    boundary list only (step f).
    """

    def __init__(self, local_wl, remote_wl, prec: int, device="cuda"):
        self.prec = prec
        self.grid = grid_struct(local_wl.grid)
        self.params = params_struct(local_wl.params, prec)
        self.nc = ncells(local_wl.grid)
        self.nl, self.nr = local_wl.n, remote_wl.n
        self.LA = Particles.upload(local_wl, prec, device)
        self.LB = Particles(self.nl, prec, False, device)
        self.RA = Particles.upload(remote_wl, prec, device)
        self.RB = Particles(self.nr, prec, False, device)
        self.lperm = torch.zeros(self.nl, dtype=torch.int32, device=device)
        self.rperm = torch.zeros(self.nr, dtype=torch.int32, device=device)
        self.lstart = torch.zeros(self.nc + 1, dtype=torch.int32, device=device)
        self.rstart = torch.zeros(self.nc + 1, dtype=torch.int32, device=device)
        nmax = max(self.nl, self.nr)
        self.ws_bytes = L.sph_workspace_size(self.grid, nmax, prec, L.SPH_FLUID_TAIT)
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=device)
        self.comm = torch.zeros(self.nl, dtype=torch.int32, device=device)
        self.bidx = torch.zeros(self.nl, dtype=torch.int32, device=device)
        self.nb = torch.zeros(1, dtype=torch.int32, device=device)
        self.payload = Particles(self.nl, prec, False, device)
        self.rates = Rates(self.nl, prec, False, device)
        self.diag = torch.zeros(8, dtype=torch.float64, device=device)
        st = stream_handle()
        for P in (self.LA, self.RA):
            L.sph_integrate(self.params, L.SPH_STAGE_EOS, P.struct(), None, None, self.diag.data_ptr(),
                            self.ws.data_ptr(), self.ws_bytes, st)

    def build(self):
        st = stream_handle()
        L.sph_build_cells(self.grid, self.LA.struct(), self.LB.struct(), self.lperm.data_ptr(),
                          cells_struct(self.lstart, self.nc), self.ws.data_ptr(), self.ws_bytes, st)
        L.sph_build_cells(self.grid, self.RA.struct(), self.RB.struct(), self.rperm.data_ptr(),
                          cells_struct(self.rstart, self.nc), self.ws.data_ptr(), self.ws_bytes, st)

    def resort(self):
        """Step a on arrays that are already sorted, as at every step of a run
        (the particles arrive in the order the previous sort left them):
        sorts LB into LA and RB into RA, then swaps the roles, so LB and RB
        hold the result as after build()."""
        st = stream_handle()
        L.sph_build_cells(self.grid, self.LB.struct(), self.LA.struct(), self.lperm.data_ptr(),
                          cells_struct(self.lstart, self.nc), self.ws.data_ptr(), self.ws_bytes, st)
        L.sph_build_cells(self.grid, self.RB.struct(), self.RA.struct(), self.rperm.data_ptr(),
                          cells_struct(self.rstart, self.nc), self.ws.data_ptr(), self.ws_bytes, st)
        self.LA, self.LB = self.LB, self.LA
        self.RA, self.RB = self.RB, self.RA

    def mark(self):
        L.sph_mark_boundary(self.grid, self.LB.struct(), cells_struct(self.rstart, self.nc), self.comm.data_ptr(),
                            self.bidx.data_ptr(), self.nl, self.nb.data_ptr(), None, self.ws.data_ptr(),
                            self.ws_bytes, stream_handle())

    def pack(self):
        L.sph_pack_boundary(self.LB.struct(), self.bidx.data_ptr(), self.nb.data_ptr(), self.payload.struct(),
                            stream_handle())

    def interact_local(self):
        a = self.LB.struct()
        L.sph_interact(self.params, self.grid, L.SPH_PASS_FORCE, a, None, None, a,
                       cells_struct(self.lstart, self.nc), 1, self.rates.struct(), self.ws.data_ptr(),
                       self.ws_bytes, stream_handle())

    def interact_remote(self):
        L.sph_interact(self.params, self.grid, L.SPH_PASS_FORCE, self.LB.struct(), self.bidx.data_ptr(),
                       self.nb.data_ptr(), self.RB.struct(), cells_struct(self.rstart, self.nc), 0,
                       self.rates.struct(), self.ws.data_ptr(), self.ws_bytes, stream_handle())

    def census(self) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        """Neighbour census of the local-local pass (every local particle) and
        of the local-remote pass (boundary list): counts and checksums, each
        indexed like the sorted local array (entries of the local-remote
        census outside the list stay 0)."""
        dev = self.LB.x.device
        out = []
        for remote in (False, True):
            cnt = torch.zeros(self.nl, dtype=torch.int32, device=dev)
            chk = torch.zeros(self.nl, dtype=torch.int64, device=dev)
            src = self.RB if remote else self.LB
            start = self.rstart if remote else self.lstart
            L.sph_neighbor_census(self.params, self.grid, L.SPH_PASS_FORCE, self.LB.struct(),
                                  self.bidx.data_ptr() if remote else None, self.nb.data_ptr() if remote else None,
                                  src.struct(), cells_struct(start, self.nc), cnt.data_ptr(), chk.data_ptr(),
                                  self.ws.data_ptr(), self.ws_bytes, stream_handle())
            out += [cnt, chk]
        torch.cuda.synchronize()
        return (out[0].cpu().numpy().view(np.uint32), out[1].cpu().numpy().view(np.uint64),
                out[2].cpu().numpy().view(np.uint32), out[3].cpu().numpy().view(np.uint64))

    def run(self):
        self.build()
        self.mark()
        self.pack()
        self.interact_local()
        self.interact_remote()
