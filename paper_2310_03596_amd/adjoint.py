"""Checkpointed hand adjoint of a fluid rollout, behind torch.autograd.

Objectives, after `nsteps` fixed-dt steps of the fluid path (hash + sort +
FORCE pass + update; free boundaries, no gravity): the kinetic energy
J = sum m |v|^2 / 2, or the mean displacement along z of a tagged set of
particles (`tag_ids`), J = mean_{i in tag} (z_i(T) - z_i(0)).  Differentiable
inputs: the initial velocities (at fixed specific internal energy, so
E0 = e0 + |v0|^2 / 2) and the sound speed c0.  The objective's value and its
seed cotangent are the caller's side and use plain tensor operations; every
step of the path, forward and reverse, runs in libsph.

Forward keeps a copy of the whole particle state every `ckpt` steps.
Backward walks the segments in reverse: it restores a segment's checkpoint,
recomputes its steps (so the neighbour tables are rebuilt) keeping each
step's sorted state, permutation, bucket table and rates, then runs the
library's reverse kernels step by step.  Every step of the path, forward and
reverse, runs in libsph; this module only sequences calls and owns buffers.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import _lib as L
from .sim import Sim
from .state import Particles, Rates, cells_struct, real_dtype, stream_handle


class Cotangent:
    """Device buffers of a state cotangent (sph_adjoint), in the form's
    precision; with solid=True also of the deviatoric stress and the plastic
    strain."""

    def __init__(self, n: int, prec: int, device, solid: bool = False):
        real = real_dtype(prec)
        self.x = torch.zeros((3, n), dtype=real, device=device)
        self.v = torch.zeros((3, n), dtype=real, device=device)
        self.m, self.w, self.E, self.rho, self.p, self.c, self.e = [
            torch.zeros(n, dtype=real, device=device) for _ in range(7)]
        self.S = torch.zeros((6, n), dtype=real, device=device) if solid else None
        self.ep = torch.zeros(n, dtype=real, device=device) if solid else None

    def _solid_fields(self, a):
        if self.S is not None:
            for k in range(6):
                a.S[k] = self.S[k].data_ptr()
            a.eps_p = self.ep.data_ptr()

    def struct(self) -> L.SphAdjoint:
        a = L.SphAdjoint()
        for d in range(3):
            a.x[d] = self.x[d].data_ptr()
            a.v[d] = self.v[d].data_ptr()
        a.m, a.omega, a.E = self.m.data_ptr(), self.w.data_ptr(), self.E.data_ptr()
        a.rho, a.p, a.c, a.e = self.rho.data_ptr(), self.p.data_ptr(), self.c.data_ptr(), self.e.data_ptr()
        self._solid_fields(a)
        return a

    def state_struct(self) -> L.SphAdjoint:
        """Only the state fields (what a permutation carries)."""
        a = L.SphAdjoint()
        for d in range(3):
            a.x[d] = self.x[d].data_ptr()
            a.v[d] = self.v[d].data_ptr()
        a.m, a.omega, a.E = self.m.data_ptr(), self.w.data_ptr(), self.E.data_ptr()
        self._solid_fields(a)
        return a


class KineticEnergyRollout:
    """Forward rollout with checkpoints, and its reverse pass."""

    def __init__(self, wl, prec: int, nsteps: int, ckpt: int, dt: float, device="cuda", tag_ids=None):
        self.wl, self.prec, self.nsteps, self.ckpt, self.dt = wl, prec, nsteps, max(1, ckpt), dt
        self.device = device
        self.e0 = wl.E - 0.5 * np.einsum("ij,ij->i", wl.v, wl.v)   # specific internal energy, held fixed
        self.tag = None if tag_ids is None else np.unique(np.asarray(tag_ids, dtype=np.int64))

    def _workload(self, v0: np.ndarray, c0: float):
        w = copy.copy(self.wl)
        w.v = np.ascontiguousarray(v0, dtype=np.float64)
        w.E = self.e0 + 0.5 * np.einsum("ij,ij->i", w.v, w.v)
        w.params = dict(self.wl.params, c0=float(c0))
        return w

    def prepare(self, v0: np.ndarray, c0: float):
        """Uploads the initial state (and its EOS) to the device: the set-up
        that forward() does before the rollout."""
        self.sim = Sim(self._workload(v0, c0), self.prec, self.device, fixed_dt=self.dt)

    def forward(self, v0: np.ndarray, c0: float) -> float:
        self.prepare(v0, c0)
        return self.run()

    def run(self) -> float:
        """The rollout from the prepared state, with its checkpoints; J."""
        sim = self.sim
        self.ckpts = []
        for k in range(self.nsteps):
            if k % self.ckpt == 0:
                self.ckpts.append(sim.A.clone())
            sim.step()
        torch.cuda.synchronize()
        self.final = sim.A
        if self.tag is None:
            return float(sim.diagnostics()[6])
        # mean z-displacement of the tagged particles (by id)
        ids = sim.A.id.cpu().numpy().astype(np.int64)
        z = sim.A.x[2].cpu().numpy()
        zt = z[np.isin(ids, self.tag)]
        z0 = self.wl.x[np.isin(np.asarray(self.wl.id, dtype=np.int64), self.tag), 2]
        return float(zt.mean() - z0.mean())

    def backward(self, gJ: float):
        sim = self.sim
        n, prec, dev = sim.n, self.prec, self.device
        bar = Cotangent(n, prec, dev)
        tmp = Cotangent(n, prec, dev)
        # dJ/d(final state), seeded by the library: J = sum m |v|^2 / 2, or
        # the mean z of the tagged particles (a byte per id marks them)
        if self.tag is None:
            L.sph_objective_adjoint(L.SPH_OBJ_KINETIC_ENERGY, self.final.struct(), None, 0, 0, gJ, bar.struct(),
                                    stream_handle())
        else:
            flags = torch.zeros(n, dtype=torch.uint8, device=dev)
            flags[torch.as_tensor(self.tag, device=dev)] = 1
            L.sph_objective_adjoint(L.SPH_OBJ_TAGGED_MEAN_Z, self.final.struct(), flags.data_ptr(), n,
                                    int(self.tag.size), gJ, bar.struct(), stream_handle())
        c0bar = torch.zeros(1, dtype=torch.float64, device=dev)
        rbar = Rates(n, prec, False, dev)
        ws_adj_bytes = L.sph_workspace_size(sim.grid, n, prec, L.SPH_SOLID_J2)
        ws_adj = torch.zeros(ws_adj_bytes, dtype=torch.uint8, device=dev)
        fixed = sim.fixed.data_ptr()
        # The recompute of a segment (forward steps from its checkpoint, saving
        # each step's sorted state, permutation, bucket table and rates) and the
        # reverse sweep over the segment after it are independent, so they run
        # on two streams and overlap: the recompute on the current stream, the
        # reverse sweep on a second one (default priority).  Two pools of saved
        # states alternate; a recompute waits until the reverse sweep that read
        # its pool two segments earlier is done, and a reverse sweep waits for
        # its segment's recompute.  The reverse sweep has its own workspace.
        sa = torch.cuda.current_stream()
        sb = torch.cuda.Stream(device=dev)
        sb.wait_stream(sa)   # the cotangents were initialised on sa
        st_a = stream_handle()
        npool = min(self.ckpt, self.nsteps)
        # every saved buffer is written whole before it is read: no fill
        pools = [[(Particles(n, prec, sim.solid, dev, zero=False), torch.empty_like(sim.perm),
                   torch.empty_like(sim.start), Rates(n, prec, False, dev, zero=False)) for _ in range(npool)]
                 for _ in range(2)]
        freed = [None, None]
        for idx, seg in enumerate(reversed(range(len(self.ckpts)))):
            q = idx % 2
            if freed[q] is not None:
                sa.wait_event(freed[q])
            k0 = seg * self.ckpt
            k1 = min(k0 + self.ckpt, self.nsteps)
            sim.A.copy_from(self.ckpts[seg])
            saved = pools[q][:k1 - k0]
            for srt, perm, start, rates in saved:
                # the step's sorted state, permutation and bucket table go
                # straight into the saved buffers; the update advances a copy
                ps = srt.struct()
                cs = cells_struct(start, sim.nc)
                L.sph_build_cells(sim.grid, sim.A.struct(), ps, perm.data_ptr(), cs, sim.ws.data_ptr(),
                                  sim.ws_bytes, st_a)
                sim.A.copy_from(srt)
                r = rates.struct()
                L.sph_interact(sim.params, sim.grid, L.SPH_PASS_FORCE, ps, None, None, ps, cs, 1, r,
                               sim.ws.data_ptr(), sim.ws_bytes, st_a)
                L.sph_integrate(sim.params, L.SPH_STAGE_MOTION, sim.A.struct(), r, fixed, sim.diag[0].data_ptr(),
                                sim.ws.data_ptr(), sim.ws_bytes, st_a)
            ready = torch.cuda.Event()
            ready.record(sa)
            sb.wait_event(ready)
            with torch.cuda.stream(sb):
                st_b = stream_handle()
                for srt, perm, start, rates in reversed(saved):
                    ps = srt.struct()
                    L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_MOTION, ps, rates.struct(), fixed,
                                            bar.struct(), rbar.struct(), None, None, 0, st_b)
                    rb = rbar.struct()
                    L.sph_interact_adjoint(sim.params, sim.grid, L.SPH_PASS_FORCE, ps, None, None, ps,
                                           cells_struct(start, sim.nc), rb, rb, bar.struct(), ws_adj.data_ptr(),
                                           ws_adj_bytes, st_b)
                    L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_EOS, ps, None, None, bar.struct(), None,
                                            c0bar.data_ptr(), ws_adj.data_ptr(), ws_adj_bytes, st_b)
                    L.sph_permute_adjoint(prec, n, perm.data_ptr(), bar.state_struct(), tmp.state_struct(), st_b)
                    bar, tmp = tmp, bar
                done = torch.cuda.Event()
                done.record(sb)
            freed[q] = done
        sa.wait_stream(sb)
        torch.cuda.synchronize()
        # the initial state is in id order; E0 = e0 + |v0|^2 / 2 adds dJ/dE0 v0 to dJ/dv0
        L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_INPUT_VELOCITY, self.ckpts[0].struct(), None, None,
                                bar.struct(), None, None, None, 0, stream_handle())
        return bar.v.double().T.cpu().numpy(), float(c0bar.cpu()[0])


class SolidKineticEnergyRollout:
    """The kinetic energy after `nsteps` fixed-dt steps of a J2 solid (linear
    EOS, free boundaries) and its hand adjoint with respect to the initial
    velocities (at fixed specific internal energy) and the initial
    deviatoric stress.  A solid step runs two interaction loops (the paper's
    note on several loops per iteration): GRADIENT, the stress stage, FORCE,
    then the update.  Reverse of one step: MOTION, FORCE pair reverse (with
    the stress terms), EOS, the stress stage's reverse (Jaumann rate and
    radial return with hardening), the GRADIENT pair reverse, the permutation.
    Checkpoints every `ckpt` steps; the recompute keeps each step's sorted
    state before and after the stress stage, its permutation, bucket table,
    velocity gradient and rates."""

    def __init__(self, wl, prec: int, nsteps: int, ckpt: int, dt: float, device="cuda"):
        assert wl.S is not None, "a solid workload"
        self.wl, self.prec, self.nsteps, self.ckpt, self.dt, self.device = wl, prec, nsteps, max(1, ckpt), dt, device
        self.e0 = wl.E - 0.5 * np.einsum("ij,ij->i", wl.v, wl.v)

    def forward(self, v0: np.ndarray, S0: np.ndarray | None = None) -> float:
        w = copy.copy(self.wl)
        w.v = np.ascontiguousarray(v0, dtype=np.float64)
        w.E = self.e0 + 0.5 * np.einsum("ij,ij->i", w.v, w.v)
        if S0 is not None:
            w.S = np.ascontiguousarray(S0, dtype=np.float64)
        sim = Sim(w, self.prec, self.device, fixed_dt=self.dt)
        self.sim = sim
        self.ckpts = []
        for k in range(self.nsteps):
            if k % self.ckpt == 0:
                self.ckpts.append(sim.A.clone())
            sim.step()
        torch.cuda.synchronize()
        self.final = sim.A
        return float(sim.diagnostics()[6])

    def backward(self, gJ: float):
        sim = self.sim
        n, prec, dev = sim.n, self.prec, self.device
        bar = Cotangent(n, prec, dev, solid=True)
        tmp = Cotangent(n, prec, dev, solid=True)
        L.sph_objective_adjoint(L.SPH_OBJ_KINETIC_ENERGY, self.final.struct(), None, 0, 0, gJ, bar.struct(),
                                stream_handle())
        c0bar = torch.zeros(1, dtype=torch.float64, device=dev)
        rbar = Rates(n, prec, True, dev)
        ws_bytes = L.sph_workspace_size(sim.grid, n, prec, L.SPH_SOLID_J2)
        ws = torch.zeros(ws_bytes, dtype=torch.uint8, device=dev)
        fixed = sim.fixed.data_ptr()
        st = stream_handle()
        FORCE, GRAD = L.SPH_PASS_FORCE, L.SPH_PASS_GRADIENT
        for seg in reversed(range(len(self.ckpts))):
            k0 = seg * self.ckpt
            k1 = min(k0 + self.ckpt, self.nsteps)
            sim.A.copy_from(self.ckpts[seg])
            saved = []
            for _ in range(k0, k1):
                sim.build()
                a, r = sim.A.struct(), sim.rates.struct()
                pre = sim.A.clone()
                L.sph_interact(sim.params, sim.grid, GRAD, a, None, None, a, sim.cells, 1, r, sim.ws.data_ptr(),
                               sim.ws_bytes, st)
                L.sph_integrate(sim.params, L.SPH_STAGE_STRESS, a, r, fixed, None, None, 0, st)
                L.sph_interact(sim.params, sim.grid, FORCE, a, None, None, a, sim.cells, 1, r, sim.ws.data_ptr(),
                               sim.ws_bytes, st)
                saved.append((pre, sim.A.clone(), sim.perm.clone(), sim.start.clone(), sim.rates.clone()))
                L.sph_integrate(sim.params, L.SPH_STAGE_MOTION, a, r, fixed, sim.diag[0].data_ptr(),
                                sim.ws.data_ptr(), sim.ws_bytes, st)
            for pre, post, perm, start, rates in reversed(saved):
                cells = cells_struct(start, sim.nc)
                ps, pp, rb = post.struct(), pre.struct(), rbar.struct()
                L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_MOTION, ps, rates.struct(), fixed, bar.struct(), rb,
                                        None, None, 0, st)
                L.sph_interact_adjoint(sim.params, sim.grid, FORCE, ps, None, None, ps, cells, rb, rb, bar.struct(),
                                       ws.data_ptr(), ws_bytes, st)
                L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_EOS, ps, None, None, bar.struct(), None,
                                        c0bar.data_ptr(), ws.data_ptr(), ws_bytes, st)
                L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_STRESS, pp, rates.struct(), fixed, bar.struct(), rb,
                                        None, None, 0, st)
                L.sph_interact_adjoint(sim.params, sim.grid, GRAD, pp, None, None, pp, cells, rb, rb, bar.struct(),
                                       ws.data_ptr(), ws_bytes, st)
                L.sph_permute_adjoint(prec, n, perm.data_ptr(), bar.state_struct(), tmp.state_struct(), st)
                bar, tmp = tmp, bar
        torch.cuda.synchronize()
        L.sph_integrate_adjoint(sim.params, L.SPH_STAGE_INPUT_VELOCITY, self.ckpts[0].struct(), None, None,
                                bar.struct(), None, None, None, 0, st)
        return bar.v.double().T.cpu().numpy(), bar.S.double().T.cpu().numpy()


class TwoSetKineticEnergyRollout:
    """The kinetic energy after `nsteps` fixed-dt steps of two particle sets
    stepping as two GPUs' shares (decomp.TwoSets without balancing: steps
    a-g of Section II for both sets, the local-remote passes reading the
    other set), and its hand adjoint, including the reverse of both
    local-remote passes (step f).  The gradient is that of the same function
    as for one set holding every particle: the split only reorders sums.

    Reverse of one step, per set X with the other set Y (rates_X sums X's
    local-local and local-remote terms):
      MOTION reverse of X -> cotangent of rates_X;
      local-local pair reverse of X (both cotangents rates_X);
      local-remote pair reverse: targets X with its boundary list, sources Y,
        weights rates_X-bar (X's pass) + sigma rates_Y-bar (Y's mirrored pass);
      EOS reverse of X (and d/dc0); permutation of X.
    """

    def __init__(self, wl, owner, prec: int, nsteps: int, ckpt: int, dt: float, device="cuda"):
        self.wl, self.owner = wl, np.asarray(owner, dtype=bool)
        self.prec, self.nsteps, self.ckpt, self.dt, self.device = prec, nsteps, max(1, ckpt), dt, device
        self.e0 = wl.E - 0.5 * np.einsum("ij,ij->i", wl.v, wl.v)

    def forward(self, v0: np.ndarray, c0: float) -> float:
        from .decomp import TwoSets
        w = copy.copy(self.wl)
        w.v = np.ascontiguousarray(v0, dtype=np.float64)
        w.E = self.e0 + 0.5 * np.einsum("ij,ij->i", w.v, w.v)
        w.params = dict(self.wl.params, c0=float(c0))
        ts = TwoSets(w, self.owner, self.prec, self.device, fixed_dt=self.dt, period=0)
        self.ts = ts
        self.ckpts = []
        for k in range(self.nsteps):
            if k % self.ckpt == 0:
                self.ckpts.append([s.A.clone() for s in ts.sides])
            ts.step()
        torch.cuda.synchronize()
        return float(sum(s.diagnostics()[6] for s in ts.sides))

    def backward(self, gJ: float):
        ts = self.ts
        prec, dev = self.prec, self.device
        sides = ts.sides
        bars = [Cotangent(s.n, prec, dev) for s in sides]
        tmps = [Cotangent(s.n, prec, dev) for s in sides]
        for s, b in zip(sides, bars):
            L.sph_objective_adjoint(L.SPH_OBJ_KINETIC_ENERGY, s.A.struct(), None, 0, 0, gJ, b.struct(),
                                    stream_handle())
        c0bar = torch.zeros(1, dtype=torch.float64, device=dev)
        rbars = [Rates(s.n, prec, False, dev) for s in sides]
        nmax = max(s.n for s in sides)
        ws_bytes = L.sph_workspace_size(ts.grid, nmax, prec, L.SPH_SOLID_J2)
        ws = torch.zeros(ws_bytes, dtype=torch.uint8, device=dev)
        fixed = sides[0].fixed.data_ptr()
        st = stream_handle()
        for seg in reversed(range(len(self.ckpts))):
            k0 = seg * self.ckpt
            k1 = min(k0 + self.ckpt, self.nsteps)
            for s, c in zip(sides, self.ckpts[seg]):
                s.A.copy_from(c)
            saved = []
            for _ in range(k0, k1):
                ts.rates_pass()
                saved.append([(s.A.clone(), s.perm.clone(), s.start.clone(), s.rates.clone()) for s in sides]
                             + [(ts.bidx[0].clone(), ts.bidx[1].clone(), ts.nb.clone())])
                ts.update(fixed)
            for rec in reversed(saved):
                (b0, b1, nb) = rec[2]
                blist = (b0, b1)
                for q in range(2):
                    srt, perm, start, rates = rec[q]
                    L.sph_integrate_adjoint(ts.params, L.SPH_STAGE_MOTION, srt.struct(), rates.struct(), fixed,
                                            bars[q].struct(), rbars[q].struct(), None, None, 0, st)
                for q in range(2):
                    srt, perm, start, rates = rec[q]
                    oth, _, ostart, _ = rec[1 - q]
                    ps, rb = srt.struct(), rbars[q].struct()
                    L.sph_interact_adjoint(ts.params, ts.grid, L.SPH_PASS_FORCE, ps, None, None, ps,
                                           cells_struct(start, ts.nc), rb, rb, bars[q].struct(), ws.data_ptr(),
                                           ws_bytes, st)
                    L.sph_interact_adjoint(ts.params, ts.grid, L.SPH_PASS_FORCE, ps, blist[q].data_ptr(),
                                           nb[q:q + 1].data_ptr(), oth.struct(), cells_struct(ostart, ts.nc), rb,
                                           rbars[1 - q].struct(), bars[q].struct(), ws.data_ptr(), ws_bytes, st)
                for q in range(2):
                    srt, perm, start, rates = rec[q]
                    L.sph_integrate_adjoint(ts.params, L.SPH_STAGE_EOS, srt.struct(), None, None, bars[q].struct(),
                                            None, c0bar.data_ptr(), ws.data_ptr(), ws_bytes, st)
                    L.sph_permute_adjoint(prec, sides[q].n, perm.data_ptr(), bars[q].state_struct(),
                                          tmps[q].state_struct(), st)
                    bars[q], tmps[q] = tmps[q], bars[q]
        torch.cuda.synchronize()
        # back to the caller's order: set A holds the particles with owner False
        vbar = np.empty((self.wl.n, 3))
        for q, mask in enumerate((~self.owner, self.owner)):
            L.sph_integrate_adjoint(ts.params, L.SPH_STAGE_INPUT_VELOCITY, self.ckpts[0][q].struct(), None, None,
                                    bars[q].struct(), None, None, None, 0, st)
            vbar[mask] = bars[q].v.double().T.cpu().numpy()
        return vbar, float(c0bar.cpu()[0])


class KineticEnergy(torch.autograd.Function):
    """J(v0, c0) with the hand adjoint as its backward.

    v0: (n, 3) float64 tensor (host), c0: 0-dim float64 tensor.  `rollout`
    is a KineticEnergyRollout that fixes the rest of the problem.
    """

    @staticmethod
    def forward(ctx, v0, c0, rollout):
        J = rollout.forward(v0.detach().cpu().numpy(), float(c0))
        ctx.rollout = rollout
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        vbar, c0bar = ctx.rollout.backward(float(gJ))
        return torch.from_numpy(vbar), torch.tensor(c0bar, dtype=torch.float64), None
