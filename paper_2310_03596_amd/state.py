"""Device particle arrays and ABI struct builders.

PyTorch serves only as the device allocator and stream provider: every
tensor here is raw device memory handed to libsph by pointer.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import _lib as L


def real_dtype(prec: int):
    return torch.float64 if prec == L.SPH_FP64 else torch.float32


def grid_struct(grid: dict) -> L.SphGrid:
    g = L.SphGrid()
    for d in range(3):
        g.origin[d] = float(grid["origin"][d])
        g.dims[d] = int(grid["dims"][d])
    g.cell = float(grid["cell"])
    return g


def ncells(grid: dict) -> int:
    d = grid["dims"]
    return int(d[0]) * int(d[1]) * int(d[2])


def params_struct(p: dict, prec: int) -> L.SphParams:
    s = L.SphParams()
    for k in ("h", "rho0", "c0", "gamma", "K", "G", "Y0", "H", "beta", "cfl"):
        setattr(s, k, float(p[k]))
    for d in range(3):
        s.gravity[d] = float(p["gravity"][d])
        s.wall_lo[d] = float(p["wall_lo"][d])
        s.wall_hi[d] = float(p["wall_hi"][d])
    s.wall_mask = int(p["wall_mask"])
    s.material = int(p["material"])
    s.prec = int(prec)
    s.eos = int(p.get("eos", L.SPH_EOS_LINEAR))
    for k in ("mg_s", "mg_gamma0", "p_cut"):
        setattr(s, k, float(p.get(k, 0.0)))
    return s


def _ptr(t):
    return None if t is None else t.data_ptr()


def _carve(buf: torch.Tensor, layout):
    """Views of one flat byte buffer, one per (name, shape, dtype) of layout
    (None where shape is None), each at a 256-byte aligned offset."""
    out, off = {}, 0
    for name, shape, dt in layout:
        if shape is None:
            out[name] = None
            continue
        nbytes = int(np.prod(shape)) * torch.empty((), dtype=dt).element_size()
        out[name] = buf[off:off + nbytes].view(dt).view(shape)
        off += (nbytes + 255) & ~255
    return out


def _carved_bytes(layout) -> int:
    off = 0
    for _, shape, dt in layout:
        if shape is not None:
            off += (int(np.prod(shape)) * torch.empty((), dtype=dt).element_size() + 255) & ~255
    return max(off, 256)


class _Flat:
    """Fields that live in one device allocation, so that a copy of the whole
    set (checkpoints, saved states of the reverse pass) is one copy."""

    def _allocate(self, layout, device, zero=True):
        """zero=False leaves the memory uninitialised (no fill kernel), for
        buffers that a call overwrites completely before anything reads them."""
        self._layout = layout
        alloc = torch.zeros if zero else torch.empty
        self._buf = alloc(_carved_bytes(layout), dtype=torch.uint8, device=device)
        self._bind()

    def _bind(self):
        for k, v in _carve(self._buf, self._layout).items():
            setattr(self, k, v)
        self._struct = None   # the ABI struct of these buffers, built on first use

    def clone(self):
        """A copy with its own storage (one device copy)."""
        q = copy.copy(self)
        q._buf = self._buf.clone()
        q._bind()
        return q

    def copy_from(self, other):
        """Overwrite every field with other's (same sizes; one device copy)."""
        self._buf.copy_(other._buf)


class Particles(_Flat):
    """One particle array in SoA form on the device."""

    REAL = ("m", "w", "rho", "p", "c", "e")

    def __init__(self, n: int, prec: int, solid: bool, device="cuda", zero: bool = True):
        real = real_dtype(prec)
        self.n, self.prec, self.solid, self.device = n, prec, solid, device
        split = prec == L.SPH_FP32_SPLIT
        layout = [("x", (3, n), torch.float64), ("off", (3, n) if split else None, torch.float32),
                  ("hash", (n,), torch.int32), ("id", (n,), torch.int32), ("v", (3, n), real)]
        layout += [(f, (n,), real) for f in self.REAL]
        layout += [("E", (n,), torch.float64), ("S", (6, n) if solid else None, real),
                   ("ep", (n,) if solid else None, real)]
        self._allocate(layout, device, zero)

    def struct(self) -> L.SphParticles:
        """The ABI struct of this array (built once: the buffers never move)."""
        if self._struct is None:
            self._struct = self._make_struct()
        return self._struct

    def _make_struct(self) -> L.SphParticles:
        s = L.SphParticles()
        s.n = self.n
        s.prec = self.prec
        if self.n == 0:
            return s
        for d in range(3):
            s.x[d] = self.x[d].data_ptr()
            s.v[d] = self.v[d].data_ptr()
            if self.off is not None:
                s.off[d] = self.off[d].data_ptr()
        s.hash = self.hash.data_ptr()
        s.id = self.id.data_ptr()
        s.m, s.omega, s.rho = self.m.data_ptr(), self.w.data_ptr(), self.rho.data_ptr()
        s.p, s.c, s.e = self.p.data_ptr(), self.c.data_ptr(), self.e.data_ptr()
        s.E = self.E.data_ptr()
        if self.solid:
            for k in range(6):
                s.S[k] = self.S[k].data_ptr()
            s.eps_p = self.ep.data_ptr()
        return s

    @classmethod
    def upload(cls, wl, prec: int, device="cuda") -> "Particles":
        p = cls(wl.n, prec, wl.S is not None, device)
        real = real_dtype(prec)
        p.x.copy_(torch.from_numpy(np.ascontiguousarray(wl.x.T)))
        p.v.copy_(torch.from_numpy(np.ascontiguousarray(wl.v.T)).to(real))
        p.m.copy_(torch.from_numpy(wl.m).to(real))
        p.w.copy_(torch.from_numpy(wl.omega).to(real))
        p.rho.copy_(torch.from_numpy(wl.rho).to(real))
        p.E.copy_(torch.from_numpy(wl.E))
        p.id.copy_(torch.from_numpy(wl.id.astype(np.int64)).to(torch.int32))
        if wl.S is not None:
            p.S.copy_(torch.from_numpy(np.ascontiguousarray(wl.S.T)).to(real))
            p.ep.copy_(torch.from_numpy(wl.eps_p).to(real))
        return p

    def host(self) -> dict:
        """Copy every field to host numpy arrays (array order, positions (n,3))."""
        out = {"x": self.x.T.cpu().numpy().copy(), "v": self.v.T.double().cpu().numpy().copy(),
               "hash": self.hash.cpu().numpy().view(np.uint32).copy(),
               "id": self.id.cpu().numpy().view(np.uint32).copy(), "E": self.E.cpu().numpy().copy()}
        for f in self.REAL:
            out[f] = getattr(self, f).double().cpu().numpy().copy()
        if self.off is not None:
            out["off"] = self.off.T.double().cpu().numpy().copy()
        if self.solid:
            out["S"] = self.S.T.double().cpu().numpy().copy()
            out["ep"] = self.ep.double().cpu().numpy().copy()
        return out


class Rates(_Flat):
    """Pair-sum outputs: FORCE rates and, for solids, the velocity gradient."""

    def __init__(self, n: int, prec: int, gradient: bool, device="cuda", zero: bool = True):
        real = real_dtype(prec)
        split = prec == L.SPH_FP32_SPLIT
        self._allocate([("hi", (6, n), real), ("lo", (6, n) if split else None, real),
                        ("Lhi", (9, n) if gradient else None, real),
                        ("Llo", (9, n) if (gradient and split) else None, real)], device, zero)

    def struct(self) -> L.SphRates:
        if self._struct is None:
            self._struct = self._make_struct()
        return self._struct

    def _make_struct(self) -> L.SphRates:
        r = L.SphRates()
        if self.hi.shape[1] == 0:
            return r
        for k in range(6):
            r.hi[k] = self.hi[k].data_ptr()
            if self.lo is not None:
                r.lo[k] = self.lo[k].data_ptr()
        if self.Lhi is not None:
            for k in range(9):
                r.Lhi[k] = self.Lhi[k].data_ptr()
                if self.Llo is not None:
                    r.Llo[k] = self.Llo[k].data_ptr()
        return r

    def force(self) -> torch.Tensor:
        """(6, n) rate sums as float64 (hi + lo)."""
        f = self.hi.double()
        return f + self.lo.double() if self.lo is not None else f

    def grad(self) -> torch.Tensor:
        f = self.Lhi.double()
        return f + self.Llo.double() if self.Llo is not None else f


def cells_struct(start: torch.Tensor, nc: int) -> L.SphCells:
    c = L.SphCells()
    c.start = start.data_ptr()
    c.ncells = nc
    return c


def stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream
