"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Each function names the step of the hot path it computes; the arithmetic
lives in ``sph_oracle.c``.  Arrays are numpy, float64 unless stated.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        _declare(_lib)
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Route every call of this module to another build of the oracle (the
    tests use it to check that a deliberately mistaken copy fails its pins)."""
    global _lib
    saved = _lib
    alt = C.CDLL(path)
    _declare(alt)
    _lib = alt
    try:
        yield alt
    finally:
        _lib = saved


class OGrid(C.Structure):
    _fields_ = [("o", C.c_double * 3), ("L", C.c_double), ("n", C.c_int32 * 3)]


class OParams(C.Structure):
    _fields_ = [("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double),
                ("gamma", C.c_double), ("K", C.c_double), ("G", C.c_double),
                ("Y0", C.c_double), ("H", C.c_double), ("beta", C.c_double),
                ("cfl", C.c_double), ("g", C.c_double * 3), ("wlo", C.c_double * 3),
                ("whi", C.c_double * 3), ("wall_mask", C.c_int32), ("material", C.c_int32),
                ("eos", C.c_int32), ("pad", C.c_int32), ("mg_s", C.c_double), ("mg_gamma0", C.c_double),
                ("p_cut", C.c_double)]


_dp = C.POINTER(C.c_double)
_up = C.POINTER(C.c_uint32)


class OState(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", _dp), ("v", _dp), ("m", _dp), ("w", _dp),
                ("rho", _dp), ("p", _dp), ("c", _dp), ("E", _dp), ("S", _dp), ("ep", _dp),
                ("id", _up), ("hash", _up)]


def _declare(L):
    vp = C.c_void_p
    L.or_hash.argtypes = [C.POINTER(OGrid), C.c_int64, vp, vp]
    L.or_sort_perm.argtypes = [C.c_int64, vp, C.c_uint32, vp]
    L.or_sort_perm.restype = C.c_int
    L.or_cell_start.argtypes = [C.c_int64, vp, C.c_uint32, vp]
    L.or_cell_start.restype = C.c_int
    L.or_gather.argtypes = [C.POINTER(OState), C.POINTER(OState), vp]
    L.or_mark.argtypes = [C.POINTER(OGrid), C.c_int64, vp, vp, vp, vp, vp]
    L.or_kernel_W.argtypes = [C.c_double, C.c_double]
    L.or_kernel_W.restype = C.c_double
    L.or_kernel_F.argtypes = [C.c_double, C.c_double]
    L.or_kernel_F.restype = C.c_double
    L.or_eos.argtypes = [C.POINTER(OParams), C.c_double, C.c_double, _dp, _dp]
    L.or_pair.argtypes = [C.POINTER(OParams), vp, vp, vp] + [C.c_double] * 10 + [vp, vp, vp]
    L.or_pair_grad.argtypes = [C.POINTER(OParams), vp, vp, vp, C.c_double, vp]
    L.or_interact.argtypes = [C.POINTER(OParams), C.POINTER(OGrid), C.c_int, C.POINTER(OState),
                              vp, C.c_int64, C.POINTER(OState), vp, C.c_int, vp, vp]
    L.or_interact_abs.argtypes = L.or_interact.argtypes
    L.or_interact_peak.argtypes = L.or_interact.argtypes
    L.or_neighbors.argtypes = [C.POINTER(OParams), C.POINTER(OGrid), C.POINTER(OState),
                               C.POINTER(OState), vp, C.c_int, vp, vp, C.c_int64]
    L.or_neighbors.restype = C.c_int64
    L.or_integrate.argtypes = [C.POINTER(OParams), C.c_int, C.POINTER(OState), vp, vp,
                               C.c_double, vp]
    L.or_run.argtypes = [C.POINTER(OParams), C.POINTER(OGrid), C.POINTER(OState), C.c_int,
                         C.c_double, vp, vp, vp]
    L.or_run.restype = C.c_int
    L.or_num_threads.restype = C.c_int
    L.or_set_threads.argtypes = [C.c_int]
    L.or_centroid.argtypes = [C.POINTER(OState), vp]
    L.or_balance_hash.argtypes = [C.POINTER(OState), vp, vp, C.c_uint32, vp]
    L.or_balance_hash.restype = C.c_int64
    L.or_balance_select.argtypes = [C.c_int64, vp, C.c_uint32, C.c_int64, vp]
    L.or_balance_select.restype = C.c_int
    L.or_swap.argtypes = [C.POINTER(OState), vp, C.POINTER(OState), vp, C.c_int64]


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_num_threads())


def set_threads(n: int):
    """Threads of the oracle's following parallel loops."""
    lib().or_set_threads(int(n))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def grid_struct(grid: dict) -> OGrid:
    g = OGrid()
    for d in range(3):
        g.o[d] = grid["origin"][d]
        g.n[d] = grid["dims"][d]
    g.L = grid["cell"]
    return g


def params_struct(p: dict) -> OParams:
    s = OParams()
    for k in ("h", "rho0", "c0", "gamma", "K", "G", "Y0", "H", "beta", "cfl"):
        setattr(s, k, float(p[k]))
    for d in range(3):
        s.g[d] = p["gravity"][d]
        s.wlo[d] = p["wall_lo"][d]
        s.whi[d] = p["wall_hi"][d]
    s.wall_mask = int(p["wall_mask"])
    s.material = int(p["material"])
    s.eos = int(p.get("eos", 0))
    for k in ("mg_s", "mg_gamma0", "p_cut"):
        setattr(s, k, float(p.get(k, 0.0)))
    return s


def ncells(grid: dict) -> int:
    d = grid["dims"]
    return int(d[0]) * int(d[1]) * int(d[2])


class State:
    """Particle state in the oracle's layout (row-major (n,3) positions)."""

    FIELDS = ("x", "v", "m", "w", "rho", "p", "c", "E", "S", "ep", "id", "hash")

    def __init__(self, n: int, solid: bool = False):
        self.n = n
        self.x = np.zeros((n, 3))
        self.v = np.zeros((n, 3))
        self.m = np.zeros(n)
        self.w = np.zeros(n)
        self.rho = np.zeros(n)
        self.p = np.zeros(n)
        self.c = np.zeros(n)
        self.E = np.zeros(n)
        self.S = np.zeros((n, 6)) if solid else None
        self.ep = np.zeros(n) if solid else None
        self.id = np.zeros(n, dtype=np.uint32)
        self.hash = np.zeros(n, dtype=np.uint32)

    @classmethod
    def from_workload(cls, wl) -> "State":
        s = cls(wl.n, wl.S is not None)
        s.x[:] = wl.x
        s.v[:] = wl.v
        s.m[:] = wl.m
        s.w[:] = wl.omega
        s.rho[:] = wl.rho
        s.E[:] = wl.E
        s.id[:] = wl.id
        if wl.S is not None:
            s.S[:] = wl.S
            s.ep[:] = wl.eps_p
        return s

    def copy(self) -> "State":
        o = State(self.n, self.S is not None)
        for f in self.FIELDS:
            a = getattr(self, f)
            if a is not None:
                getattr(o, f)[...] = a
        return o

    def struct(self) -> OState:
        s = OState()
        s.n = self.n
        for f in self.FIELDS:
            a = getattr(self, f)
            if a is not None:
                assert a.flags["C_CONTIGUOUS"]
                setattr(s, f, a.ctypes.data_as(_up if a.dtype == np.uint32 else _dp))
        return s

    def by_id(self) -> "State":
        """Copy reordered so that row k holds particle id k."""
        order = np.argsort(self.id, kind="stable")
        o = State(self.n, self.S is not None)
        for f in self.FIELDS:
            a = getattr(self, f)
            if a is not None:
                getattr(o, f)[...] = a[order]
        return o


# ----------------------------------------------------------- per-step calls

def hash_cells(grid: dict, x: np.ndarray) -> np.ndarray:
    """Bucket hash of every particle (Section I; Section II step a)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(x.shape[0], dtype=np.uint32)
    g = grid_struct(grid)
    lib().or_hash(C.byref(g), x.shape[0], _ptr(x), _ptr(out))
    return out


def sort_perm(key: np.ndarray, nkeys: int) -> np.ndarray:
    """Stable ascending order of key (Section I radix sort)."""
    key = np.ascontiguousarray(key, dtype=np.uint32)
    perm = np.empty(key.shape[0], dtype=np.uint32)
    if lib().or_sort_perm(key.shape[0], _ptr(key), nkeys, _ptr(perm)) != 0:
        raise MemoryError
    return perm


def cell_start(sorted_key: np.ndarray, nc: int) -> np.ndarray:
    sk = np.ascontiguousarray(sorted_key, dtype=np.uint32)
    start = np.empty(nc + 1, dtype=np.uint32)
    if lib().or_cell_start(sk.shape[0], _ptr(sk), nc, _ptr(start)) != 0:
        raise MemoryError
    return start


def gather(s: State, perm: np.ndarray) -> State:
    o = State(s.n, s.S is not None)
    a, b = o.struct(), s.struct()
    lib().or_gather(C.byref(a), C.byref(b), _ptr(np.ascontiguousarray(perm, dtype=np.uint32)))
    return o


def build_cells(grid: dict, s: State):
    """Hash, stable sort, gather and cell table: returns (sorted state, perm, start)."""
    h = hash_cells(grid, s.x)
    s.hash[:] = h
    perm = sort_perm(h, ncells(grid))
    o = gather(s, perm)
    start = cell_start(o.hash, ncells(grid))
    return o, perm, start


def mark_boundary(grid: dict, local_hash: np.ndarray, remote_start: np.ndarray):
    """Communication hash and MGPU boundary list (Section II, step c)."""
    n = local_hash.shape[0]
    lh = np.ascontiguousarray(local_hash, dtype=np.uint32)
    comm = np.empty(n, dtype=np.uint32)
    bidx = np.empty(n, dtype=np.uint32)
    nb = np.zeros(1, dtype=np.uint32)
    g = grid_struct(grid)
    lib().or_mark(C.byref(g), n, _ptr(lh), _ptr(np.ascontiguousarray(remote_start, dtype=np.uint32)),
                  _ptr(comm), _ptr(bidx), _ptr(nb))
    return comm, bidx[: int(nb[0])].copy()


def kernel_W(r: float, h: float) -> float:
    return lib().or_kernel_W(r, h)


def kernel_F(r: float, h: float) -> float:
    return lib().or_kernel_F(r, h)


def eos(params: dict, rho: float, e: float = 0.0):
    """(p, c) at density rho and specific internal energy e (e matters only
    for the Mie-Gruneisen solid)."""
    p, c = C.c_double(), C.c_double()
    P = params_struct(params)
    lib().or_eos(C.byref(P), rho, e, C.byref(p), C.byref(c))
    return p.value, c.value


def pair(params: dict, d, vi, vj, wi, wj, rhoi, rhoj, pi, pj, ci, cj, ei, ej, Si=None, Sj=None):
    """FORCE terms (mdot, mvdot[3], mEdot, wdot) of target i from source j."""
    P = params_struct(params)
    d = np.ascontiguousarray(d, dtype=np.float64)
    vi = np.ascontiguousarray(vi, dtype=np.float64)
    vj = np.ascontiguousarray(vj, dtype=np.float64)
    Si = None if Si is None else np.ascontiguousarray(Si, dtype=np.float64)
    Sj = None if Sj is None else np.ascontiguousarray(Sj, dtype=np.float64)
    out = np.empty(6)
    lib().or_pair(C.byref(P), _ptr(d), _ptr(vi), _ptr(vj), wi, wj, rhoi, rhoj, pi, pj, ci, cj,
                  ei, ej, _ptr(Si), _ptr(Sj), _ptr(out))
    return out


def pair_grad(params: dict, d, vi, vj, wj):
    P = params_struct(params)
    out = np.empty(9)
    lib().or_pair_grad(C.byref(P), _ptr(np.ascontiguousarray(d, dtype=np.float64)),
                       _ptr(np.ascontiguousarray(vi, dtype=np.float64)),
                       _ptr(np.ascontiguousarray(vj, dtype=np.float64)), wj, _ptr(out))
    return out.reshape(3, 3)


FORCE, GRADIENT = 0, 1
MOTION, STRESS, EOS = 0, 1, 2


def interact(params: dict, grid: dict, pass_: int, tgt: State, src: State, src_start,
             self_pass: bool, rates=None, L=None, tidx=None):
    """Accumulate pair sums into rates (n,6) or L (n,9) (Section II steps e, f)."""
    P = params_struct(params)
    g = grid_struct(grid)
    if pass_ == FORCE and rates is None:
        rates = np.zeros((tgt.n, 6))
    if pass_ == GRADIENT and L is None:
        L = np.zeros((tgt.n, 9))
    ti = None if tidx is None else np.ascontiguousarray(tidx, dtype=np.uint32)
    nt = tgt.n if ti is None else ti.shape[0]
    a, b = tgt.struct(), src.struct()
    lib().or_interact(C.byref(P), C.byref(g), pass_, C.byref(a), _ptr(ti), nt, C.byref(b),
                      _ptr(np.ascontiguousarray(src_start, dtype=np.uint32)), int(self_pass),
                      _ptr(rates), _ptr(L))
    return rates if pass_ == FORCE else L


def interact_abs(params: dict, grid: dict, pass_: int, tgt: State, src: State, src_start,
                 self_pass: bool, tidx=None, peak: bool = False):
    """Per-target sums of |pair term| (the round-off scale of each rate); with
    peak=True every term is rescaled to the kernel's peak strength F_max / F."""
    P = params_struct(params)
    g = grid_struct(grid)
    out = np.zeros((tgt.n, 6 if pass_ == FORCE else 9))
    ti = None if tidx is None else np.ascontiguousarray(tidx, dtype=np.uint32)
    nt = tgt.n if ti is None else ti.shape[0]
    a, b = tgt.struct(), src.struct()
    fn = lib().or_interact_peak if peak else lib().or_interact_abs
    fn(C.byref(P), C.byref(g), pass_, C.byref(a), _ptr(ti), nt, C.byref(b),
       _ptr(np.ascontiguousarray(src_start, dtype=np.uint32)), int(self_pass),
       _ptr(out) if pass_ == FORCE else None, _ptr(out) if pass_ == GRADIENT else None)
    return out


def neighbors(params: dict, grid: dict, tgt: State, src: State, src_start, self_pass: bool):
    """Ordered (i, j) pairs visited with r < 2h, in visiting order."""
    P = params_struct(params)
    g = grid_struct(grid)
    a, b = tgt.struct(), src.struct()
    st = np.ascontiguousarray(src_start, dtype=np.uint32)
    cnt = lib().or_neighbors(C.byref(P), C.byref(g), C.byref(a), C.byref(b), _ptr(st),
                             int(self_pass), None, None, 0)
    pi = np.empty(cnt, dtype=np.uint32)
    pj = np.empty(cnt, dtype=np.uint32)
    lib().or_neighbors(C.byref(P), C.byref(g), C.byref(a), C.byref(b), _ptr(st),
                       int(self_pass), _ptr(pi), _ptr(pj), cnt)
    return pi, pj


def integrate(params: dict, stage: int, s: State, rates=None, L=None, dt: float = 0.0):
    """Update s in place (Section II step g); returns the 7 diagnostics."""
    P = params_struct(params)
    diag = np.zeros(7)
    a = s.struct()
    r = None if rates is None else np.ascontiguousarray(rates, dtype=np.float64)
    l = None if L is None else np.ascontiguousarray(L, dtype=np.float64)
    lib().or_integrate(C.byref(P), stage, C.byref(a), _ptr(r), _ptr(l), dt, _ptr(diag))
    return diag


def run(params: dict, grid: dict, s: State, nsteps: int, fixed_dt: float = 0.0, dts_in=None):
    """Whole steps in C; s is updated in place.  Returns (dts used, last diag)."""
    P = params_struct(params)
    g = grid_struct(grid)
    dts = np.zeros(max(nsteps, 1))
    diag = np.zeros(7)
    di = None if dts_in is None else np.ascontiguousarray(dts_in, dtype=np.float64)
    a = s.struct()
    if lib().or_run(C.byref(P), C.byref(g), C.byref(a), nsteps, fixed_dt, _ptr(di), _ptr(dts),
                    _ptr(diag)) != 0:
        raise MemoryError
    return dts[:nsteps], diag


def prime(params: dict, s: State):
    """EOS stage on the initial state: rho = m / w, p, c; returns diagnostics."""
    return integrate(params, EOS, s)


# ------------------------------------------------------------- balancing

HMAX = 1000   # maximum balancing hash (Section III.A: "typically 1000")


def centroid(s: State):
    """(Cg (3,), total mass): mass-weighted centre of gravity (Section III.A)."""
    out = np.zeros(4)
    lib().or_centroid(C.byref(s.struct()), _ptr(out))
    return out[:3].copy(), float(out[3])


def balance_hash(s: State, cg_own, cg_other, hmax: int = HMAX):
    """Balancing hash of every particle towards the other GPU's Cg, and the
    number with a positive hash (Section III.A)."""
    own = np.ascontiguousarray(cg_own, dtype=np.float64)
    oth = np.ascontiguousarray(cg_other, dtype=np.float64)
    h = np.zeros(s.n, dtype=np.uint32)
    npos = lib().or_balance_hash(C.byref(s.struct()), _ptr(own), _ptr(oth), hmax, _ptr(h))
    return h, int(npos)


def balance_select(bhash: np.ndarray, k: int, hmax: int = HMAX) -> np.ndarray:
    """Indices of the k largest balancing hashes, ties in ascending index."""
    bhash = np.ascontiguousarray(bhash, dtype=np.uint32)
    sel = np.zeros(max(k, 1), dtype=np.uint32)
    if lib().or_balance_select(bhash.shape[0], _ptr(bhash), hmax, k, _ptr(sel)) != 0:
        raise MemoryError
    return sel[:k]


# ------------------------------------------- several particle types (III.B)
# Every type is balanced on its own with the rule of Section III.A, towards
# centres biased to the centre of all the particles:
#   Cg'_t = alpha Cg_all + (1 - alpha) Cg_t,  alpha = 0.1.
# Labels of ntypes or more take no part.  These functions apply the
# single-type steps above to each type's particles in turn.

ALPHA = 0.1   # Section III.B


def _part(s: State, mask: np.ndarray) -> State:
    """The particles of s selected by mask (positions and masses)."""
    o = State(int(mask.sum()))
    o.x[:] = s.x[mask]
    o.m[:] = s.m[mask]
    return o


def centroid_types(s: State, types: np.ndarray, ntypes: int, alpha: float = ALPHA) -> np.ndarray:
    """(ntypes + 1, 4) records: row t < ntypes holds Cg'_t and the mass of
    type t (zeros for a type without mass), row ntypes holds Cg_all over the
    particles of every valid type and their mass (Section III.B)."""
    types = np.asarray(types)
    out = np.zeros((ntypes + 1, 4))
    call, mall = centroid(_part(s, types < ntypes))
    out[ntypes, :3], out[ntypes, 3] = call, mall
    for t in range(ntypes):
        ct, mt = centroid(_part(s, types == t))
        if mt > 0:
            out[t, :3] = alpha * call + (1.0 - alpha) * ct
        out[t, 3] = mt
    return out


def balance_hash_types(s: State, types: np.ndarray, ntypes: int, cg_own, cg_other, hmax: int = HMAX):
    """Balancing hash of every particle towards its own type's centres (rows
    of cg_own, cg_other), and the number of positive hashes per type."""
    types = np.asarray(types)
    h = np.zeros(s.n, dtype=np.uint32)
    npos = np.zeros(ntypes, dtype=np.int64)
    for t in range(ntypes):
        m = types == t
        ht, nt = balance_hash(_part(s, m), np.asarray(cg_own)[t, :3], np.asarray(cg_other)[t, :3], hmax)
        h[m] = ht
        npos[t] = nt
    return h, npos


def balance_select_types(bhash: np.ndarray, types: np.ndarray, ntypes: int, npos_own, npos_other,
                         hmax: int = HMAX):
    """Per type t, k_t = min(npos_own[t], npos_other[t], count of type t) and
    the indices of its k_t largest hashes (ties in ascending index), one type
    after another.  Returns (sel, k, offsets) with offsets[ntypes] = len(sel)."""
    types = np.asarray(types)
    bhash = np.asarray(bhash, dtype=np.uint32)
    parts = []
    k = np.zeros(ntypes, dtype=np.int64)
    off = np.zeros(ntypes + 1, dtype=np.int64)
    for t in range(ntypes):
        idx = np.nonzero(types == t)[0]
        kt = min(int(npos_own[t]), int(npos_other[t]), idx.size)
        parts.append(idx[balance_select(bhash[idx], kt, hmax)].astype(np.uint32))
        k[t] = kt
        off[t + 1] = off[t] + kt
    sel = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint32)
    return sel, k, off


def swap(a: State, sel_a: np.ndarray, b: State, sel_b: np.ndarray):
    """Exchange the selected particles of a and b pairwise (in place)."""
    k = len(sel_a)
    assert len(sel_b) == k
    sa = np.ascontiguousarray(sel_a, dtype=np.uint32)
    sb = np.ascontiguousarray(sel_b, dtype=np.uint32)
    lib().or_swap(C.byref(a.struct()), _ptr(sa), C.byref(b.struct()), _ptr(sb), k)
