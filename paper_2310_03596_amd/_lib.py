"""ctypes binding of libsph (the C ABI declared in include/sph.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libsph.so.  Importing this module fails loudly if the library
has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK, SPH_ERR_ARG, SPH_ERR_WORKSPACE, SPH_ERR_HIP, SPH_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
SPH_FP64, SPH_FP32_SPLIT = 0, 1
SPH_FLUID_TAIT, SPH_SOLID_J2 = 0, 1
SPH_PASS_FORCE, SPH_PASS_GRADIENT = 0, 1
SPH_STAGE_MOTION, SPH_STAGE_STRESS, SPH_STAGE_EOS, SPH_STAGE_INPUT_VELOCITY = 0, 1, 2, 3
SPH_OBJ_KINETIC_ENERGY, SPH_OBJ_TAGGED_MEAN_Z = 0, 1
SPH_EOS_LINEAR, SPH_EOS_MIE_GRUNEISEN = 0, 1
SPH_MAX_TYPES = 8   # particle types of the per-type balancing calls

_vp = C.c_void_p


class SphGrid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("cell", C.c_double), ("dims", C.c_int32 * 3),
                ("reserved", C.c_int32)]


class SphParams(C.Structure):
    _fields_ = [("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double), ("gamma", C.c_double),
                ("K", C.c_double), ("G", C.c_double), ("Y0", C.c_double), ("H", C.c_double),
                ("beta", C.c_double), ("cfl", C.c_double), ("gravity", C.c_double * 3),
                ("wall_lo", C.c_double * 3), ("wall_hi", C.c_double * 3), ("wall_mask", C.c_uint32),
                ("material", C.c_int32), ("prec", C.c_int32), ("eos", C.c_int32), ("mg_s", C.c_double),
                ("mg_gamma0", C.c_double), ("p_cut", C.c_double)]


class SphParticles(C.Structure):
    _fields_ = [("n", C.c_uint32), ("prec", C.c_int32), ("x", _vp * 3), ("off", _vp * 3), ("hash", _vp),
                ("id", _vp), ("v", _vp * 3), ("m", _vp), ("omega", _vp), ("rho", _vp), ("p", _vp),
                ("c", _vp), ("e", _vp), ("E", _vp), ("S", _vp * 6), ("eps_p", _vp)]


class SphCells(C.Structure):
    _fields_ = [("start", _vp), ("ncells", C.c_uint32), ("reserved", C.c_uint32)]


class SphRates(C.Structure):
    _fields_ = [("hi", _vp * 6), ("lo", _vp * 6), ("Lhi", _vp * 9), ("Llo", _vp * 9)]


class SphAdjoint(C.Structure):
    _fields_ = [("x", _vp * 3), ("v", _vp * 3), ("m", _vp), ("omega", _vp), ("E", _vp), ("rho", _vp),
                ("p", _vp), ("c", _vp), ("e", _vp), ("S", _vp * 6), ("eps_p", _vp)]


EXPORTS = ("sph_version", "sph_last_error", "sph_workspace_size", "sph_build_cells", "sph_mark_boundary",
           "sph_mark_boundary_noalloc", "sph_pack_boundary", "sph_interact", "sph_count_pairs", "sph_set_pair_events",
           "sph_neighbor_census", "sph_integrate", "sph_interact_adjoint",
           "sph_integrate_adjoint", "sph_objective_adjoint", "sph_permute_adjoint", "sph_centroid", "sph_balance_hash",
           "sph_balance_select", "sph_swap", "sph_centroid_types", "sph_balance_hash_types",
           "sph_balance_select_types")

_lib = None


class SphError(RuntimeError):
    def __init__(self, name, code, msg):
        super().__init__(f"{name} failed with status {code}: {msg}")
        self.code = code


def load():
    """Load libsph.so (raises if it is missing: the library must be built first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsph.so not built at {LIB_PATH}; run __graft_entry__.build() "
                           "or python paper_2310_03596_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.sph_version.restype = C.c_char_p
    L.sph_last_error.restype = C.c_char_p
    L.sph_workspace_size.argtypes = [P(SphGrid), C.c_uint32, C.c_int, C.c_int]
    L.sph_workspace_size.restype = C.c_size_t
    L.sph_build_cells.argtypes = [P(SphGrid), P(SphParticles), P(SphParticles), _vp, SphCells, _vp,
                                  C.c_size_t, _vp]
    L.sph_mark_boundary.argtypes = [P(SphGrid), P(SphParticles), SphCells, _vp, _vp, C.c_uint32, _vp, _vp, _vp,
                                    C.c_size_t, _vp]
    L.sph_mark_boundary_noalloc.argtypes = [P(SphGrid), P(SphParticles), SphCells, _vp, _vp, C.c_uint32, _vp, _vp,
                                            _vp]
    L.sph_pack_boundary.argtypes = [P(SphParticles), _vp, _vp, P(SphParticles), _vp]
    L.sph_interact.argtypes = [P(SphParams), P(SphGrid), C.c_int, P(SphParticles), _vp, _vp,
                               P(SphParticles), SphCells, C.c_int, P(SphRates), _vp, C.c_size_t, _vp]
    L.sph_count_pairs.argtypes = [P(SphParams), P(SphGrid), P(SphParticles), _vp, _vp, P(SphParticles),
                                  SphCells, _vp, _vp]
    L.sph_set_pair_events.argtypes = [_vp, _vp]
    L.sph_neighbor_census.argtypes = [P(SphParams), P(SphGrid), C.c_int, P(SphParticles), _vp, _vp,
                                      P(SphParticles), SphCells, _vp, _vp, _vp, C.c_size_t, _vp]
    L.sph_integrate.argtypes = [P(SphParams), C.c_int, P(SphParticles), P(SphRates), _vp, _vp, _vp,
                                C.c_size_t, _vp]
    L.sph_interact_adjoint.argtypes = [P(SphParams), P(SphGrid), C.c_int, P(SphParticles), _vp, _vp,
                                       P(SphParticles), SphCells, P(SphRates), P(SphRates), P(SphAdjoint), _vp,
                                       C.c_size_t, _vp]
    L.sph_integrate_adjoint.argtypes = [P(SphParams), C.c_int, P(SphParticles), P(SphRates), _vp,
                                        P(SphAdjoint), P(SphRates), _vp, _vp, C.c_size_t, _vp]
    L.sph_objective_adjoint.argtypes = [C.c_int, P(SphParticles), _vp, C.c_uint32, C.c_uint32, C.c_double,
                                        P(SphAdjoint), _vp]
    L.sph_permute_adjoint.argtypes = [C.c_int, C.c_uint32, _vp, P(SphAdjoint), P(SphAdjoint), _vp]
    L.sph_centroid.argtypes = [P(SphParticles), _vp, _vp, C.c_size_t, _vp]
    L.sph_balance_hash.argtypes = [P(SphParticles), _vp, _vp, C.c_uint32, _vp, _vp, _vp, C.c_size_t, _vp]
    L.sph_balance_select.argtypes = [C.c_uint32, _vp, C.c_uint32, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]
    L.sph_swap.argtypes = [P(SphParticles), _vp, P(SphParticles), _vp, _vp, C.c_uint32, _vp]
    L.sph_centroid_types.argtypes = [P(SphParticles), _vp, C.c_uint32, C.c_double, _vp, _vp, C.c_size_t, _vp]
    L.sph_balance_hash_types.argtypes = [P(SphParticles), _vp, C.c_uint32, _vp, _vp, C.c_uint32, _vp, _vp, _vp,
                                         C.c_size_t, _vp]
    L.sph_balance_select_types.argtypes = [C.c_uint32, _vp, C.c_uint32, _vp, C.c_uint32, _vp, _vp, _vp, _vp, _vp,
                                           _vp, C.c_size_t, _vp]
    for name in EXPORTS[3:]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(name, code):
    if code != SPH_OK:
        raise SphError(name, code, load().sph_last_error().decode())
    return code


def _ref(s):
    return None if s is None else C.byref(s)


# Same names as the C ABI; arguments are the ctypes structs above, raw device
# pointers (int) and the stream handle (int).

def sph_version() -> str:
    return load().sph_version().decode()


def sph_workspace_size(grid: SphGrid, n_max: int, prec: int, material: int) -> int:
    return load().sph_workspace_size(C.byref(grid), n_max, prec, material)


def sph_build_cells(grid, inp, out, perm_ptr, cells, ws_ptr, ws_bytes, stream):
    return check("sph_build_cells", load().sph_build_cells(C.byref(grid), C.byref(inp), C.byref(out), perm_ptr,
                                                           cells, ws_ptr, ws_bytes, stream))


def sph_mark_boundary(grid, local, remote_cells, comm_ptr, bidx_ptr, cap, nb_ptr, nflag_ptr, ws_ptr, ws_bytes,
                      stream):
    return check("sph_mark_boundary", load().sph_mark_boundary(C.byref(grid), C.byref(local), remote_cells,
                                                               comm_ptr, bidx_ptr, cap, nb_ptr, nflag_ptr, ws_ptr,
                                                               ws_bytes, stream))


def sph_mark_boundary_noalloc(grid, local, remote_cells, comm_ptr, bidx_ptr, cap, nb_ptr, nflag_ptr, stream):
    return check("sph_mark_boundary_noalloc",
                 load().sph_mark_boundary_noalloc(C.byref(grid), C.byref(local), remote_cells, comm_ptr, bidx_ptr, cap,
                                                  nb_ptr, nflag_ptr, stream))


def sph_pack_boundary(local, bidx_ptr, nb_ptr, payload, stream):
    return check("sph_pack_boundary", load().sph_pack_boundary(C.byref(local), bidx_ptr, nb_ptr,
                                                               C.byref(payload), stream))


def sph_interact(params, grid, pass_, targets, tidx_ptr, nt_ptr, sources, source_cells, zero_first, rates,
                 ws_ptr, ws_bytes, stream):
    return check("sph_interact", load().sph_interact(C.byref(params), C.byref(grid), pass_, C.byref(targets),
                                                     tidx_ptr, nt_ptr, C.byref(sources), source_cells,
                                                     zero_first, C.byref(rates), ws_ptr, ws_bytes, stream))


def sph_count_pairs(params, grid, targets, tidx_ptr, nt_ptr, sources, source_cells, counts_ptr, stream):
    return check("sph_count_pairs", load().sph_count_pairs(C.byref(params), C.byref(grid), C.byref(targets),
                                                           tidx_ptr, nt_ptr, C.byref(sources), source_cells,
                                                           counts_ptr, stream))


def sph_set_pair_events(begin_event, end_event):
    """Measurement hook: hipEvent_t handles (int) recorded around every later
    pair-kernel launch; None, None stops it."""
    return check("sph_set_pair_events", load().sph_set_pair_events(begin_event or None, end_event or None))


def sph_neighbor_census(params, grid, pass_, targets, tidx_ptr, nt_ptr, sources, source_cells, count_ptr, sum_ptr,
                        ws_ptr, ws_bytes, stream):
    return check("sph_neighbor_census",
                 load().sph_neighbor_census(C.byref(params), C.byref(grid), pass_, C.byref(targets), tidx_ptr, nt_ptr,
                                            C.byref(sources), source_cells, count_ptr, sum_ptr, ws_ptr, ws_bytes,
                                            stream))


def sph_integrate(params, stage, p, rates, dt_ptr, diag_ptr, ws_ptr, ws_bytes, stream):
    return check("sph_integrate", load().sph_integrate(C.byref(params), stage, C.byref(p), _ref(rates), dt_ptr,
                                                       diag_ptr, ws_ptr, ws_bytes, stream))


def sph_interact_adjoint(params, grid, pass_, targets, tidx_ptr, nt_ptr, sources, source_cells, rbar_targets,
                         rbar_sources, bar, ws_ptr, ws_bytes, stream):
    return check("sph_interact_adjoint",
                 load().sph_interact_adjoint(C.byref(params), C.byref(grid), pass_, C.byref(targets), tidx_ptr, nt_ptr,
                                             C.byref(sources), source_cells, _ref(rbar_targets), _ref(rbar_sources),
                                             C.byref(bar), ws_ptr, ws_bytes, stream))


def sph_integrate_adjoint(params, stage, p, rates, dt_ptr, bar, rates_bar, pbar_ptr, ws_ptr, ws_bytes, stream):
    return check("sph_integrate_adjoint", load().sph_integrate_adjoint(C.byref(params), stage, C.byref(p),
                                                                       _ref(rates), dt_ptr, C.byref(bar),
                                                                       _ref(rates_bar), pbar_ptr, ws_ptr,
                                                                       ws_bytes, stream))


def sph_objective_adjoint(objective, p, tag_ptr, tag_len, ntag, scale, bar, stream):
    return check("sph_objective_adjoint", load().sph_objective_adjoint(objective, C.byref(p), tag_ptr, tag_len, ntag,
                                                                       float(scale), C.byref(bar), stream))


def sph_permute_adjoint(prec, n, perm_ptr, inp, out, stream):
    return check("sph_permute_adjoint", load().sph_permute_adjoint(prec, n, perm_ptr, C.byref(inp),
                                                                   C.byref(out), stream))


def sph_centroid(p, cg_ptr, ws_ptr, ws_bytes, stream):
    return check("sph_centroid", load().sph_centroid(C.byref(p), cg_ptr, ws_ptr, ws_bytes, stream))


def sph_balance_hash(p, cg_own_ptr, cg_other_ptr, hmax, bhash_ptr, npos_ptr, ws_ptr, ws_bytes, stream):
    return check("sph_balance_hash", load().sph_balance_hash(C.byref(p), cg_own_ptr, cg_other_ptr, hmax, bhash_ptr,
                                                             npos_ptr, ws_ptr, ws_bytes, stream))


def sph_balance_select(n, bhash_ptr, hmax, npos_own_ptr, npos_other_ptr, sel_ptr, k_ptr, ws_ptr, ws_bytes, stream):
    return check("sph_balance_select", load().sph_balance_select(n, bhash_ptr, hmax, npos_own_ptr, npos_other_ptr,
                                                                 sel_ptr, k_ptr, ws_ptr, ws_bytes, stream))


def sph_swap(a, sel_a_ptr, b, sel_b_ptr, k_ptr, k_max, stream):
    return check("sph_swap", load().sph_swap(C.byref(a), sel_a_ptr, C.byref(b), sel_b_ptr, k_ptr, k_max, stream))


def sph_centroid_types(p, type_ptr, ntypes, alpha, cg_ptr, ws_ptr, ws_bytes, stream):
    return check("sph_centroid_types", load().sph_centroid_types(C.byref(p), type_ptr, ntypes, alpha, cg_ptr,
                                                                 ws_ptr, ws_bytes, stream))


def sph_balance_hash_types(p, type_ptr, ntypes, cg_own_ptr, cg_other_ptr, hmax, bhash_ptr, npos_ptr, ws_ptr,
                           ws_bytes, stream):
    return check("sph_balance_hash_types",
                 load().sph_balance_hash_types(C.byref(p), type_ptr, ntypes, cg_own_ptr, cg_other_ptr, hmax,
                                               bhash_ptr, npos_ptr, ws_ptr, ws_bytes, stream))


def sph_balance_select_types(n, type_ptr, ntypes, bhash_ptr, hmax, npos_own_ptr, npos_other_ptr, sel_ptr, k_ptr,
                             off_ptr, ws_ptr, ws_bytes, stream):
    return check("sph_balance_select_types",
                 load().sph_balance_select_types(n, type_ptr, ntypes, bhash_ptr, hmax, npos_own_ptr, npos_other_ptr,
                                                 sel_ptr, k_ptr, off_ptr, ws_ptr, ws_bytes, stream))
