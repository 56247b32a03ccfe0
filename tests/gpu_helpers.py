"""Helpers for GPU parity tests: convert device state to the oracle's layout
and compare with stated tolerances."""
from __future__ import annotations

import numpy as np

import sph_synth as S
from oracle import cpu


def oracle_state(h: dict, solid: bool) -> cpu.State:
    """Oracle state holding exactly the values the device holds (array order)."""
    s = cpu.State(h["x"].shape[0], solid)
    s.x[:] = h["x"]
    s.v[:] = h["v"]
    s.m[:] = h["m"]
    s.w[:] = h["w"]
    s.rho[:] = h["rho"]
    s.p[:] = h["p"]
    s.c[:] = h["c"]
    s.E[:] = h["E"]
    s.id[:] = h["id"]
    s.hash[:] = h["hash"]
    if solid:
        s.S[:] = h["S"]
        s.ep[:] = h["ep"]
    return s


def assert_close_scaled(got, ref, scale, rtol, what=""):
    """|got - ref| <= rtol * scale elementwise (scale: per-entry round-off scale)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref)
    bound = rtol * np.asarray(scale, dtype=np.float64) + 1e-300
    bad = ~(err <= bound)   # a NaN on either side fails
    if bad.any():
        idx = np.argwhere(bad)[:5]
        ratio = (err / np.maximum(scale, 1e-300)).max()
        raise AssertionError(f"{what}: {bad.sum()} entries exceed {rtol} x scale (worst err/scale {ratio:.3e}); "
                             f"first {idx.tolist()} got {got[tuple(idx[0])]} ref {ref[tuple(idx[0])]}")


# Round-off bound of a pair sum: rtol of B plus rtol_edge of B_peak.  B sums
# the oracle's magnitude bound of every term (inputs in absolute value,
# differences as sums, |n_k| -> 1), which bounds both the rounding of the
# term's ~30 operations and a relative perturbation of positions or
# velocities; B_peak is the same with every pair at the kernel's peak
# strength, covering the support edge where F ~ (2 - q)^2 turns a one-ulp
# change of q (FP64) or a float-offset rounding of r (FP32) into a large
# relative change of a vanishing term, and a pair within round-off of r = 2h.
RATE_TOL = {0: (1e-13, 1e-14), 1: (2e-5, 2e-6)}


def rate_bound(params, grid, pass_, tg, src, start, self_pass, prec, tidx=None):
    rtol, rtol_edge = RATE_TOL[prec]
    a = cpu.interact_abs(params, grid, pass_, tg, src, start, self_pass, tidx=tidx)
    b = cpu.interact_abs(params, grid, pass_, tg, src, start, self_pass, tidx=tidx, peak=True)
    return rtol * a + rtol_edge * b


def assert_within(got, ref, bound, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref)
    bad = ~(err <= bound + 1e-300)   # a NaN on either side fails
    if bad.any():
        idx = np.argwhere(bad)[:5]
        ratio = (err / np.maximum(bound, 1e-300)).max()
        raise AssertionError(f"{what}: {bad.sum()} entries exceed the bound (worst err/bound {ratio:.3e}); "
                             f"first {idx.tolist()} got {got[tuple(idx[0])]} ref {ref[tuple(idx[0])]}")


def pressure_scale(params: dict) -> float:
    """Scale of the terms whose difference is p: gamma B for Tait (p = B (s^gamma - 1)
    cancels near s = 1), K for the linear solid EOS, rho0 c0^2 for Mie-Gruneisen."""
    if params["material"] == S.FLUID_TAIT:
        return params["gamma"] * params["rho0"] * params["c0"] ** 2 / params["gamma"]
    if params.get("eos", S.EOS_LINEAR) == S.EOS_MIE_GRUNEISEN:
        return params["rho0"] * params["c0"] ** 2
    return params["K"]


def field_errors(gpu: dict, ref: cpu.State, fields=("x", "v", "m", "w", "rho", "p", "c", "E"),
                 scales=None) -> dict:
    """max |gpu - ref| / scale per field, rows matched by array position; the scale
    is max |ref| unless ``scales`` gives one."""
    out = {}
    scales = scales or {}
    for f in fields:
        a = np.asarray(gpu[f], dtype=np.float64)
        b = np.asarray(getattr(ref, f), dtype=np.float64)
        den = scales.get(f, np.abs(b).max())
        out[f] = float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())
    return out


def dense_cell_cloud(n: int, seed: int) -> S.Workload:
    """Many particles packed into a few buckets (long candidate rows)."""
    w = S.random_cloud(n, seed=seed, h=0.05, box=1.0)
    w.x = 0.45 + 0.1 * (w.x - 0.0)          # all inside [0.45, 0.55]^3 -> ~3^3 buckets of side 0.1
    return w
