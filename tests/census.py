"""Expected neighbour census of an interaction pass, from the definition.

Section I puts every neighbour of a particle (|x_j - x_i| < 2h) in its own
bucket or the 26 around it; the pair kernel finds them through a staged,
filtered search.  ``sph_neighbor_census`` reports, per target, how many
sources that search evaluates and a checksum of their ids (the sum modulo
2^64 of SplitMix64 of each id).  This module computes the same two numbers
from positions alone: candidates within a slightly larger radius from a k-d
tree (a library primitive that only proposes pairs), then the predicate
r^2 = ((dx dx + dy dy) + dz dz) < (2h)^2 evaluated left to right in FP64, as
the neighbour set is defined.  Pairs at r = 0 (the target itself in a
local-local pass, coincident particles) are evaluated by the pass and add
exactly zero; they are counted here too.

For the FP32-split form, whose position differences are rebuilt from float
offsets, a pair with |r / 2h - 1| below ``window`` may fall on either side;
``match`` then looks for the subset of those ambiguous pairs that reproduces
the device's count and checksum, and reports how many pairs differ.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.spatial import cKDTree

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def mix64(ids) -> np.ndarray:
    """SplitMix64 output function of each id (Steele, Lea and Flood 2014)."""
    with np.errstate(over="ignore"):
        z = np.asarray(ids, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sum64(values) -> int:
    """Sum modulo 2^64 of uint64 values."""
    return int(np.sum(np.asarray(values, dtype=np.uint64), dtype=np.uint64)) if len(values) else 0


class Expected:
    """Per-target sets: ``core`` (in the set whatever the rounding of r) and
    ``amb`` (|r / 2h - 1| < window), as arrays of source indices."""

    def __init__(self, core, amb, amb_in):
        self.core = core
        self.amb = amb
        self.amb_in = amb_in   # per ambiguous pair: whether FP64 puts it inside


def expected(x_t: np.ndarray, x_s: np.ndarray, h: float, window: float = 0.0) -> Expected:
    """Neighbour sets of the targets x_t among the sources x_s."""
    R = 2.0 * h
    R2 = R * R
    tree = cKDTree(x_s)
    cand = tree.query_ball_point(x_t, R * (1.0 + window) * (1.0 + 1e-9) + 1e-300)
    core, amb, amb_in = [], [], []
    for i, js in enumerate(cand):
        js = np.asarray(sorted(js), dtype=np.int64)
        d = x_s[js] - x_t[i]
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        inside = r2 < R2
        if window > 0.0:
            near = np.abs(np.sqrt(r2) / R - 1.0) < window
        else:
            near = np.zeros(js.shape, dtype=bool)
        core.append(js[inside & ~near])
        amb.append(js[near])
        amb_in.append(inside[near])
    return Expected(core, amb, amb_in)


def match(count: int, checksum: int, core_ids: np.ndarray, amb_ids: np.ndarray, amb_in: np.ndarray,
          max_amb: int = 12):
    """Number of pairs by which the device's set differs from the FP64 set,
    or None when no subset of the ambiguous pairs reproduces the device's
    count and checksum (a lost or extra neighbour)."""
    base_n = len(core_ids)
    base_s = sum64(mix64(core_ids))
    mixed_amb = [int(v) for v in mix64(amb_ids)]
    k = len(amb_ids)
    if k > max_amb:
        raise ValueError(f"{k} ambiguous pairs for one target")
    for size in range(k + 1):
        if base_n + size != count:
            continue
        for sub in itertools.combinations(range(k), size):
            s = (base_s + sum(mixed_amb[q] for q in sub)) & 0xFFFFFFFFFFFFFFFF
            if s == checksum:
                chosen = np.zeros(k, dtype=bool)
                chosen[list(sub)] = True
                return int(np.sum(chosen != np.asarray(amb_in, dtype=bool)))
    return None
