"""Brute-force O(N^2) references written straight from the definitions.

They use no bucket grid for the neighbour predicate, so they check the
oracle's bucket search for completeness and exactness (Section I: a particle's
neighbours lie in its own or the surrounding buckets), and the
communication-hash predicate of Section II (step c) over all
(local, remote) pairs.
"""
from __future__ import annotations

import numpy as np


def neighbor_pairs(x_t: np.ndarray, x_s: np.ndarray, h: float, self_pass: bool):
    """Set of (i, j) with 0 < ((dx^2 + dy^2) + dz^2) < (2h)^2, j != i when self_pass."""
    R = 2.0 * h
    R2 = R * R
    out = set()
    for i in range(x_t.shape[0]):
        d = x_s - x_t[i]
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        js = np.flatnonzero((r2 < R2) & (r2 > 0.0))
        for j in js:
            if self_pass and j == i:
                continue
            out.add((i, int(j)))
    return out


def cells_of(grid: dict, x: np.ndarray) -> np.ndarray:
    """Integer bucket coordinates with clamping, from floor((x - o) / L)."""
    o = np.asarray(grid["origin"], dtype=np.float64)
    n = np.asarray(grid["dims"], dtype=np.int64)
    c = np.floor((x - o) / grid["cell"]).astype(np.int64)
    return np.clip(c, 0, n - 1)


def boundary_flags(grid: dict, x_local: np.ndarray, x_remote: np.ndarray) -> np.ndarray:
    """flag_i = exists remote j whose bucket differs from i's by at most 1 on every axis."""
    cl = cells_of(grid, x_local)
    cr = cells_of(grid, x_remote)
    flags = np.zeros(x_local.shape[0], dtype=bool)
    if cr.shape[0] == 0:
        return flags
    occupied = {tuple(c) for c in cr}
    for i, c in enumerate(cl):
        hit = False
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (c[0] + dx, c[1] + dy, c[2] + dz) in occupied:
                        hit = True
                        break
                if hit:
                    break
            if hit:
                break
        flags[i] = hit
    return flags
