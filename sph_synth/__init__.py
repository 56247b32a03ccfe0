"""Seeded synthetic inputs for the particle-decomposition SPH hot path.

This module is shared by the CPU oracle, the tests, the HIP binding's
drivers and the benchmark.  It only draws and lays out input particles and
states the physical constants of each workload; it performs none of the
method's arithmetic (no hashing, sorting, kernel, flux or update).

Every workload follows one recipe: particles on a regular lattice with
spacing ``dx`` at cell-centred sites ``(i + 1/2) dx``, optional uniform
jitter, a velocity field, a density field, ``omega = dx^3`` (particle
volume), ``m = rho * omega`` and total specific energy ``E = e + |v|^2 / 2``
with internal energy ``e = 0``.  The smoothing length is one value for all
particles, ``h = 1.3 dx``, as the particle decomposition assumes a constant
smoothing length (Section II); the bucket side is ``2h`` (Section I).

Random draws use ``numpy.random.default_rng(seed)`` in the order documented
in each function, so any two consumers see bit-identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

FLUID_TAIT = 0
SOLID_J2 = 1
EOS_LINEAR, EOS_MIE_GRUNEISEN = 0, 1


@dataclass
class Workload:
    """One synthetic input: particle arrays (id order) plus physical constants.

    Arrays: ``x`` (n,3) f64 positions, ``v`` (n,3) f64 velocities, ``m``,
    ``omega``, ``rho``, ``E`` (n,) f64, ``id`` (n,) u32.  Solids also carry
    ``S`` (n,6) deviatoric stress (xx, yy, zz, xy, xz, yz) and ``eps_p`` (n,).
    ``grid`` is (origin[3], cell, dims[3]); ``params`` the constants.
    """

    name: str
    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    omega: np.ndarray
    rho: np.ndarray
    E: np.ndarray
    id: np.ndarray
    grid: dict
    params: dict
    S: np.ndarray | None = None
    eps_p: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, mask: np.ndarray, name: str | None = None) -> "Workload":
        """Particles selected by ``mask``, keeping their ids."""
        def pick(a):
            return None if a is None else np.ascontiguousarray(a[mask])
        return Workload(name or self.name, pick(self.x), pick(self.v), pick(self.m),
                        pick(self.omega), pick(self.rho), pick(self.E), pick(self.id),
                        dict(self.grid), dict(self.params), pick(self.S), pick(self.eps_p),
                        dict(self.extra))


def _lattice(nx: int, ny: int, nz: int, dx: float, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Cell-centred lattice sites, x index fastest."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = np.empty((nx * ny * nz, 3))
    x[:, 0] = origin[0] + (ix.ravel() + 0.5) * dx
    x[:, 1] = origin[1] + (iy.ravel() + 0.5) * dx
    x[:, 2] = origin[2] + (iz.ravel() + 0.5) * dx
    return x


def make_grid(lo, hi, cell: float) -> dict:
    """Bucket grid of side ``cell`` covering the box [lo, hi]."""
    lo = [float(a) for a in lo]
    dims = [int(math.ceil((float(b) - a) / cell)) for a, b in zip(lo, hi)]
    dims = [max(d, 1) for d in dims]
    return {"origin": lo, "cell": float(cell), "dims": dims}


def fluid_params(h, rho0=1000.0, c0=50.0, gamma=7.0, cfl=0.3, gravity=(0.0, 0.0, 0.0),
                 wall_lo=(0.0, 0.0, 0.0), wall_hi=(0.0, 0.0, 0.0), wall_mask=0, beta=1.0):
    return {"h": float(h), "rho0": rho0, "c0": c0, "gamma": gamma, "K": 0.0, "G": 0.0,
            "Y0": 0.0, "H": 0.0, "beta": beta, "cfl": cfl, "gravity": list(gravity),
            "wall_lo": list(wall_lo), "wall_hi": list(wall_hi), "wall_mask": int(wall_mask),
            "material": FLUID_TAIT}


def _fluid_state(x, v, rho, dx, wid=None):
    n = x.shape[0]
    omega = np.full(n, dx ** 3)
    m = rho * omega
    E = 0.5 * np.einsum("ij,ij->i", v, v)
    ids = np.arange(n, dtype=np.uint32) if wid is None else wid
    return omega, m, E, ids


ALL_WALLS = 0x3F


def c1_cube(seed: int = 1, n_side: int = 20, dx: float = 1e-3) -> Workload:
    """Jittered cube of n_side^3 fluid particles in a reflective box.

    Draw order: jitter U(-0.05dx, 0.05dx) (n,3), then v ~ N(0, 0.5^2) (n,3).
    Box [0, n_side*dx]^3, rho0 = 1000, c0 = 50, gamma = 7, CFL 0.3, no gravity.
    """
    rng = np.random.default_rng(seed)
    x = _lattice(n_side, n_side, n_side, dx)
    x += rng.uniform(-0.05 * dx, 0.05 * dx, size=x.shape)
    v = rng.normal(0.0, 0.5, size=x.shape)
    rho = np.full(x.shape[0], 1000.0)
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    h = 1.3 * dx
    ext = n_side * dx
    p = fluid_params(h, c0=50.0, wall_lo=(0, 0, 0), wall_hi=(ext, ext, ext), wall_mask=ALL_WALLS)
    g = make_grid((0, 0, 0), (ext, ext, ext), 2 * h)
    return Workload("cube", x, v, m, omega, rho, E, ids, g, p, extra={"dx": dx, "steps": 10})


def c2_column(nx: int = 74, ny: int = 74, nz: int = 148, dx: float = 5.4e-3,
              box=(1.6, 0.4, 0.8), c0: float = 40.0) -> Workload:
    """Water column (nx*dx, ny*dx, nz*dx) at rest in the corner of a reflective box.

    No random draws.  Hydrostatic start: the density whose Tait pressure
    balances the weight of the water above, rho = rho0 (1 + rho0 g (Hc - z) / B)^(1/gamma)
    with B = rho0 c0^2 / gamma and Hc the column height; gravity -9.81 z.
    """
    x = _lattice(nx, ny, nz, dx)
    rho0, gamma, gz = 1000.0, 7.0, 9.81
    B = rho0 * c0 * c0 / gamma
    Hc = nz * dx
    rho = rho0 * (1.0 + rho0 * gz * (Hc - x[:, 2]) / B) ** (1.0 / gamma)
    v = np.zeros_like(x)
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    h = 1.3 * dx
    p = fluid_params(h, c0=c0, gravity=(0.0, 0.0, -gz), wall_lo=(0, 0, 0), wall_hi=box,
                     wall_mask=ALL_WALLS)
    g = make_grid((0, 0, 0), box, 2 * h)
    return Workload("column", x, v, m, omega, rho, E, ids, g, p, extra={"dx": dx, "steps": 1000})


def c3_cylinder(dx: float = 1.5777e-4, radius: float = 0.01, nlayers: int = 316,
                vz: float = -200.0) -> Workload:
    """Elastic-plastic cylinder moving at vz onto a rigid wall at z = 0.

    No random draws.  Lattice sites (i + 1/2) dx in x, y (symmetric about the
    axis) kept where x^2 + y^2 <= radius^2, layers z = (k + 1/2) dx.
    rho0 = 2700, E = 70 GPa, nu = 0.33, Y0 = 300 MPa, linear hardening
    modulus H = E / 100 (a stated choice; the workload gives none).
    """
    nr = int(math.ceil(radius / dx)) + 1
    c = (np.arange(-nr, nr) + 0.5) * dx
    X, Y = np.meshgrid(c, c, indexing="ij")
    keep = (X * X + Y * Y) <= radius * radius
    # x index fastest within a layer
    xy = np.stack([X.T[keep.T], Y.T[keep.T]], axis=1)
    nxy = xy.shape[0]
    x = np.empty((nxy * nlayers, 3))
    for k in range(nlayers):
        x[k * nxy:(k + 1) * nxy, :2] = xy
        x[k * nxy:(k + 1) * nxy, 2] = (k + 0.5) * dx
    v = np.zeros_like(x)
    v[:, 2] = vz
    rho0 = 2700.0
    Ey, nu = 70e9, 0.33
    K = Ey / (3.0 * (1.0 - 2.0 * nu))
    G = Ey / (2.0 * (1.0 + nu))
    rho = np.full(x.shape[0], rho0)
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    h = 1.3 * dx
    p = {"h": h, "rho0": rho0, "c0": math.sqrt((K + 4.0 * G / 3.0) / rho0), "gamma": 1.0,
         "K": K, "G": G, "Y0": 300e6, "H": Ey / 100.0, "beta": 1.0, "cfl": 0.3,
         "gravity": [0.0, 0.0, 0.0], "wall_lo": [0.0, 0.0, 0.0], "wall_hi": [0.0, 0.0, 0.0],
         "wall_mask": 1 << 4, "material": SOLID_J2}
    g = make_grid((-0.012, -0.012, 0.0), (0.012, 0.012, 0.051), 2 * h)
    n = x.shape[0]
    return Workload("cylinder", x, v, m, omega, rho, E, ids, g, p, S=np.zeros((n, 6)),
                    eps_p=np.zeros(n), extra={"dx": dx, "steps": 500})


def c4_share(layout: str = "slab", seed: int = 4, nx: int = 250, ny: int = 200, nz: int = 200,
             dx: float = 1e-3, split_ix: int = 200, mix_p: float = 0.30):
    """One GPU's share of a 16-GPU particle decomposition: (local, remote).

    Lattice nx*ny*nz with jitter.  ``slab``: local = {ix < split_ix},
    remote = {ix >= split_ix}.  ``mixed``: sites are selected with
    probability mix_p and the owner labels are permuted among the selected
    sites, so the local and remote counts are those of the slab.
    Draw order: jitter (n,3); v ~ N(0, 0.5^2) (n,3); density noise N(0,1) (n,);
    selection U(0,1) (n,); permutation of the selected labels; remote owner
    labels U{1..15}.  rho = rho0 (1 + 1e-3 noise).
    """
    rng = np.random.default_rng(seed)
    x = _lattice(nx, ny, nz, dx)
    x += rng.uniform(-0.05 * dx, 0.05 * dx, size=x.shape)
    v = rng.normal(0.0, 0.5, size=x.shape)
    rho = 1000.0 * (1.0 + 1e-3 * rng.normal(0.0, 1.0, size=x.shape[0]))
    n = x.shape[0]
    ix = np.arange(n) % nx
    is_local = ix < split_ix
    sel = rng.uniform(0.0, 1.0, size=n) < mix_p
    if layout == "mixed":
        idx = np.flatnonzero(sel)
        labels = is_local[idx]
        is_local = is_local.copy()
        is_local[idx] = labels[rng.permutation(idx.size)]
    elif layout != "slab":
        raise ValueError(layout)
    owner = rng.integers(1, 16, size=n).astype(np.uint8)
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    h = 1.3 * dx
    p = fluid_params(h, c0=50.0)
    g = make_grid((0, 0, 0), (nx * dx, ny * dx, nz * dx), 2 * h)
    full = Workload(f"share-{layout}", x, v, m, omega, rho, E, ids, g, p, extra={"dx": dx})
    local = full.subset(is_local, f"share-{layout}-local")
    remote = full.subset(~is_local, f"share-{layout}-remote")
    remote.extra["owner"] = owner[~is_local]
    return local, remote


def c6_hvi(dx: float = 6.5e-5, plate_half: float = 0.015, plate_t: float = 2e-3, bead_r: float = 1.5e-3,
           speed: float = 4050.0, tilt_deg: float = 32.0) -> Workload:
    """Hypervelocity impact in the style of Section IV.A: an aluminium bead
    (radius 1.5 mm) at 4.05 km/s, tilted 32 degrees from the plate normal,
    onto a 2 mm aluminium plate.  With the defaults (65 um lattice, plate
    30 x 30 mm) about 6.5 million particles, the paper's count.

    No random draws.  Plate: cubic lattice (i + 1/2) dx in
    [-plate_half, plate_half]^2 x [0, plate_t]; bead: lattice points within
    bead_r of its centre, placed 1.5 dx above the plate along z and shifted
    back along the flight path.  Material (stated choices; the paper gives
    none): rho0 = 2700, bulk c0 = 5350 m/s, Us-up slope 1.34, Gamma0 = 2.0,
    G = 26.3 GPa, Y0 = 300 MPa elastic perfectly plastic (H = 0), spall
    cut-off -1.2 GPa.  extra["types"]: 0 plate, 1 bead.
    """
    n_xy = int(round(2 * plate_half / dx))
    n_z = int(round(plate_t / dx))
    g = (np.arange(n_xy) + 0.5) * dx - plate_half
    gz = (np.arange(n_z) + 0.5) * dx
    Z, Y, X = np.meshgrid(gz, g, g, indexing="ij")      # x fastest
    plate = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    t = math.radians(tilt_deg)
    rise = bead_r + 1.5 * dx
    centre = np.array([-math.tan(t) * rise, 0.0, plate_t + rise])
    nb = int(math.ceil(bead_r / dx)) + 1
    b = (np.arange(-nb, nb) + 0.5) * dx
    Zb, Yb, Xb = np.meshgrid(b, b, b, indexing="ij")
    bead = np.stack([Xb.ravel(), Yb.ravel(), Zb.ravel()], axis=1)
    bead = bead[np.linalg.norm(bead, axis=1) <= bead_r] + centre
    x = np.concatenate([plate, bead])
    v = np.zeros_like(x)
    v[plate.shape[0]:] = speed * np.array([math.sin(t), 0.0, -math.cos(t)])
    rho0 = 2700.0
    rho = np.full(x.shape[0], rho0)
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    h = 1.3 * dx
    p = {"h": h, "rho0": rho0, "c0": 5350.0, "gamma": 1.0, "K": 0.0, "G": 26.3e9, "Y0": 300e6, "H": 0.0,
         "beta": 1.0, "cfl": 0.3, "gravity": [0.0, 0.0, 0.0], "wall_lo": [0.0, 0.0, 0.0],
         "wall_hi": [0.0, 0.0, 0.0], "wall_mask": 0, "material": SOLID_J2, "eos": EOS_MIE_GRUNEISEN,
         "mg_s": 1.34, "mg_gamma0": 2.0, "p_cut": -1.2e9}
    lo = (-plate_half - 2 * dx, -plate_half - 2 * dx, -plate_t)
    hi = (plate_half + 2 * dx, plate_half + 2 * dx, plate_t + 2 * rise + 2 * dx)
    grid = make_grid(lo, hi, 2 * h)
    n = x.shape[0]
    types = np.concatenate([np.zeros(plate.shape[0], np.uint8), np.ones(bead.shape[0], np.uint8)])
    return Workload("hvi", x, v, m, omega, rho, E, ids, grid, p, S=np.zeros((n, 6)), eps_p=np.zeros(n),
                    extra={"dx": dx, "steps": 20, "types": types})


def particle_types(x: np.ndarray, centre, radius: float, seed: int = 0, p_third: float = 0.0) -> np.ndarray:
    """Type labels (u8) for the per-type balancing: 1 inside a sphere (a bead,
    like the projectile of a hypervelocity impact), 0 outside; with
    p_third > 0 a uniformly drawn fraction of all particles gets type 2.
    Draw order: U(0,1) (n,)."""
    x = np.asarray(x)
    t = (np.linalg.norm(x - np.asarray(centre, dtype=np.float64), axis=1) < radius).astype(np.uint8)
    if p_third > 0.0:
        rng = np.random.default_rng(seed)
        t[rng.uniform(0.0, 1.0, size=x.shape[0]) < p_third] = 2
    return t


def c5_box(seed: int = 5, n_side: int = 63, dx: float = 2e-3, margin_cells: int = 2) -> Workload:
    """Free fluid box for the adjoint: n_side^3 jittered lattice, v ~ N(0, 1).

    Draw order: jitter (n,3), then v (n,3).  c0 = 50, free boundaries,
    fixed dt = 1.4e-5 s.  The bucket grid is the lattice box widened by
    ``margin_cells`` buckets on every side and held fixed.
    """
    rng = np.random.default_rng(seed)
    x = _lattice(n_side, n_side, n_side, dx)
    x += rng.uniform(-0.05 * dx, 0.05 * dx, size=x.shape)
    v = rng.normal(0.0, 1.0, size=x.shape)
    rho = np.full(x.shape[0], 1000.0)
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    h = 1.3 * dx
    L = 2 * h
    ext = n_side * dx
    p = fluid_params(h, c0=50.0)
    g = make_grid((-margin_cells * L,) * 3, (ext + margin_cells * L,) * 3, L)
    return Workload("adjoint-box", x, v, m, omega, rho, E, ids, g, p,
                    extra={"dx": dx, "dt": 1.4e-5, "steps": 50, "ckpt": 10})


def random_cloud(n: int, seed: int, box=1.0, h: float = 0.05, v_sigma: float = 0.5,
                 rho_sigma: float = 0.0) -> Workload:
    """Uniform random particles in [0, box]^3 (draws: x, v, density noise)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, box, size=(n, 3))
    v = rng.normal(0.0, v_sigma, size=(n, 3))
    rho = 1000.0 * (1.0 + rho_sigma * rng.normal(0.0, 1.0, size=n))
    dx = box / max(round(n ** (1.0 / 3.0)), 1)
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    p = fluid_params(h, c0=50.0)
    g = make_grid((0, 0, 0), (box, box, box), 2 * h)
    return Workload("cloud", x, v, m, omega, rho, E, ids, g, p, extra={"dx": dx})


def jittered_lattice(n_side: int, seed: int, dx: float = 1e-3, jitter: float = 0.05,
                     v_sigma: float = 0.5, rho_sigma: float = 0.0, c0: float = 50.0,
                     walls: bool = False, dims=None) -> Workload:
    """Small jittered lattice (draws: jitter, v, density noise)."""
    nx, ny, nz = dims if dims is not None else (n_side, n_side, n_side)
    rng = np.random.default_rng(seed)
    x = _lattice(nx, ny, nz, dx)
    x += rng.uniform(-jitter * dx, jitter * dx, size=x.shape)
    v = rng.normal(0.0, v_sigma, size=x.shape)
    rho = 1000.0 * (1.0 + rho_sigma * rng.normal(0.0, 1.0, size=x.shape[0]))
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    h = 1.3 * dx
    hi = (nx * dx, ny * dx, nz * dx)
    p = fluid_params(h, c0=c0, wall_lo=(0, 0, 0), wall_hi=hi,
                     wall_mask=ALL_WALLS if walls else 0)
    g = make_grid((0, 0, 0), hi, 2 * h)
    return Workload("lattice", x, v, m, omega, rho, E, ids, g, p, extra={"dx": dx})


def solid_block(n_side: int, seed: int, dx: float = 1e-3, vz: float = -50.0,
                s_sigma: float = 0.0, s_axial: float = 0.0, stretch_rate: float = 0.0) -> Workload:
    """Small jittered block of C3's material moving onto the z = 0 wall.

    Draws: jitter (n,3), velocity perturbation N(0, 1) (n,3), stress N(0, s_sigma) (n,6).
    Optional, no draws: a uniaxial deviatoric stress s_axial diag(2/3, -1/3, -1/3)
    (von Mises stress s_axial) added to S, and an isochoric stretch along x,
    v += stretch_rate (x - xc, -(y - yc) / 2, -(z - zc) / 2), which raises it.
    """
    rng = np.random.default_rng(seed)
    x = _lattice(n_side, n_side, n_side, dx)
    x += rng.uniform(-0.05 * dx, 0.05 * dx, size=x.shape)
    v = rng.normal(0.0, 1.0, size=x.shape)
    v[:, 2] += vz
    S = rng.normal(0.0, s_sigma, size=(x.shape[0], 6)) if s_sigma > 0 else np.zeros((x.shape[0], 6))
    # deviatoric: remove the trace
    tr = (S[:, 0] + S[:, 1] + S[:, 2]) / 3.0
    S[:, :3] -= tr[:, None]
    if s_axial:
        S[:, :3] += s_axial * np.array([2.0 / 3.0, -1.0 / 3.0, -1.0 / 3.0])
    if stretch_rate:
        xc = x.mean(0)
        v += stretch_rate * (x - xc) * np.array([1.0, -0.5, -0.5])
    w = c3_cylinder(dx=dx, radius=2 * dx, nlayers=2)
    rho = np.full(x.shape[0], w.params["rho0"])
    omega, m, E, ids = _fluid_state(x, v, rho, dx)
    p = dict(w.params)
    p["h"] = 1.3 * dx
    ext = n_side * dx
    g = make_grid((-2 * dx, -2 * dx, 0.0), (ext + 2 * dx, ext + 2 * dx, ext + 2 * dx), 2.6 * dx)
    return Workload("solid-block", x, v, m, omega, rho, E, ids, g, p, S=S,
                    eps_p=np.zeros(x.shape[0]), extra={"dx": dx})
