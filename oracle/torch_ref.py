"""Dense float64 PyTorch (CPU) forward of the fluid step, for reverse mode.

TEST INFRASTRUCTURE ONLY (part of the oracle).  It evaluates the same
reading of the scheme as sph_oracle.c (all pairs with 0 < r < 2h, cubic
spline, acoustic Riemann solver, symplectic Euler, Tait EOS; free
boundaries, no gravity, fixed dt), written directly on (N, N) pair tensors
so that torch.autograd differentiates it.  Small N only (O(N^2) memory).
Its gradient of the kinetic energy after a few steps is the reverse-mode
reference for the hand adjoint.
"""
from __future__ import annotations

import math

import torch


def kernel_F(r, h):
    """-dW/dr of the cubic spline with sigma = 1 / (pi h^3) (0 outside 2h)."""
    q = r / h
    s = 1.0 / (math.pi * h ** 3)
    inner = s * (3.0 * q - 2.25 * q * q) / h
    t = torch.clamp(2.0 - q, min=0.0)
    outer = s * 0.75 * t * t / h
    return torch.where(q < 1.0, inner, outer)


def eos(rho, P, c0):
    s = rho / P["rho0"]
    B = P["rho0"] * c0 * c0 / P["gamma"]
    p = B * (s ** P["gamma"] - 1.0)
    c = c0 * s ** (0.5 * (P["gamma"] - 1.0))
    return p, c


def rates(x, v, m, w, E, P, c0):
    """(mdot, mvdot (n,3), mEdot, wdot) summed over all pairs with 0 < r < 2h."""
    h = P["h"]
    rho = m / w
    p, c = eos(rho, P, c0)
    e = E - 0.5 * (v * v).sum(1)
    d = x[None, :, :] - x[:, None, :]                    # d[i, j] = x_j - x_i
    r2 = (d * d).sum(-1)
    R = 2.0 * h
    mask = (r2 < R * R) & (r2 > 0.0)
    r = torch.sqrt(torch.where(mask, r2, torch.ones_like(r2)))
    F = torch.where(mask, kernel_F(r, h), torch.zeros_like(r))
    n = d / r[..., None]
    g = F[..., None] * n
    ui = (v[:, None, :] * n).sum(-1)
    uj = (v[None, :, :] * n).sum(-1)
    rb = 0.5 * (rho[:, None] + rho[None, :])
    cb = 0.5 * (c[:, None] + c[None, :])
    pb = 0.5 * (p[:, None] + p[None, :])
    Z = rb * cb
    beta = P["beta"]
    du = beta * (p[:, None] - p[None, :]) / (2.0 * Z)
    ps = pb + beta * Z * (ui - uj) * 0.5
    vs = 0.5 * (v[:, None, :] + v[None, :, :]) + du[..., None] * n
    Es = 0.5 * (e[:, None] + e[None, :]) + 0.5 * (vs * vs).sum(-1)
    A = 2.0 * w[:, None] * w[None, :]
    Phi = rb * du * F
    t = ps[..., None] * g
    mdot = (-A * Phi).sum(1)
    mvdot = (-A[..., None] * (Phi[..., None] * vs + t)).sum(1)
    mEdot = (-A * (Phi * Es + (t * vs).sum(-1))).sum(1)
    wdot = (w[:, None] * w[None, :] * ((v[None, :, :] - v[:, None, :]) * g).sum(-1)).sum(1)
    return mdot, mvdot, mEdot, wdot


def step(x, v, m, w, E, P, c0, dt):
    mdot, mvdot, mEdot, wdot = rates(x, v, m, w, E, P, c0)
    mn = m + dt * mdot
    vn = (m[:, None] * v + dt * mvdot) / mn[:, None]
    En = (m * E + dt * mEdot) / mn
    wn = w + dt * wdot
    xn = x + dt * vn
    return xn, vn, mn, wn, En


def kinetic_energy_after(x0, v0, m0, w0, e0, P, c0, dt, nsteps):
    """J = sum m |v|^2 / 2 after nsteps, with E0 = e0 + |v0|^2 / 2."""
    x, v, m, w = x0, v0, m0, w0
    E = e0 + 0.5 * (v0 * v0).sum(1)
    for _ in range(nsteps):
        x, v, m, w, E = step(x, v, m, w, E, P, c0, dt)
    return 0.5 * (m * (v * v).sum(1)).sum()


def gradient(wl, c0, dt, nsteps):
    """(J, dJ/dv0 (n,3), dJ/dc0) by reverse mode, float64."""
    x0 = torch.tensor(wl.x, dtype=torch.float64)
    v0 = torch.tensor(wl.v, dtype=torch.float64, requires_grad=True)
    m0 = torch.tensor(wl.m, dtype=torch.float64)
    w0 = torch.tensor(wl.omega, dtype=torch.float64)
    e0 = torch.tensor(wl.E - 0.5 * (wl.v * wl.v).sum(1), dtype=torch.float64)
    c = torch.tensor(float(c0), dtype=torch.float64, requires_grad=True)
    J = kinetic_energy_after(x0, v0, m0, w0, e0, wl.params, c, dt, nsteps)
    gv, gc = torch.autograd.grad(J, (v0, c))
    return float(J.detach()), gv.numpy(), float(gc)


def z_displacement_after(x0, v0, m0, w0, e0, P, c0, dt, nsteps, tag):
    """J = mean over the tagged rows of (z after nsteps - z0)."""
    x, v, m, w = x0, v0, m0, w0
    E = e0 + 0.5 * (v0 * v0).sum(1)
    for _ in range(nsteps):
        x, v, m, w, E = step(x, v, m, w, E, P, c0, dt)
    return (x[tag, 2] - x0[tag, 2]).mean()


def gradient_z_displacement(wl, c0, dt, nsteps, tag):
    """(J, dJ/dv0 (n,3), dJ/dc0) of the tagged mean z-displacement, float64."""
    x0 = torch.tensor(wl.x, dtype=torch.float64)
    v0 = torch.tensor(wl.v, dtype=torch.float64, requires_grad=True)
    m0 = torch.tensor(wl.m, dtype=torch.float64)
    w0 = torch.tensor(wl.omega, dtype=torch.float64)
    e0 = torch.tensor(wl.E - 0.5 * (wl.v * wl.v).sum(1), dtype=torch.float64)
    c = torch.tensor(float(c0), dtype=torch.float64, requires_grad=True)
    t = torch.as_tensor(tag, dtype=torch.int64)
    J = z_displacement_after(x0, v0, m0, w0, e0, wl.params, c, dt, nsteps, t)
    gv, gc = torch.autograd.grad(J, (v0, c))
    return float(J.detach()), gv.numpy(), float(gc)


def final_state(wl, c0, dt, nsteps):
    """State after nsteps (id order) as numpy arrays."""
    with torch.no_grad():
        x = torch.tensor(wl.x, dtype=torch.float64)
        v = torch.tensor(wl.v, dtype=torch.float64)
        m = torch.tensor(wl.m, dtype=torch.float64)
        w = torch.tensor(wl.omega, dtype=torch.float64)
        E = torch.tensor(wl.E, dtype=torch.float64)
        for _ in range(nsteps):
            x, v, m, w, E = step(x, v, m, w, E, wl.params, float(c0), dt)
    return {"x": x.numpy(), "v": v.numpy(), "m": m.numpy(), "w": w.numpy(), "E": E.numpy()}


# ---------------------------------------------------------------- J2 solids
# The solid step of the same reading: a GRADIENT loop L_i = sum_j w_j
# (v_j - v_i) (x) g_ij, the stress stage (Jaumann rate of the deviatoric
# stress, radial return to the yield surface Y0 + H eps_p), the FORCE loop
# with the Cauchy stress -p I + S (normal stress P = p - n.S.n in the Riemann
# solution, traction -mean(S) n), the update and the linear EOS
# p = K (rho / rho0 - 1) with a constant sound speed.  Free boundaries.

_SYM = ((0, 3, 4), (3, 1, 5), (4, 5, 2))   # stored (xx yy zz xy xz yz) -> full


def sym_full(S):
    """(n, 6) stored symmetric tensors -> (n, 3, 3)."""
    return torch.stack([torch.stack([S[:, _SYM[a][b]] for b in range(3)], -1) for a in range(3)], -2)


def _pairs(x, h):
    d = x[None, :, :] - x[:, None, :]                    # d[i, j] = x_j - x_i
    r2 = (d * d).sum(-1)
    R = 2.0 * h
    mask = (r2 < R * R) & (r2 > 0.0)
    r = torch.sqrt(torch.where(mask, r2, torch.ones_like(r2)))
    F = torch.where(mask, kernel_F(r, h), torch.zeros_like(r))
    n = d / r[..., None]
    return n, F[..., None] * n, F


def velocity_gradient(x, v, w, P):
    """L_i[a, b] = sum_j w_j (v_j - v_i)_a g_ij[b]."""
    _, g, _ = _pairs(x, P["h"])
    dv = v[None, :, :] - v[:, None, :]
    return (w[None, :, None, None] * dv[..., :, None] * g[..., None, :]).sum(1)


def stress_stage(S, ep, L, P, dt):
    """Jaumann update of the stored deviatoric stress and J2 radial return."""
    G = P["G"]
    D = 0.5 * (L + L.transpose(1, 2))
    W = 0.5 * (L - L.transpose(1, 2))
    Sf = sym_full(S)
    tr = D[:, 0, 0] + D[:, 1, 1] + D[:, 2, 2]
    eye = torch.eye(3, dtype=S.dtype)
    Sd = 2.0 * G * (D - tr[:, None, None] / 3.0 * eye) + W @ Sf - Sf @ W
    St = Sf + dt * Sd
    St6 = torch.stack([St[:, 0, 0], St[:, 1, 1], St[:, 2, 2], St[:, 0, 1], St[:, 0, 2], St[:, 1, 2]], 1)
    J = (St6[:, :3] ** 2).sum(1) + 2.0 * (St6[:, 3:] ** 2).sum(1)
    q = torch.sqrt(1.5 * J)
    sy = P["Y0"] + P["H"] * ep
    plastic = q > sy
    dep = torch.where(plastic, (q - sy) / (3.0 * G + P["H"]), torch.zeros_like(q))
    f = torch.where(plastic, 1.0 - 3.0 * G * dep / torch.where(plastic, q, torch.ones_like(q)), torch.ones_like(q))
    return St6 * f[:, None], ep + dep


def solid_rates(x, v, m, w, E, S, P):
    """(mdot, mvdot, mEdot, wdot) of the solid FORCE loop."""
    rho = m / w
    p = P["K"] * (rho / P["rho0"] - 1.0)
    c = torch.full_like(rho, math.sqrt((P["K"] + 4.0 * P["G"] / 3.0) / P["rho0"]))
    e = E - 0.5 * (v * v).sum(1)
    n, g, F = _pairs(x, P["h"])
    Sf = sym_full(S)
    ai = torch.einsum("iab,ijb->ija", Sf, n)             # S_i n
    bj = torch.einsum("jab,ijb->ija", Sf, n)             # S_j n
    Pi = p[:, None] - (n * ai).sum(-1)
    Pj = p[None, :] - (n * bj).sum(-1)
    Snbar = 0.5 * (ai + bj)
    ui = (v[:, None, :] * n).sum(-1)
    uj = (v[None, :, :] * n).sum(-1)
    rb = 0.5 * (rho[:, None] + rho[None, :])
    cb = 0.5 * (c[:, None] + c[None, :])
    pb = 0.5 * (p[:, None] + p[None, :])
    Z = rb * cb
    beta = P["beta"]
    du = beta * (Pi - Pj) / (2.0 * Z)
    ps = pb + beta * Z * (ui - uj) * 0.5
    vs = 0.5 * (v[:, None, :] + v[None, :, :]) + du[..., None] * n
    Es = 0.5 * (e[:, None] + e[None, :]) + 0.5 * (vs * vs).sum(-1)
    A = 2.0 * w[:, None] * w[None, :]
    Phi = rb * du * F
    t = ps[..., None] * g - F[..., None] * Snbar
    mdot = (-A * Phi).sum(1)
    mvdot = (-A[..., None] * (Phi[..., None] * vs + t)).sum(1)
    mEdot = (-A * (Phi * Es + (t * vs).sum(-1))).sum(1)
    wdot = (w[:, None] * w[None, :] * ((v[None, :, :] - v[:, None, :]) * g).sum(-1)).sum(1)
    return mdot, mvdot, mEdot, wdot


def solid_step(x, v, m, w, E, S, ep, P, dt):
    L = velocity_gradient(x, v, w, P)
    S, ep = stress_stage(S, ep, L, P, dt)
    mdot, mvdot, mEdot, wdot = solid_rates(x, v, m, w, E, S, P)
    mn = m + dt * mdot
    vn = (m[:, None] * v + dt * mvdot) / mn[:, None]
    En = (m * E + dt * mEdot) / mn
    wn = w + dt * wdot
    xn = x + dt * vn
    return xn, vn, mn, wn, En, S, ep


def solid_kinetic_energy_after(x0, v0, m0, w0, e0, S0, ep0, P, dt, nsteps):
    x, v, m, w, S, ep = x0, v0, m0, w0, S0, ep0
    E = e0 + 0.5 * (v0 * v0).sum(1)
    for _ in range(nsteps):
        x, v, m, w, E, S, ep = solid_step(x, v, m, w, E, S, ep, P, dt)
    return 0.5 * (m * (v * v).sum(1)).sum()


def solid_gradient(wl, dt, nsteps):
    """(J, dJ/dv0 (n,3), dJ/dS0 (n,6)) by reverse mode, float64, at fixed e0."""
    x0 = torch.tensor(wl.x, dtype=torch.float64)
    v0 = torch.tensor(wl.v, dtype=torch.float64, requires_grad=True)
    m0 = torch.tensor(wl.m, dtype=torch.float64)
    w0 = torch.tensor(wl.omega, dtype=torch.float64)
    e0 = torch.tensor(wl.E - 0.5 * (wl.v * wl.v).sum(1), dtype=torch.float64)
    S0 = torch.tensor(wl.S, dtype=torch.float64, requires_grad=True)
    ep0 = torch.tensor(wl.eps_p, dtype=torch.float64)
    J = solid_kinetic_energy_after(x0, v0, m0, w0, e0, S0, ep0, wl.params, dt, nsteps)
    gv, gS = torch.autograd.grad(J, (v0, S0))
    return float(J.detach()), gv.numpy(), gS.numpy()


def solid_final_state(wl, dt, nsteps):
    with torch.no_grad():
        x = torch.tensor(wl.x, dtype=torch.float64)
        v = torch.tensor(wl.v, dtype=torch.float64)
        m = torch.tensor(wl.m, dtype=torch.float64)
        w = torch.tensor(wl.omega, dtype=torch.float64)
        E = torch.tensor(wl.E, dtype=torch.float64)
        S = torch.tensor(wl.S, dtype=torch.float64)
        ep = torch.tensor(wl.eps_p, dtype=torch.float64)
        for _ in range(nsteps):
            x, v, m, w, E, S, ep = solid_step(x, v, m, w, E, S, ep, wl.params, dt)
    return {"x": x.numpy(), "v": v.numpy(), "m": m.numpy(), "w": w.numpy(), "E": E.numpy(), "S": S.numpy(),
            "ep": ep.numpy()}
