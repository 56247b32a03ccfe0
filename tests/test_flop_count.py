"""The algorithmic flop counts of the FORCE pass that the benchmark's roofline
figure rests on, counted rather than asserted.

The pair terms of the documented reading (acoustic Riemann solver along
n between particle i and j, cubic-spline kernel) are written here in their
plain form and evaluated on a number type that counts every add, subtract,
multiply, divide and square root (FMA-free: each is one flop; constants that
depend only on h or beta are folded).  Each item's count must equal the
benchmark's table, and the values must equal the oracle's pair terms, so the
counted expression is the one the pass computes.
"""
import contextlib
import math

import numpy as np

import bench
import sph_synth as S
from oracle import cpu


class Num:
    """A float that counts the arithmetic done on it."""

    ops = 0

    def __init__(self, v):
        self.v = float(v.v if isinstance(v, Num) else v)

    @staticmethod
    def _v(o):
        return o.v if isinstance(o, Num) else float(o)

    def _op(self, r):
        Num.ops += 1
        return Num(r)

    def __add__(self, o):
        return self._op(self.v + self._v(o))

    __radd__ = __add__

    def __sub__(self, o):
        return self._op(self.v - self._v(o))

    def __rsub__(self, o):
        return self._op(self._v(o) - self.v)

    def __mul__(self, o):
        return self._op(self.v * self._v(o))

    __rmul__ = __mul__

    def __truediv__(self, o):
        return self._op(self.v / self._v(o))

    def __neg__(self):
        return Num(-self.v)   # a sign change, not a flop

    def __lt__(self, o):
        return self.v < self._v(o)


def nsqrt(x):
    Num.ops += 1
    return Num(math.sqrt(x.v))


def plain_pair(d, r2, vi, vj, wi, wj, rhoi, rhoj, pi_, pj, ci, cj, ei, ej, h, beta):
    """Fluid pair terms in their plain form; returns (terms, flops per item)."""
    counts = {}

    @contextlib.contextmanager
    def item(name):
        before = Num.ops
        yield
        counts[name] = Num.ops - before

    hinv = 1.0 / h
    Fc = 1.0 / (math.pi * h ** 4)          # F = Fc f(q), folded with h
    hb = 0.5 * beta                        # folded with beta
    with item("r = sqrt(r2)"):
        r = nsqrt(r2)
    with item("q and F(q)"):
        q = r * hinv
        F = Fc * (q * (3.0 - 2.25 * q)) if q < 1.0 else (0.75 * Fc) * ((2.0 - q) * (2.0 - q))
    with item("n = d / r"):
        n = [d[a] / r for a in range(3)]
    with item("g = F n"):
        g = [F * n[a] for a in range(3)]
    with item("u_i, u_j"):
        ui = vi[0] * n[0] + vi[1] * n[1] + vi[2] * n[2]
        uj = vj[0] * n[0] + vj[1] * n[1] + vj[2] * n[2]
    with item("means of rho, c, p"):
        rb, cb, pb = 0.5 * (rhoi + rhoj), 0.5 * (ci + cj), 0.5 * (pi_ + pj)
    with item("Z"):
        Z = rb * cb
    with item("u* - ubar"):
        du = hb * (pi_ - pj) / Z
    with item("p*"):
        ps = pb + hb * Z * (ui - uj)
    with item("v*"):
        vs = [0.5 * (vi[a] + vj[a]) + du * n[a] for a in range(3)]
    with item("E*"):
        Es = 0.5 * (ei + ej) + 0.5 * (vs[0] * vs[0] + vs[1] * vs[1] + vs[2] * vs[2])
    with item("A = 2 w_i w_j"):
        A = 2.0 * wi * wj
    with item("Phi"):
        Phi = rb * du * F
    with item("traction p* g"):
        t = [ps * g[a] for a in range(3)]
    with item("mdot"):
        o0 = -(A * Phi)
    with item("mvdot"):
        o1 = [-(A * (Phi * vs[a] + t[a])) for a in range(3)]
    with item("mEdot"):
        o4 = -(A * (Phi * Es + (t[0] * vs[0] + t[1] * vs[1] + t[2] * vs[2])))
    with item("wdot"):
        dv = [vj[a] - vi[a] for a in range(3)]
        o5 = wi * wj * (dv[0] * g[0] + dv[1] * g[1] + dv[2] * g[2])
    acc = [Num(0.0) for _ in range(6)]
    with item("accumulate 6 rates"):
        acc = [a + o for a, o in zip(acc, [o0] + o1 + [o4, o5])]
    return [a.v for a in acc], counts


def plain_candidate(xi, xj, R2):
    counts = {}
    before = Num.ops
    d = [xj[a] - xi[a] for a in range(3)]
    counts["x_j - x_i"] = Num.ops - before
    before = Num.ops
    r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    counts["|d|^2"] = Num.ops - before
    return d, r2, r2 < R2, counts


def test_flop_tables_are_the_plain_definition():
    wl = S.jittered_lattice(6, seed=81, rho_sigma=0.01)
    p = dict(wl.params)
    h = p["h"]
    rng = np.random.default_rng(82)
    done = set()
    npairs = 0
    for _ in range(400):
        i, j = rng.choice(wl.n, size=2, replace=False)
        xi = [Num(v) for v in wl.x[i]]
        xj = [Num(v) for v in wl.x[j]]
        d, r2, inside, cc = plain_candidate(xi, xj, (2 * h) ** 2)
        assert cc == bench.FLOPS_CAND_ITEMS
        if not inside:
            continue
        rho = wl.rho
        pr = [cpu.eos(p, float(rho[k]))[0] for k in (i, j)]
        cs = [cpu.eos(p, float(rho[k]))[1] for k in (i, j)]
        vi, vj = [Num(v) for v in wl.v[i]], [Num(v) for v in wl.v[j]]
        e = [0.37, 0.61]
        got, counts = plain_pair(d, r2, vi, vj, Num(wl.omega[i]), Num(wl.omega[j]), Num(rho[i]), Num(rho[j]),
                                 Num(pr[0]), Num(pr[1]), Num(cs[0]), Num(cs[1]), Num(e[0]), Num(e[1]), h, p["beta"])
        assert counts == bench.FLOPS_PAIR_ITEMS
        ref = cpu.pair(p, np.array([v.v for v in d]), wl.v[i], wl.v[j], wl.omega[i], wl.omega[j], rho[i], rho[j],
                       pr[0], pr[1], cs[0], cs[1], e[0], e[1])
        scale = np.abs(ref).max()
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * scale), (got, ref)
        done.add(bool(float(np.sqrt(r2.v)) / h < 1.0))
        npairs += 1
    assert done == {True, False}   # both branches of the kernel were counted
    assert npairs >= 50
    assert bench.FLOPS_CAND[0] == bench.FLOPS_CAND[1] == 8
    assert bench.FLOPS_PAIR[0] == bench.FLOPS_PAIR[1] == sum(bench.FLOPS_PAIR_ITEMS.values())
