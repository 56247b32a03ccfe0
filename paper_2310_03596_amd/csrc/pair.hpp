// Pair terms of the SPH-ALE interaction loops (device functions).
//
// The paper (Section I) names Gamma-SPH-ALE but gives no equations, so the
// pair terms follow the documented reading: a cubic-spline kernel with
// support 2h and, along n = (x_j - x_i) / r, the linearised (acoustic)
// Riemann solution between particle i (left) and j (right) with impedance
// Z = mean(rho) mean(c):
//   du = u* - mean(u) = beta (P_i - P_j) / (2 Z)
//   p* = mean(p) + beta Z (u_i - u_j) / 2
//   v* = mean(v) + du n,  E* = mean(e) + |v*|^2 / 2
// With A = 2 w_i w_j, g = F n (F = -dW/dr), Phi = mean(rho) du F and the
// traction t = p* g - mean(S) g:
//   mdot = -A Phi, mvdot = -A (Phi v* + t), mEdot = -A (Phi E* + t . v*),
//   wdot = w_i w_j (v_j - v_i) . g.
// P = p for fluids and p - n.S.n for solids.  The GRADIENT loop of solids
// sums L_ab = w_j (v_j - v_i)_a g_b.  Every quantity is written so it is
// exactly even or odd under i <-> j, so mass, momentum and energy terms of a
// pair cancel exactly.
#pragma once

#include "common.hpp"

namespace sph {

template <typename real>
__device__ inline real rcp(real x);
template <>
__device__ inline float rcp<float>(float x)
{
    return __builtin_amdgcn_rcpf(x);
}
// FP64: the hardware estimate refined by two Newton steps y += y (1 - x y),
// each of which about doubles the correct bits; the result is within an ulp
// or two of 1 / x, at a third of the instructions of an IEEE division.
template <>
__device__ inline double rcp<double>(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// 1 / sqrt(r2) and sqrt(r2); r2 = 0 (a particle with itself, or a
// coincident pair) gives r = 0, so n = 0 and, with F(0) = 0, every pair term
// is exactly zero.  In FP32 the argument is r2 + 2^-126, which equals r2 for
// every r2 above 2^-101 and makes rinv = 2^63 at r2 = 0, a finite factor that
// every term then multiplies by an exact zero; in FP64 it is r2 + 2^-1022
// (equal to r2 above 2^-969; rinv = 2^511 at r2 = 0).  rinv is a function of
// r2 alone, so it is the same for (i, j) and (j, i) and every term keeps its
// parity.
template <typename real>
__device__ inline void inv_len(real r2, real &r, real &rinv);
template <>
__device__ inline void inv_len<float>(float r2, float &r, float &rinv)
{
    rinv = __builtin_amdgcn_rsqf(r2 + 0x1p-126f);
    r = r2 * rinv;
}
// FP64: the hardware estimate of 1 / sqrt refined by two Newton steps
// y += (y / 2)(1 - a y^2), within an ulp or two of the exact value, in place
// of an IEEE square root and division (about 25 instructions).
template <>
__device__ inline void inv_len<double>(double r2, double &r, double &rinv)
{
    const double a = r2 + 0x1p-1022;
    double y = __builtin_amdgcn_rsq(a);
    y = fma(0.5 * y, fma(-(a * y), y, 1.0), y);
    y = fma(0.5 * y, fma(-(a * y), y, 1.0), y);
    rinv = y;
    r = r2 * y;
}

// Kernel and Riemann constants in the form's precision: F3, F225 and F075
// are Fc times the cubic spline's coefficients 3, 9/4 and 3/4; hb4 = 2 beta
// and hbq = beta / 8 are the Riemann factor beta / 2 times 4 and 1 / 4 (powers
// of two: exact).
template <typename real>
struct PairK {
    real hinv, Fc, beta, half_beta;
    real F3, F225, F075;
    real hb4, hbq;
};

template <typename real>
__device__ inline PairK<real> make_pair_k(const Params &P)
{
    PairK<real> K;
    K.hinv = (real)P.hinv;
    K.Fc = (real)P.Fc;
    K.beta = (real)P.beta;
    K.half_beta = (real)(0.5 * P.beta);
    K.F3 = (real)(3.0 * P.Fc);
    K.F225 = (real)(2.25 * P.Fc);
    K.F075 = (real)(0.75 * P.Fc);
    K.hb4 = (real)(2.0 * P.beta);
    K.hbq = (real)(0.125 * P.beta);
    return K;
}

// F(r) for r < 2h (the callers have applied the neighbour predicate; at the
// support's edge F and dF/dr vanish, so a q that rounds to just above 2 gives
// F of the order of the rounding squared).
template <typename real>
__device__ inline real kernel_F(real r, const PairK<real> &K)
{
    const real q = r * K.hinv;
    const real t = real(2) - q;
    if constexpr (sizeof(real) == 4) {
        const real fin = q * (K.F3 - K.F225 * q);
        const real fout = (K.F075 * t) * t;
        return q < real(1) ? fin : fout;
    } else {
        // fewer live constants: the FP64 pass is short of registers
        const real fin = q * (real(3) - real(2.25) * q);
        const real fout = real(0.75) * t * t;
        return K.Fc * (q < real(1) ? fin : fout);
    }
}

// Per-particle quantities the FORCE pair terms read.
template <typename real, bool SOLID>
struct Part {
    real v[3];
    real w, rho, p, c, e;
    real S[SOLID ? 6 : 1];
};

template <typename real, bool SOLID>
__device__ inline void load_part(const PV<real> &a, uint32_t k, Part<real, SOLID> &o)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) o.v[d] = a.v[d][k];
    o.w = a.w[k];
    o.rho = a.rho[k];
    o.p = a.p[k];
    o.c = a.c[k];
    o.e = a.e[k];
    if constexpr (SOLID) {
#pragma unroll
        for (int q = 0; q < 6; ++q) o.S[q] = a.S[q][k];
    }
}

// S n for symmetric S stored (xx yy zz xy xz yz).
template <typename real>
__device__ inline void sym_mul(const real *S, const real n[3], real o[3])
{
    o[0] = S[0] * n[0] + S[3] * n[1] + S[4] * n[2];
    o[1] = S[3] * n[0] + S[1] * n[1] + S[5] * n[2];
    o[2] = S[4] * n[0] + S[5] * n[1] + S[2] * n[2];
}

// FORCE terms of target i from source j; d = x_j - x_i, r2 = |d|^2.
// The formulas above, evaluated on the unnormalised d with one reciprocal
// square root (n = d rinv, g = G d with G = F rinv), the sums and
// differences of the two velocities (sv = v_i + v_j even, dv = v_j - v_i
// odd) and their projections s1 = dv . d (even) and s2 = sv . d (odd):
//   u_i - u_j = -s1 rinv,  v* = sv / 2 + du rinv d,
//   |v*|^2 = |sv|^2 / 4 + du (s2 rinv + du),  v* . d = s2 / 2 + du r,
//   wdot = w_i w_j G s1.
// Every product keeps the parity of its factors, so each term stays exactly
// even (volume) or odd (mass, momentum, energy) under i <-> j.
template <typename real, bool SOLID>
__device__ inline void pair_force(const real d[3], real r2, const Part<real, SOLID> &I,
                                  const Part<real, SOLID> &J, const PairK<real> &K, real out[6])
{
    real r, rinv;
    inv_len<real>(r2, r, rinv);
    const real F = kernel_F<real>(r, K);
    const real G = F * rinv;
    const real sv[3] = {I.v[0] + J.v[0], I.v[1] + J.v[1], I.v[2] + J.v[2]};
    const real dv[3] = {J.v[0] - I.v[0], J.v[1] - I.v[1], J.v[2] - I.v[2]};
    const real s1 = dv[0] * d[0] + dv[1] * d[1] + dv[2] * d[2];
    const real s2 = sv[0] * d[0] + sv[1] * d[1] + sv[2] * d[2];
    const real rb = real(0.5) * (I.rho + J.rho);
    const real pb = real(0.5) * (I.p + J.p);
    const real Z4 = (I.rho + J.rho) * (I.c + J.c);   // 4 Z
    real Pi = I.p, Pj = J.p;
    real Sd[3] = {real(0), real(0), real(0)};   // (S_i + S_j) d
    if constexpr (SOLID) {
        real si[3], sj[3];
        sym_mul<real>(I.S, d, si);
        sym_mul<real>(J.S, d, sj);
        const real r2inv = rinv * rinv;
        Pi = I.p - (d[0] * si[0] + d[1] * si[1] + d[2] * si[2]) * r2inv;
        Pj = J.p - (d[0] * sj[0] + d[1] * sj[1] + d[2] * sj[2]) * r2inv;
#pragma unroll
        for (int a = 0; a < 3; ++a) Sd[a] = si[a] + sj[a];
    }
    // du = (beta / 2) (P_i - P_j) / Z and p* = mean(p) - (beta / 2) Z s1 / r
    real du, ps;
    if constexpr (sizeof(real) == 4) {
        du = K.hb4 * (Pi - Pj) * rcp<real>(Z4);
        ps = pb - (K.hbq * Z4 * s1) * rinv;
    } else {
        // fewer live constants: the FP64 pass is short of registers
        const real Z = real(0.25) * Z4;
        du = K.half_beta * (Pi - Pj) * rcp<real>(Z);
        ps = pb - (K.half_beta * Z * s1) * rinv;
    }
    const real A = real(2) * I.w * J.w;
    const real Phi = rb * du * F;
    const real mA = -A;
    const real psG = ps * G;
    out[0] = mA * Phi;
    const real ca = real(0.5) * out[0];                       // -A Phi / 2
    const real k1 = mA * ((Phi * du) * rinv + psG);            // even
    const real kS = real(0.5) * A * G;                         // traction of mean(S): +A F Snb = kS Sd
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        real m = ca * sv[a] + k1 * d[a];
        if constexpr (SOLID) m += kS * Sd[a];
        out[1 + a] = m;
    }
    const real sv2 = sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
    const real vs2 = real(0.25) * sv2 + du * (s2 * rinv + du);
    const real Es2 = (I.e + J.e) + vs2;                        // 2 E*
    const real vsd = real(0.5) * s2 + du * r;                  // v* . d
    real tv = psG * vsd;                                       // t . v* (fluid part)
    if constexpr (SOLID) {
        // - F mean(S) n . v* = -(G / 2) Sd . (sv / 2 + du rinv d)
        const real sdsv = Sd[0] * sv[0] + Sd[1] * sv[1] + Sd[2] * sv[2];
        const real sdd = Sd[0] * d[0] + Sd[1] * d[1] + Sd[2] * d[2];
        tv -= real(0.5) * G * (real(0.5) * sdsv + du * rinv * sdd);
    }
    out[4] = ca * Es2 - A * tv;                                // -A (Phi E* + t . v*)
    out[5] = real(0.5) * A * G * s1;
}

// Reverse mode of pair_force with respect to the TARGET's inputs: given
// cotangents wb[6] of the six terms, adds to g the cotangents of
// (x_i[3], v_i[3], omega_i, rho_i, p_i, c_i, e_i) and, for solids, of the
// stored deviatoric stress S_i[6] (g[11..16]).  Every intermediate of the
// forward evaluation is recomputed, then differentiated in reverse order.
// A pair with r = 0 contributes nothing.
template <typename real, bool SOLID>
__device__ inline void pair_force_vjp(const real d[3], real r2, const Part<real, SOLID> &I,
                                      const Part<real, SOLID> &J, const PairK<real> &K, const real wb[6],
                                      real g[SOLID ? 17 : 11])
{
    if (!(r2 > real(0))) return;
    // forward
    real r, rinv;
    inv_len<real>(r2, r, rinv);
    const real q = r * K.hinv;
    const real tq = max(real(2) - q, real(0));
    const bool inner = q < real(1);
    const real f = inner ? q * (real(3) - real(2.25) * q) : real(0.75) * tq * tq;
    const real fp = inner ? real(3) - real(4.5) * q : real(-1.5) * tq;   // df/dq
    const real F = K.Fc * f;
    const real G = F * rinv;
    const real sv[3] = {I.v[0] + J.v[0], I.v[1] + J.v[1], I.v[2] + J.v[2]};
    const real dv[3] = {J.v[0] - I.v[0], J.v[1] - I.v[1], J.v[2] - I.v[2]};
    const real s1 = dv[0] * d[0] + dv[1] * d[1] + dv[2] * d[2];
    const real s2 = sv[0] * d[0] + sv[1] * d[1] + sv[2] * d[2];
    const real rb = real(0.5) * (I.rho + J.rho);
    const real cb = real(0.5) * (I.c + J.c);
    const real pb = real(0.5) * (I.p + J.p);
    const real Z = rb * cb;
    const real Zinv = rcp<real>(Z);
    // solids: si = S_i d, sj = S_j d, P = p - d.S.d / r^2, Sd = si + sj
    real si[3] = {0, 0, 0}, sj[3] = {0, 0, 0}, Sd[3] = {0, 0, 0};
    real dsi = 0, dsj = 0, r2inv = 0, Pi = I.p, Pj = J.p;
    if constexpr (SOLID) {
        sym_mul<real>(I.S, d, si);
        sym_mul<real>(J.S, d, sj);
        r2inv = rinv * rinv;
        dsi = d[0] * si[0] + d[1] * si[1] + d[2] * si[2];
        dsj = d[0] * sj[0] + d[1] * sj[1] + d[2] * sj[2];
        Pi = I.p - dsi * r2inv;
        Pj = J.p - dsj * r2inv;
#pragma unroll
        for (int a = 0; a < 3; ++a) Sd[a] = si[a] + sj[a];
    }
    const real du = K.half_beta * (Pi - Pj) * Zinv;
    const real ps = pb - (K.half_beta * Z * s1) * rinv;
    const real A = real(2) * I.w * J.w;
    const real Phi = rb * du * F;
    const real k1 = -A * ((Phi * du) * rinv + ps * G);
    const real ca = real(-0.5) * A * Phi;
    const real kS = real(0.5) * A * G;
    const real sv2 = sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
    const real vs2 = real(0.25) * sv2 + du * (s2 * rinv + du);
    const real Es = real(0.5) * (I.e + J.e) + real(0.5) * vs2;
    const real vsd = real(0.5) * s2 + du * r;
    const real sdsv = Sd[0] * sv[0] + Sd[1] * sv[1] + Sd[2] * sv[2];
    const real sdd = Sd[0] * d[0] + Sd[1] * d[1] + Sd[2] * d[2];
    const real tv = ps * G * vsd - (SOLID ? real(0.5) * G * (real(0.5) * sdsv + du * rinv * sdd) : real(0));
    // reverse
    real bA = 0, bG = 0, bs1 = 0, bs2 = 0, bPhi = 0, bdu = 0, bps = 0, br = 0, brinv = 0, bF = 0;
    real bsv[3] = {0, 0, 0}, bd[3] = {0, 0, 0}, bSd[3] = {0, 0, 0};
    // o5 = A G s1 / 2
    bA += real(0.5) * wb[5] * G * s1;
    bG += real(0.5) * wb[5] * A * s1;
    bs1 += real(0.5) * wb[5] * A * G;
    // o4 = -A (Phi Es + tv)
    bA -= wb[4] * (Phi * Es + tv);
    bPhi -= wb[4] * A * Es;
    const real bEs = -wb[4] * A * Phi;
    const real btv = -wb[4] * A;
    // tv = ps G vsd - (G / 2) (sdsv / 2 + du rinv sdd)
    bps += btv * G * vsd;
    bG += btv * ps * vsd;
    const real bvsd = btv * ps * G;
    real bsdsv = 0, bsdd = 0;
    if constexpr (SOLID) {
        bG -= btv * real(0.5) * (real(0.5) * sdsv + du * rinv * sdd);
        bsdsv -= btv * real(0.25) * G;
        bdu -= btv * real(0.5) * G * rinv * sdd;
        brinv -= btv * real(0.5) * G * du * sdd;
        bsdd -= btv * real(0.5) * G * du * rinv;
    }
    // vsd = s2 / 2 + du r
    bs2 += real(0.5) * bvsd;
    bdu += bvsd * r;
    br += bvsd * du;
    // Es = (e_i + e_j) / 2 + vs2 / 2
    g[10] += real(0.5) * bEs;
    const real bvs2 = real(0.5) * bEs;
    // vs2 = sv2 / 4 + du (s2 rinv + du)
    const real bsv2 = real(0.25) * bvs2;
    bdu += bvs2 * (s2 * rinv + real(2) * du);
    bs2 += bvs2 * du * rinv;
    brinv += bvs2 * du * s2;
    // o_{1+a} = ca sv_a + k1 d_a + kS Sd_a
    real bca = 0, bk1 = 0, bkS = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bca += wb[1 + a] * sv[a];
        bsv[a] += wb[1 + a] * ca + real(2) * bsv2 * sv[a];
        bk1 += wb[1 + a] * d[a];
        bd[a] += wb[1 + a] * k1;
        if constexpr (SOLID) {
            bkS += wb[1 + a] * Sd[a];
            bSd[a] += wb[1 + a] * kS;
        }
    }
    if constexpr (SOLID) {
        // kS = A G / 2; sdsv = Sd . sv; sdd = Sd . d
        bA += real(0.5) * G * bkS;
        bG += real(0.5) * A * bkS;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            bSd[a] += bsdsv * sv[a] + bsdd * d[a];
            bsv[a] += bsdsv * Sd[a];
            bd[a] += bsdd * Sd[a];
        }
    }
    // k1 = -A (Phi du rinv + ps G)
    bA -= bk1 * ((Phi * du) * rinv + ps * G);
    bPhi -= bk1 * A * du * rinv;
    bdu -= bk1 * A * Phi * rinv;
    brinv -= bk1 * A * Phi * du;
    bps -= bk1 * A * G;
    bG -= bk1 * A * ps;
    // ca = -A Phi / 2 ; o0 = -A Phi
    bA -= (real(0.5) * bca + wb[0]) * Phi;
    bPhi -= (real(0.5) * bca + wb[0]) * A;
    // Phi = rb du F
    real brb = bPhi * du * F;
    bdu += bPhi * rb * F;
    bF += bPhi * rb * du;
    // A = 2 w_i w_j
    g[6] += real(2) * bA * J.w;
    // ps = pb - hb Z s1 rinv
    const real bpb = bps;
    real bZ = -bps * K.half_beta * s1 * rinv;
    bs1 -= bps * K.half_beta * Z * rinv;
    brinv -= bps * K.half_beta * Z * s1;
    // du = hb (P_i - P_j) / Z
    const real bPi = bdu * K.half_beta * Zinv;
    const real bPj = -bPi;
    bZ -= bdu * du * Zinv;
    // P_i = p_i - dsi / r^2 (fluids: P_i = p_i)
    g[8] += bPi;
    if constexpr (SOLID) {
        const real bdsi = -bPi * r2inv, bdsj = -bPj * r2inv;
        const real br2inv = -(bPi * dsi + bPj * dsj);
        brinv += real(2) * rinv * br2inv;
        // dsi = d.S_i d, dsj = d.S_j d; si = S_i d, sj = S_j d (S symmetric)
        real bsi[3], bsj[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            bsi[a] = bSd[a];
            bsj[a] = bSd[a];
            bd[a] += real(2) * (bdsi * si[a] + bdsj * sj[a]);
        }
        real t[3];
        sym_mul<real>(I.S, bsi, t);
#pragma unroll
        for (int a = 0; a < 3; ++a) bd[a] += t[a];
        sym_mul<real>(J.S, bsj, t);
#pragma unroll
        for (int a = 0; a < 3; ++a) bd[a] += t[a];
        // stored (xx yy zz xy xz yz): d(d.S d) = d_a d_b (off-diagonals twice),
        // d(S d)_a / dS_ab = d_b
        g[11] += bdsi * d[0] * d[0] + bsi[0] * d[0];
        g[12] += bdsi * d[1] * d[1] + bsi[1] * d[1];
        g[13] += bdsi * d[2] * d[2] + bsi[2] * d[2];
        g[14] += real(2) * bdsi * d[0] * d[1] + bsi[0] * d[1] + bsi[1] * d[0];
        g[15] += real(2) * bdsi * d[0] * d[2] + bsi[0] * d[2] + bsi[2] * d[0];
        g[16] += real(2) * bdsi * d[1] * d[2] + bsi[1] * d[2] + bsi[2] * d[1];
    }
    // Z = rb cb ; rb, cb, pb are means
    brb += bZ * cb;
    const real bcb = bZ * rb;
    g[7] += real(0.5) * brb;
    g[9] += real(0.5) * bcb;
    g[8] += real(0.5) * bpb;
    // s1 = dv . d, s2 = sv . d ; sv = v_i + v_j, dv = v_j - v_i
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bd[a] += bs1 * dv[a] + bs2 * sv[a];
        bsv[a] += bs2 * d[a];
        g[3 + a] += bsv[a] - bs1 * d[a];
    }
    // G = F rinv ; F = Fc f(q), q = r hinv
    bF += bG * rinv;
    brinv += bG * F;
    br += bF * K.Fc * fp * K.hinv;
    // r = sqrt(r2), rinv = r2^-1/2 ; r2 = d . d ; d = x_j - x_i
    const real br2 = real(0.5) * rinv * (br - brinv * rinv * rinv);
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] -= bd[a] + real(2) * br2 * d[a];
}

// Reverse of the GRADIENT loop for one pair (target i, source j).  With
// g = G(r) d (d = x_j - x_i, G = F / r), dv = v_j - v_i, the loop puts
// w_j dv (x) g into L_i and, from the mirrored pair, w_i dv (x) g into L_j.
// Given the cotangents Lbar_i and Lbar_j (row-major 3 x 3) and
// M = w_j Lbar_i + w_i Lbar_j, the pair's part of the target's cotangents:
//   vbar_i -= M g,  wbar_i += dv . Lbar_j g,
//   xbar_i -= G M^T dv + ((F' - G) / r^2) (dv . M d) d.
// out: (x_i[3], v_i[3], omega_i).  A pair with r = 0 contributes nothing.
template <typename real>
__device__ inline void pair_grad_vjp(const real d[3], real r2, const real vi[3], const real vj[3], real wi, real wj,
                                     const real Li[9], const real Lj[9], const PairK<real> &K, real out[7])
{
    if (!(r2 > real(0))) return;
    real r, rinv;
    inv_len<real>(r2, r, rinv);
    const real q = r * K.hinv;
    const real tq = max(real(2) - q, real(0));
    const bool inner = q < real(1);
    const real f = inner ? q * (real(3) - real(2.25) * q) : real(0.75) * tq * tq;
    const real fp = inner ? real(3) - real(4.5) * q : real(-1.5) * tq;
    const real F = K.Fc * f;
    const real Fr = K.Fc * fp * K.hinv;   // dF/dr
    const real G = F * rinv;
    const real gv[3] = {G * d[0], G * d[1], G * d[2]};
    const real dv[3] = {vj[0] - vi[0], vj[1] - vi[1], vj[2] - vi[2]};
    real Mg[3], Mtdv[3] = {0, 0, 0}, Ljg[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Mg[a] = 0;
        Ljg[a] = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const real M = wj * Li[3 * a + b] + wi * Lj[3 * a + b];
            Mg[a] += M * gv[b];
            Mtdv[b] += M * dv[a];
            Ljg[a] += Lj[3 * a + b] * gv[b];
        }
    }
    const real s = Mtdv[0] * d[0] + Mtdv[1] * d[1] + Mtdv[2] * d[2];
    const real k = (Fr - G) * rinv * rinv * s;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        out[a] -= G * Mtdv[a] + k * d[a];
        out[3 + a] -= Mg[a];
    }
    out[6] += dv[0] * Ljg[0] + dv[1] * Ljg[1] + dv[2] * Ljg[2];
}

// GRADIENT terms: L_ab = w_j (v_j - v_i)_a g_b.
template <typename real>
__device__ inline void pair_grad(const real d[3], real r2, const real vi[3], const real vj[3], real wj,
                                 const PairK<real> &K, real out[9])
{
    real r, rinv;
    inv_len<real>(r2, r, rinv);
    real F = kernel_F<real>(r, K);
    real fr = F * rinv;
    real g[3] = {fr * d[0], fr * d[1], fr * d[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        real dv = wj * (vj[a] - vi[a]);
#pragma unroll
        for (int b = 0; b < 3; ++b) out[3 * a + b] = dv * g[b];
    }
}

}  // namespace sph
