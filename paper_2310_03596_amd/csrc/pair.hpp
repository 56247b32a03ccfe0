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
template <>
__device__ inline double rcp<double>(double x)
{
    return 1.0 / x;
}

// 1 / sqrt(r2) and sqrt(r2); r2 = 0 (a particle with itself, or a
// coincident pair) gives r = 0 and rinv = 0, so n = 0 and, with F(0) = 0,
// every pair term is exactly zero.
template <typename real>
__device__ inline void inv_len(real r2, real &r, real &rinv);
template <>
__device__ inline void inv_len<float>(float r2, float &r, float &rinv)
{
    rinv = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
    r = r2 * rinv;
}
template <>
__device__ inline void inv_len<double>(double r2, double &r, double &rinv)
{
    r = sqrt(r2);
    rinv = r2 > 0.0 ? 1.0 / r : 0.0;
}

// Compensated (hi, lo) accumulator for float (TwoSum: the rounding error of
// every addition is kept exactly in lo); plain sum for double.
template <typename real>
struct Sum;
template <>
struct Sum<float> {
    float s, c;
    __device__ inline void add(float x)
    {
        float t = s + x;
        float bp = t - s;
        float ap = t - bp;
        c += (s - ap) + (x - bp);
        s = t;
    }
};
template <>
struct Sum<double> {
    double s, c;
    __device__ inline void add(double x) { s += x; }
};

// Kernel and Riemann constants in the form's precision.
template <typename real>
struct PairK {
    real hinv, Fc, beta, half_beta;
};

template <typename real>
__device__ inline real kernel_F(real r, const PairK<real> &K)
{
    real q = r * K.hinv;
    real t = max(real(2) - q, real(0));      // zero beyond the support
    real fin = q * (real(3) - real(2.25) * q);
    real fout = real(0.75) * t * t;
    return K.Fc * (q < real(1) ? fin : fout);
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
    const real cb = real(0.5) * (I.c + J.c);
    const real pb = real(0.5) * (I.p + J.p);
    const real Z = rb * cb;
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
    const real du = K.half_beta * (Pi - Pj) * rcp<real>(Z);
    const real ps = pb - (K.half_beta * Z * s1) * rinv;
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
    const real Es = real(0.5) * (I.e + J.e) + real(0.5) * vs2;
    const real vsd = real(0.5) * s2 + du * r;                  // v* . d
    real tv = psG * vsd;                                       // t . v* (fluid part)
    if constexpr (SOLID) {
        // - F mean(S) n . v* = -(G / 2) Sd . (sv / 2 + du rinv d)
        const real sdsv = Sd[0] * sv[0] + Sd[1] * sv[1] + Sd[2] * sv[2];
        const real sdd = Sd[0] * d[0] + Sd[1] * d[1] + Sd[2] * d[2];
        tv -= real(0.5) * G * (real(0.5) * sdsv + du * rinv * sdd);
    }
    out[4] = mA * (Phi * Es + tv);
    out[5] = real(0.5) * A * G * s1;
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
