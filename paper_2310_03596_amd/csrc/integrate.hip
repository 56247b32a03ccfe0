// Step g of Section II: explicit update, equation of state, solid stress
// stage, and deterministic FP64 diagnostics (next dt and conserved totals).
//
// Elementwise and HBM-bound: every stage reads and writes each particle once
// in coalesced SoA order; arithmetic runs in FP64 in both forms (free next to
// the memory traffic) and is stored back in the form's precision.  Totals
// are reduced per workgroup in a fixed order into a partial record, then one
// workgroup folds the records in a fixed order, so the result does not
// depend on scheduling.
#include "common.hpp"

namespace sph {

namespace {

// Mie-Gruneisen EOS of a solid with the linear shock-velocity Hugoniot
// (Us = c0 + s up) as reference and Gamma rho = Gamma0 rho0, a spall cut-off
// and the longitudinal sound speed (bulk plus shear).  Section IV.A names the
// EOS and the cut-off; the form is the usual one for metals.
__device__ inline void eos_mie_gruneisen(const Params &P, double rho, double e, double &p, double &c)
{
#pragma clang fp contract(off)
    const double mu = rho / P.rho0 - 1.0;
    const double k0 = P.rho0 * P.c0 * P.c0;
    const double th = P.mg_gamma0 * P.rho0 * e;
    double pu, cb2;
    if (mu > 0.0) {
        const double b = P.mg_s - 1.0;
        const double D = fmax(1.0 - b * mu, 0.0625);
        pu = k0 * mu * (1.0 + (1.0 - 0.5 * P.mg_gamma0) * mu) / (D * D) + th;
        cb2 = P.c0 * P.c0 * (1.0 + (2.0 - P.mg_gamma0 + b) * mu) / (D * D * D);
    } else {
        pu = k0 * mu + th;
        cb2 = P.c0 * P.c0;
    }
    cb2 += P.mg_gamma0 * P.rho0 * fmax(pu, 0.0) / (rho * rho);
    p = fmax(pu, P.p_cut);
    c = sqrt(cb2 + 4.0 * P.G / (3.0 * rho));
}

template <typename real>
__device__ inline void eos(const Params &P, double rho, double e, double &p, double &c)
{
    if (P.material == SPH_FLUID_TAIT) {
        double sg, sh;
        tait_powers<real>(P, rho / P.rho0, sg, sh);
        p = P.B * (sg - 1.0);
        c = P.c0 * sh;
    } else if (P.eos == SPH_EOS_MIE_GRUNEISEN) {
        eos_mie_gruneisen(P, rho, e, p, c);
    } else {
        p = P.K * (rho / P.rho0 - 1.0);
        c = P.c_solid;
    }
}

// Fixed-order workgroup reduction of the record: slot 0 by max, the rest by sum.
__device__ inline void block_reduce_record(double r[kDiag], double *out)
{
    __shared__ double sh[kDiag][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kDiag; ++k) {
        double v = r[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            double o = __shfl_down(v, off, kWave);
            v = (k == 0) ? fmax(v, o) : v + o;
        }
        if (lane == 0) sh[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kDiag; ++k) {
            double v = sh[k][0];
            for (int w = 1; w < kBlock / kWave; ++w) v = (k == 0) ? fmax(v, sh[k][w]) : v + sh[k][w];
            out[k] = v;
        }
        for (int k = kDiag; k < kDiagPartial; ++k) out[k] = 0.0;
    }
}

// EOS of the stored state, then the particle's share of the diagnostics:
// c + |v| for the next dt, mass, momentum, energy, kinetic energy, and 1 in
// slot 7 when any stored field (or `bad`, the caller's own check) is not
// finite, so a blow-up is seen on the device without reading the state back.
template <typename real>
__device__ inline void finish(const Params &P, const PV<real> &s, uint32_t i, double m, double w, const double v[3],
                              double E, double rec[kDiag], bool bad = false)
{
    double rho = m / w;
    double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double e = E - 0.5 * v2;
    double p, c;
    eos<real>(P, rho, e, p, c);
    s.rho[i] = (real)rho;
    s.p[i] = (real)p;
    s.c[i] = (real)c;
    s.e[i] = (real)e;
    rec[0] = fmax(rec[0], c + sqrt(v2));
    rec[1] += m;
    rec[2] += m * v[0];
    rec[3] += m * v[1];
    rec[4] += m * v[2];
    rec[5] += m * E;
    rec[6] += 0.5 * m * v2;
    const bool ok = isfinite(m) && isfinite(w) && isfinite(v2) && isfinite(E) && isfinite((double)(real)rho) &&
                    isfinite((double)(real)p) && isfinite((double)(real)c);
    rec[7] += (ok && !bad) ? 0.0 : 1.0;
}

// The update and EOS kernels run on at most kDiagBlocks workgroups, each
// thread taking particles i, i + T, ... (T the grid's threads), so the final
// fold of the per-workgroup records reads at most kDiagBlocks records in one
// round trip; the records depend on n only, so the totals stay deterministic.
#ifndef SPH_DIAG_BLOCKS
// measured on the 810k column (300 steps, two rounds each): 1024 workgroups
// 0.4706 ms per step, 2048 0.4750, 3072 0.4773, 4096 (one particle per
// thread) slower still: a thread with several particles keeps more loads in
// flight
#define SPH_DIAG_BLOCKS 1024
#endif
constexpr uint32_t kDiagBlocks = SPH_DIAG_BLOCKS;

template <typename real, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_motion(Params P, PV<real> s, RV<real> R, const double *__restrict__ dtp,
                                                   double *__restrict__ partials)
{
    double rec[kDiag] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < s.n; i += stride) {
        const double dt = *dtp;
        double r[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) r[k] = (double)R.hi[k][i] + (SPLIT ? (double)R.lo[k][i] : 0.0);
        double m = (double)s.m[i];
        double v[3] = {(double)s.v[0][i], (double)s.v[1][i], (double)s.v[2][i]};
        // every input is read before the first store: the stores below could
        // alias them as far as the compiler knows, and reads issued after a
        // store would each wait a full memory round trip
        const double x0[3] = {s.x[0][i], s.x[1][i], s.x[2][i]};
        const double E0 = s.E[i], w0 = (double)s.w[i];
        double mn = m + dt * r[0];
        double gv = P.g[0] * v[0] + P.g[1] * v[1] + P.g[2] * v[2];
        double vn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) vn[a] = (m * v[a] + dt * (r[1 + a] + m * P.g[a])) / mn;
        double En = (m * E0 + dt * (r[4] + m * gv)) / mn;
        double wn = w0 + dt * r[5];
        bool bad = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double xn = x0[a] + dt * vn[a];
            bad = bad || !isfinite(xn);
            if ((P.wall_mask >> (2 * a)) & 1u)
                if (xn < P.wlo[a]) {
                    xn = 2.0 * P.wlo[a] - xn;
                    vn[a] = -vn[a];
                }
            if ((P.wall_mask >> (2 * a + 1)) & 1u)
                if (xn > P.whi[a]) {
                    xn = 2.0 * P.whi[a] - xn;
                    vn[a] = -vn[a];
                }
            s.x[a][i] = xn;
            s.v[a][i] = (real)vn[a];
        }
        real mr = (real)mn, wr = (real)wn;
        s.m[i] = mr;
        s.w[i] = wr;
        s.E[i] = En;
        // the stored (possibly rounded) state defines the EOS and the totals
        double vs[3] = {(double)(real)vn[0], (double)(real)vn[1], (double)(real)vn[2]};
        finish<real>(P, s, i, (double)mr, (double)wr, vs, En, rec, bad);
    }
    block_reduce_record(rec, partials + (size_t)blockIdx.x * kDiagPartial);
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_eos(Params P, PV<real> s, double *__restrict__ partials)
{
    double rec[kDiag] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < s.n; i += stride) {
        double v[3] = {(double)s.v[0][i], (double)s.v[1][i], (double)s.v[2][i]};
        const bool bad = !(isfinite(s.x[0][i]) && isfinite(s.x[1][i]) && isfinite(s.x[2][i]));
        finish<real>(P, s, i, (double)s.m[i], (double)s.w[i], v, s.E[i], rec, bad);
    }
    block_reduce_record(rec, partials + (size_t)blockIdx.x * kDiagPartial);
}

// The final fold of the per-block records: one workgroup of 1024 threads
// reads the records as one flat array in coalesced order, so thread t folds
// component t % kDiagPartial of every (1024 / kDiagPartial)-th record.  The
// records were written on every XCD, so each read goes to memory: a thread
// issues up to 16 reads before it folds them, and the fold of at most
// kDiagBlocks records takes one round trip instead of one per read.  The
// values in order, then the lanes holding the same component (a fixed
// butterfly), then the wavefronts (in order) are combined, so the
// diagnostics are deterministic.  Slot 0 folds by max, the others by sum.
constexpr int kFinalBlock = 1024;
static_assert(kFinalBlock % kDiagPartial == 0 && kWave % kDiagPartial == 0, "components stay on their lanes");
__global__ __launch_bounds__(kFinalBlock) void k_diag_final(const double *__restrict__ partials, uint32_t nblocks,
                                                            double cfl_h, double *__restrict__ diag)
{
    const uint32_t t = threadIdx.x;
    const bool is_max = t % kDiagPartial == 0;
    const uint32_t total = nblocks * kDiagPartial;
    auto fold = [&](double a, double b) { return is_max ? fmax(a, b) : a + b; };
    constexpr int kU = 16;
    double a = 0.0;
    for (uint32_t f0 = t; f0 < total; f0 += kU * kFinalBlock) {
        double q[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t f = f0 + (uint32_t)u * kFinalBlock;
            q[u] = f < total ? partials[f] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) a = fold(a, q[u]);
    }
#pragma unroll
    for (int off = kDiagPartial; off < kWave; off <<= 1) a = fold(a, __shfl_xor(a, off, kWave));
    __shared__ double sh[kFinalBlock / kWave][kDiagPartial];
    const int lane = t & (kWave - 1), wave = t / kWave;
    if (lane < kDiagPartial) sh[wave][lane] = a;
    __syncthreads();
    if (t < kDiag) {
        double v = sh[0][t];
        for (int w = 1; w < kFinalBlock / kWave; ++w) v = t == 0 ? fmax(v, sh[w][t]) : v + sh[w][t];
        diag[t] = t == 0 ? (v > 0.0 ? cfl_h / v : __builtin_huge_val()) : v;
    }
}

// Jaumann rate of the deviatoric stress and J2 radial return with linear hardening.
template <typename real, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_stress(Params P, PV<real> s, RV<real> R, const double *__restrict__ dtp)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const double dt = *dtp;
    double L[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) L[k] = (double)R.Lhi[k][i] + (SPLIT ? (double)R.Llo[k][i] : 0.0);
    double D[3][3], W[3][3], S[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            D[a][b] = 0.5 * (L[3 * a + b] + L[3 * b + a]);
            W[a][b] = 0.5 * (L[3 * a + b] - L[3 * b + a]);
        }
    double s6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) s6[k] = (double)s.S[k][i];
    S[0][0] = s6[0]; S[1][1] = s6[1]; S[2][2] = s6[2];
    S[0][1] = S[1][0] = s6[3];
    S[0][2] = S[2][0] = s6[4];
    S[1][2] = S[2][1] = s6[5];
    const double tr = D[0][0] + D[1][1] + D[2][2];
    double Sd[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double ws = 0.0, sw = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ws += W[a][k] * S[k][b];
                sw += S[a][k] * W[k][b];
            }
            Sd[a][b] = 2.0 * P.G * (D[a][b] - (a == b ? tr / 3.0 : 0.0)) + ws - sw;
        }
    double St[6] = {S[0][0] + dt * Sd[0][0], S[1][1] + dt * Sd[1][1], S[2][2] + dt * Sd[2][2],
                    S[0][1] + dt * Sd[0][1], S[0][2] + dt * Sd[0][2], S[1][2] + dt * Sd[1][2]};
    double J = St[0] * St[0] + St[1] * St[1] + St[2] * St[2] + 2.0 * (St[3] * St[3] + St[4] * St[4] + St[5] * St[5]);
    double q = sqrt(1.5 * J);
    double ep = (double)s.ep[i];
    double sy = P.Y0 + P.H * ep;
    if (q > sy) {
        double dep = (q - sy) / (3.0 * P.G + P.H);
        double f = 1.0 - 3.0 * P.G * dep / q;
#pragma unroll
        for (int k = 0; k < 6; ++k) St[k] *= f;
        ep += dep;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) s.S[k][i] = (real)St[k];
    s.ep[i] = (real)ep;
}

template <typename real>
hipError_t go(const Params &P, int stage, const sph_particles &p, const sph_rates &r, const double *dt,
              double *diag, const Workspace &ws, hipStream_t s)
{
    constexpr bool SPLIT = sizeof(real) == 4;
    uint32_t blocks = div_up(p.n, kBlock);
    if (stage == SPH_STAGE_STRESS) {
        if (blocks) k_stress<real, SPLIT><<<blocks, kBlock, 0, s>>>(P, view<real>(p), view<real>(r), dt);
        return hipGetLastError();
    }
    const uint32_t rblocks = blocks < kDiagBlocks ? blocks : kDiagBlocks;   // records: at most one per kBlock particles
    if (rblocks) {
        if (stage == SPH_STAGE_MOTION)
            k_motion<real, SPLIT><<<rblocks, kBlock, 0, s>>>(P, view<real>(p), view<real>(r), dt, ws.partials);
        else
            k_eos<real><<<rblocks, kBlock, 0, s>>>(P, view<real>(p), ws.partials);
    }
    if (diag) k_diag_final<<<1, kFinalBlock, 0, s>>>(ws.partials, rblocks, P.cfl * P.h, diag);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_integrate(const Params &P, int prec, int stage, const sph_particles &p, const sph_rates &r,
                            const double *dt, double *diag, const Workspace &ws, hipStream_t s)
{
    if (prec == SPH_FP64) return go<double>(P, stage, p, r, dt, diag, ws, s);
    return go<float>(P, stage, p, r, dt, diag, ws, s);
}

}  // namespace sph
