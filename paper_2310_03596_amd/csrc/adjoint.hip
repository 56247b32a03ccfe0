// Hand-written adjoint of the fluid step (reverse of steps g and e of
// Section II; the pair-pass reverse lives with the pair kernel).
//
// State of one step: x, v, m, omega, E (per particle).  Derived fields that
// the pair terms read: rho = m / omega, p and c from the Tait EOS, e = E -
// |v|^2 / 2.  One reverse step, for a step that started from the hash-sorted
// state s (saved or recomputed) with rates R and time step dt:
//   1. MOTION:  cotangent of the updated state -> direct cotangent of s and
//               cotangents of the rates (k_motion_adj);
//   2. pair pass reverse (sph_interact_adjoint) -> cotangents of x, v, omega
//               and of the derived rho, p, c, e;
//   3. EOS:     fold the derived cotangents into m, omega, v, E and c0
//               (k_eos_adj, deterministic sum for c0);
//   4. permute: scatter back through the step's sort permutation.
// Elementwise and HBM-bound; arithmetic in FP64, storage in the form's
// precision.
#include "common.hpp"

namespace sph {

namespace {

template <typename real, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_motion_adj(PV<real> s, RV<real> R, const double *__restrict__ dtp,
                                                       AV<real> bar, RV<real> rbar)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const double dt = *dtp;
    double r[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) r[k] = (double)R.hi[k][i] + (SPLIT ? (double)R.lo[k][i] : 0.0);
    const double m = (double)s.m[i];
    const double E = s.E[i];
    double v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = (double)s.v[a][i];
    // forward: mn = m + dt r0, V = m v + dt r_{1+a}, vn = V / mn,
    // EE = m E + dt r4, En = EE / mn, wn = w + dt r5, xn = x + dt vn
    const double mn = m + dt * r[0];
    const double minv = 1.0 / mn;
    double vn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) vn[a] = (m * v[a] + dt * r[1 + a]) * minv;
    const double En = (m * E + dt * r[4]) * minv;
    // reverse
    double bxn[3], bvn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bxn[a] = (double)bar.x[a][i];
        bvn[a] = (double)bar.v[a][i] + dt * bxn[a];
    }
    const double bEn = (double)bar.E[i];
    const double bwn = (double)bar.w[i];
    double bmn = (double)bar.m[i] - bEn * En * minv;
    double bV[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bmn -= bvn[a] * vn[a] * minv;
        bV[a] = bvn[a] * minv;
    }
    const double bEE = bEn * minv;
    double bm = bmn + bEE * E;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bm += bV[a] * v[a];
        bar.x[a][i] = (real)bxn[a];
        bar.v[a][i] = (real)(bV[a] * m);
        rbar.hi[1 + a][i] = (real)(dt * bV[a]);
    }
    bar.m[i] = (real)bm;
    bar.E[i] = (real)(bEE * m);
    bar.w[i] = (real)bwn;
    rbar.hi[0][i] = (real)(dt * bmn);
    rbar.hi[4][i] = (real)(dt * bEE);
    rbar.hi[5][i] = (real)(dt * bwn);
}

// Fold the cotangents of rho, p, c, e into m, omega, v, E; clear them; the
// per-block partial of d/dc0 goes to partials (slot 0).  Tait fluid:
// p' = c^2, c' = c (gamma - 1) / (2 rho), and p and c scale as c0^2 and c0;
// linear solid EOS: p' = K / rho0 and a constant c (no c0 term).
template <typename real>
__global__ __launch_bounds__(kBlock) void k_eos_adj(Params P, PV<real> s, AV<real> bar, double *__restrict__ partials)
{
    __shared__ double sh[kBlock / kWave];
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    double dc0 = 0.0;
    if (i < s.n) {
        // every input is read before the first write (bar could alias s as
        // far as the compiler knows, and a read issued after a write would
        // wait out the write's round trip)
        const double m = (double)s.m[i], w = (double)s.w[i];
        const double bp = (double)bar.p[i], bc = (double)bar.c[i], be = (double)bar.e[i];
        double brho = (double)bar.rho[i];
        const double bm = (double)bar.m[i], bw = (double)bar.w[i], bE = (double)bar.E[i];
        double vv[3], bv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            vv[a] = (double)s.v[a][i];
            bv[a] = (double)bar.v[a][i];
        }
        const double rho = m / w;
        if (P.material == SPH_FLUID_TAIT) {
            const double sr = rho / P.rho0;
            double s_gam, s_half;
            tait_powers<real>(P, sr, s_gam, s_half);
            const double p = P.B * (s_gam - 1.0);
            const double c = P.c0 * s_half;
            brho += bp * c * c + bc * c * (P.gamma - 1.0) / (2.0 * rho);
            dc0 = (bp * 2.0 * p + bc * c) / P.c0;
        } else {
            brho += bp * P.K / P.rho0;
        }
        bar.m[i] = (real)(bm + brho / w);
        bar.w[i] = (real)(bw - brho * rho / w);
        bar.E[i] = (real)(bE + be);
#pragma unroll
        for (int a = 0; a < 3; ++a) bar.v[a][i] = (real)(bv[a] - be * vv[a]);
        bar.rho[i] = real(0);
        bar.p[i] = real(0);
        bar.c[i] = real(0);
        bar.e[i] = real(0);
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) dc0 += __shfl_down(dc0, off, kWave);
    if (lane == 0) sh[wave] = dc0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / kWave; ++k) t += sh[k];
        partials[blockIdx.x] = t;
    }
}

// Reverse of the stress stage (Jaumann rate and J2 radial return with linear
// hardening), one thread per particle.  s holds the stress and plastic strain
// BEFORE the stage, L the velocity gradient it used; on entry bar.S and
// bar.ep hold the cotangents of the stage's outputs S+ and eps_p+, on return
// those of its inputs S and eps_p, and Lbar (overwritten) that of L.  On the
// plastic branch S+ = f S_tr with f = (1 - a) + a sy / q, a = 3G / (3G + H),
// and eps_p+ = eps_p + (q - sy) / (3G + H), sy = Y0 + H eps_p.
template <typename real, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_stress_adj(Params P, PV<real> s, RV<real> R, const double *__restrict__ dtp,
                                                       AV<real> bar, RV<real> Lbar)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const double dt = *dtp, G = P.G;
    double L[3][3], D[3][3], W[3][3], S[3][3];
#pragma unroll
    for (int k = 0; k < 9; ++k) L[k / 3][k % 3] = (double)R.Lhi[k][i] + (SPLIT ? (double)R.Llo[k][i] : 0.0);
    const double s6[6] = {(double)s.S[0][i], (double)s.S[1][i], (double)s.S[2][i],
                          (double)s.S[3][i], (double)s.S[4][i], (double)s.S[5][i]};
    const int sym[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            D[a][b] = 0.5 * (L[a][b] + L[b][a]);
            W[a][b] = 0.5 * (L[a][b] - L[b][a]);
            S[a][b] = s6[sym[a][b]];
        }
    const double tr = D[0][0] + D[1][1] + D[2][2];
    double St[3][3];
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
            St[a][b] = S[a][b] + dt * (2.0 * G * (D[a][b] - (a == b ? tr / 3.0 : 0.0)) + ws - sw);
        }
    const double t6[6] = {St[0][0], St[1][1], St[2][2], St[0][1], St[0][2], St[1][2]};
    const double J = (t6[0] * t6[0] + t6[1] * t6[1] + t6[2] * t6[2]) + 2.0 * (t6[3] * t6[3] + t6[4] * t6[4] + t6[5] * t6[5]);
    const double q = sqrt(1.5 * J);
    const double ep = (double)s.ep[i];
    const double sy = P.Y0 + P.H * ep;
    double bS6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) bS6[k] = (double)bar.S[k][i];
    const double bep_out = (double)bar.ep[i];
    double bt6[6], bep = bep_out;
    if (q > sy) {
        const double a = 3.0 * G / (3.0 * G + P.H);
        const double f = (1.0 - a) + a * sy / q;
        double bf = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            bt6[k] = f * bS6[k];
            bf += bS6[k] * t6[k];
        }
        const double bq = -bf * a * sy / (q * q) + bep_out / (3.0 * G + P.H);
        const double bsy = bf * a / q - bep_out / (3.0 * G + P.H);
        bep += P.H * bsy;
        // q = sqrt(3/2 J), J counts the off-diagonals twice
#pragma unroll
        for (int k = 0; k < 6; ++k) bt6[k] += bq * 1.5 * (k < 3 ? 1.0 : 2.0) * t6[k] / q;
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) bt6[k] = bS6[k];
    }
    // full symmetric cotangent B of S_tr (a stored off-diagonal splits in two halves)
    double B[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) B[a][b] = a == b ? bt6[sym[a][b]] : 0.5 * bt6[sym[a][b]];
    // S_tr = S + dt (2G dev D + W S - S W):
    //   Sbar += B + dt (B W - W B),  Lbar = dt (2G dev B + B S - S B)
    const double trB = B[0][0] + B[1][1] + B[2][2];
    double bSf[3][3], bL[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double bw = 0.0, wb = 0.0, bs = 0.0, sb = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                bw += B[a][k] * W[k][b];
                wb += W[a][k] * B[k][b];
                bs += B[a][k] * S[k][b];
                sb += S[a][k] * B[k][b];
            }
            bSf[a][b] = B[a][b] + dt * (bw - wb);
            bL[a][b] = dt * (2.0 * G * (B[a][b] - (a == b ? trB / 3.0 : 0.0)) + bs - sb);
        }
    const double out6[6] = {bSf[0][0], bSf[1][1], bSf[2][2], bSf[0][1] + bSf[1][0], bSf[0][2] + bSf[2][0],
                            bSf[1][2] + bSf[2][1]};
#pragma unroll
    for (int k = 0; k < 6; ++k) bar.S[k][i] = (real)out6[k];
    bar.ep[i] = (real)bep;
#pragma unroll
    for (int k = 0; k < 9; ++k) Lbar.Lhi[k][i] = (real)bL[k / 3][k % 3];
}

// One workgroup folds the block partials in a fixed order and adds to *out.
__global__ __launch_bounds__(kBlock) void k_sum_into(const double *__restrict__ partials, uint32_t nblocks,
                                                     double *__restrict__ out)
{
    __shared__ double sh[kBlock];
    double t = 0.0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += kBlock) t += partials[b];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out += sh[0];
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_permute(uint32_t n, const uint32_t *__restrict__ perm, AV<real> in,
                                                    AV<real> out)
{
    uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    uint32_t d = perm[k];
    // every cotangent is read before the first write (in and out could
    // alias as far as the compiler knows, and a read issued after a write
    // would wait out the write's round trip)
    real x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, S[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (in.x[a]) x[a] = in.x[a][k];
        if (in.v[a]) v[a] = in.v[a][k];
    }
    const real m = in.m ? in.m[k] : real(0), w = in.w ? in.w[k] : real(0), E = in.E ? in.E[k] : real(0);
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (in.S[q]) S[q] = in.S[q][k];
    const real ep = in.ep ? in.ep[k] : real(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (in.x[a]) out.x[a][d] = x[a];
        if (in.v[a]) out.v[a][d] = v[a];
    }
    if (in.m) out.m[d] = m;
    if (in.w) out.w[d] = w;
    if (in.E) out.E[d] = E;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (in.S[q]) out.S[q][d] = S[q];
    if (in.ep) out.ep[d] = ep;
}

// Seed of a reverse pass: the cotangent of the objective with respect to the
// final state, scaled by `scale`; every non-NULL field of bar is written.
// Kinetic energy J = sum m |v|^2 / 2: v-bar = scale m v, m-bar = scale |v|^2 / 2.
// Tagged mean z: z-bar = scale / ntag (stag) on the particles whose id is
// tagged.  FP64 arithmetic, rounded once to the form's precision.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_seed(int objective, PV<real> s, const uint8_t *__restrict__ tag,
                                                 uint32_t tag_len, double stag, double scale, AV<real> bar)
{
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    double vb[3] = {0.0, 0.0, 0.0}, mb = 0.0, zb = 0.0;
    if (objective == SPH_OBJ_KINETIC_ENERGY) {
        const double v[3] = {(double)s.v[0][i], (double)s.v[1][i], (double)s.v[2][i]};
        const double sm = scale * (double)s.m[i];
#pragma unroll
        for (int d = 0; d < 3; ++d) vb[d] = sm * v[d];
        mb = scale * 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    } else {
        const uint32_t id = s.id[i];
        zb = (id < tag_len && tag[id]) ? stag : 0.0;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (bar.x[d]) bar.x[d][i] = (real)(d == 2 ? zb : 0.0);
        if (bar.v[d]) bar.v[d][i] = (real)vb[d];
    }
    if (bar.m) bar.m[i] = (real)mb;
    real *zero[] = {bar.w, bar.E, bar.rho, bar.p, bar.c, bar.e, bar.S[0], bar.S[1], bar.S[2], bar.S[3], bar.S[4],
                    bar.S[5], bar.ep};
#pragma unroll
    for (int k = 0; k < 13; ++k)
        if (zero[k]) zero[k][i] = real(0);
}

// Reverse of taking the velocities as the input at fixed specific internal
// energy (E = e + |v|^2 / 2 with e held): v-bar += E-bar v, in place.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_input_v_adj(PV<real> s, AV<real> bar)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const double Eb = (double)bar.E[i];
    double v[3], vb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v[d] = (double)s.v[d][i];
        vb[d] = (double)bar.v[d][i];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) bar.v[d][i] = (real)(vb[d] + Eb * v[d]);
}

template <typename real>
hipError_t go(const Params &P, int stage, const sph_particles &p, const sph_rates &r, const double *dt,
              const sph_adjoint &bar, const sph_rates &rbar, double *pbar, const Workspace &ws, hipStream_t s)
{
    constexpr bool SPLIT = sizeof(real) == 4;
    uint32_t blocks = div_up(p.n, kBlock);
    if (stage == SPH_STAGE_MOTION) {
        if (blocks)
            k_motion_adj<real, SPLIT><<<blocks, kBlock, 0, s>>>(view<real>(p), view<real>(r), dt, view<real>(bar),
                                                                view<real>(rbar));
    } else if (stage == SPH_STAGE_STRESS) {
        if (blocks)
            k_stress_adj<real, SPLIT><<<blocks, kBlock, 0, s>>>(P, view<real>(p), view<real>(r), dt, view<real>(bar),
                                                                view<real>(rbar));
    } else if (stage == SPH_STAGE_INPUT_VELOCITY) {
        if (blocks) k_input_v_adj<real><<<blocks, kBlock, 0, s>>>(view<real>(p), view<real>(bar));
    } else {
        if (blocks) k_eos_adj<real><<<blocks, kBlock, 0, s>>>(P, view<real>(p), view<real>(bar), ws.partials);
        k_sum_into<<<1, kBlock, 0, s>>>(ws.partials, blocks, pbar);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_integrate_adjoint(const Params &P, int prec, int stage, const sph_particles &p, const sph_rates &r,
                                    const double *dt, const sph_adjoint &bar, const sph_rates &rbar, double *pbar,
                                    const Workspace &ws, hipStream_t s)
{
    if (prec == SPH_FP64) return go<double>(P, stage, p, r, dt, bar, rbar, pbar, ws, s);
    return go<float>(P, stage, p, r, dt, bar, rbar, pbar, ws, s);
}

hipError_t launch_objective_adjoint(int prec, int objective, const sph_particles &p, const uint8_t *tag,
                                    uint32_t tag_len, uint32_t ntag, double scale, const sph_adjoint &bar,
                                    hipStream_t s)
{
    const uint32_t blocks = div_up(p.n, kBlock);
    const double stag = ntag ? scale / (double)ntag : 0.0;
    if (prec == SPH_FP64)
        k_seed<double><<<blocks, kBlock, 0, s>>>(objective, view<double>(p), tag, tag_len, stag, scale,
                                                 view<double>(bar));
    else
        k_seed<float><<<blocks, kBlock, 0, s>>>(objective, view<float>(p), tag, tag_len, stag, scale,
                                                view<float>(bar));
    return hipGetLastError();
}

hipError_t launch_permute_adjoint(int prec, uint32_t n, const uint32_t *perm, const sph_adjoint &in,
                                  const sph_adjoint &out, hipStream_t s)
{
    uint32_t blocks = div_up(n, kBlock);
    if (prec == SPH_FP64)
        k_permute<double><<<blocks, kBlock, 0, s>>>(n, perm, view<double>(in), view<double>(out));
    else
        k_permute<float><<<blocks, kBlock, 0, s>>>(n, perm, view<float>(in), view<float>(out));
    return hipGetLastError();
}

}  // namespace sph
