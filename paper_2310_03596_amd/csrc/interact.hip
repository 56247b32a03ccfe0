// Interaction loops: steps e (local-local) and f (local x received boundary
// particles) of Section II, FORCE and GRADIENT passes, FP64 and FP32-split.
//
// One lane per target particle.  The 27 surrounding buckets of a target are
// 9 rows of up to 3 buckets that are contiguous in hash order (the hash runs
// x-fastest), so each row is one contiguous source range [b, e) of the
// sorted arrays; rows are visited in ascending hash order, so every target
// sums its sources in ascending index.  In the FP32-split form the position
// difference is rebuilt from bucket indices and float offsets,
// d = (c_j - c_i) L + (off_j - off_i), which is exactly odd under i <-> j
// and never cancels the way a difference of large float positions would.
#include "pair.hpp"

namespace sph {

namespace {

// (2h)^2 predicate on FP64 differences without FMA contraction, identical
// to a left-to-right IEEE evaluation of ((dx dx + dy dy) + dz dz).
__device__ inline double r2_exact(double a, double b, double c)
{
#pragma clang fp contract(off)
    return (a * a + b * b) + c * c;
}

template <typename real>
__device__ inline real r2_of(const real d[3]);
template <>
__device__ inline double r2_of<double>(const double d[3])
{
    return r2_exact(d[0], d[1], d[2]);
}
template <>
__device__ inline float r2_of<float>(const float d[3])
{
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

template <typename real, int PASS, bool SOLID, bool SELF>
__global__ __launch_bounds__(kBlock) void k_interact(Params P, Grid g, PV<real> tg,
                                                     const uint32_t *__restrict__ tidx,
                                                     const uint32_t *__restrict__ ntdev, PV<real> sr,
                                                     const uint32_t *__restrict__ sstart, int zero_first,
                                                     RV<real> R)
{
    constexpr bool SPLIT = sizeof(real) == 4;
    constexpr int NOUT = PASS == SPH_PASS_FORCE ? 6 : 9;
    uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    uint32_t nt = tg.n;
    if (tidx) {
        uint32_t c = *ntdev;
        nt = c < nt ? c : nt;
    }
    if (t >= nt) return;
    const uint32_t i = tidx ? tidx[t] : t;

    PairK<real> K;
    K.hinv = (real)P.hinv;
    K.Fc = (real)P.Fc;
    K.beta = (real)P.beta;
    K.half_beta = (real)(0.5 * P.beta);
    const real R2 = (real)P.R2;
    const real Lf = SPLIT ? (real)g.Lf : real(0);

    const uint32_t h = tg.hash[i];
    const int cx = (int)(h % (uint32_t)g.nx);
    const int cy = (int)((h / (uint32_t)g.nx) % (uint32_t)g.ny);
    const int cz = (int)(h / ((uint32_t)g.nx * (uint32_t)g.ny));
    const int x0 = cx > 0 ? cx - 1 : 0;
    const int x1 = cx + 1 < g.nx ? cx + 1 : g.nx - 1;

    double xi[3];
    real oi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if constexpr (SPLIT)
            oi[d] = tg.off[d][i];
        else
            xi[d] = tg.x[d][i];
    }
    Part<real, SOLID> I;
    real vi[3];
    real wj_dummy = 0;
    (void)wj_dummy;
    if constexpr (PASS == SPH_PASS_FORCE) {
        load_part<real, SOLID>(tg, i, I);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) vi[d] = tg.v[d][i];
    }

    Sum<real> acc[NOUT];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        real *hi = PASS == SPH_PASS_FORCE ? R.hi[k] : R.Lhi[k];
        real *lo = PASS == SPH_PASS_FORCE ? R.lo[k] : R.Llo[k];
        acc[k].s = zero_first ? real(0) : hi[i];
        acc[k].c = (zero_first || !SPLIT) ? real(0) : lo[i];
    }

    for (int dz = -1; dz <= 1; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= g.nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = cy + dy;
            if (y < 0 || y >= g.ny) continue;
            const uint32_t row = (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
            const uint32_t jb = sstart[row + x0];
            const uint32_t je = sstart[row + x1 + 1];
            const uint32_t sA = sstart[row + cx];
            const uint32_t sB = sstart[row + cx + 1];
            const real ddy = (real)dy * Lf, ddz = (real)dz * Lf;
            for (uint32_t j = jb; j < je; ++j) {
                if (SELF && j == i) continue;
                real d[3];
                if constexpr (SPLIT) {
                    const int dcx = (int)(j >= sB) - (int)(j < sA);
                    d[0] = (real)dcx * Lf + (sr.off[0][j] - oi[0]);
                    d[1] = ddy + (sr.off[1][j] - oi[1]);
                    d[2] = ddz + (sr.off[2][j] - oi[2]);
                } else {
                    d[0] = sr.x[0][j] - xi[0];
                    d[1] = sr.x[1][j] - xi[1];
                    d[2] = sr.x[2][j] - xi[2];
                }
                const real r2 = r2_of<real>(d);
                if (!(r2 < R2)) continue;
                if constexpr (PASS == SPH_PASS_FORCE) {
                    Part<real, SOLID> J;
                    load_part<real, SOLID>(sr, j, J);
                    real o[6];
                    pair_force<real, SOLID>(d, r2, I, J, K, o);
#pragma unroll
                    for (int k = 0; k < 6; ++k) acc[k].add(o[k]);
                } else {
                    real vj[3] = {sr.v[0][j], sr.v[1][j], sr.v[2][j]};
                    real o[9];
                    pair_grad<real>(d, r2, vi, vj, sr.w[j], K, o);
#pragma unroll
                    for (int k = 0; k < 9; ++k) acc[k].add(o[k]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        real *hi = PASS == SPH_PASS_FORCE ? R.hi[k] : R.Lhi[k];
        real *lo = PASS == SPH_PASS_FORCE ? R.lo[k] : R.Llo[k];
        hi[i] = acc[k].s;
        if (SPLIT) lo[i] = acc[k].c;
    }
}

// Candidates and hits of one pass, same traversal and predicate as k_interact.
template <typename real, bool SELF>
__global__ __launch_bounds__(kBlock) void k_count(Params P, Grid g, PV<real> tg, const uint32_t *__restrict__ tidx,
                                                  const uint32_t *__restrict__ ntdev, PV<real> sr,
                                                  const uint32_t *__restrict__ sstart,
                                                  unsigned long long *__restrict__ counts)
{
    constexpr bool SPLIT = sizeof(real) == 4;
    uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    uint32_t nt = tg.n;
    if (tidx) {
        uint32_t c = *ntdev;
        nt = c < nt ? c : nt;
    }
    unsigned long long cand = 0, hits = 0;
    if (t < nt) {
        const uint32_t i = tidx ? tidx[t] : t;
        const real R2 = (real)P.R2;
        const real Lf = SPLIT ? (real)g.Lf : real(0);
        const uint32_t h = tg.hash[i];
        const int cx = (int)(h % (uint32_t)g.nx);
        const int cy = (int)((h / (uint32_t)g.nx) % (uint32_t)g.ny);
        const int cz = (int)(h / ((uint32_t)g.nx * (uint32_t)g.ny));
        const int x0 = cx > 0 ? cx - 1 : 0;
        const int x1 = cx + 1 < g.nx ? cx + 1 : g.nx - 1;
        double xi[3];
        real oi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if constexpr (SPLIT)
                oi[d] = tg.off[d][i];
            else
                xi[d] = tg.x[d][i];
        }
        for (int dz = -1; dz <= 1; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= g.nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= g.ny) continue;
                const uint32_t row = (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
                const uint32_t jb = sstart[row + x0], je = sstart[row + x1 + 1];
                const uint32_t sA = sstart[row + cx], sB = sstart[row + cx + 1];
                const real ddy = (real)dy * Lf, ddz = (real)dz * Lf;
                for (uint32_t j = jb; j < je; ++j) {
                    if (SELF && j == i) continue;
                    real d[3];
                    if constexpr (SPLIT) {
                        const int dcx = (int)(j >= sB) - (int)(j < sA);
                        d[0] = (real)dcx * Lf + (sr.off[0][j] - oi[0]);
                        d[1] = ddy + (sr.off[1][j] - oi[1]);
                        d[2] = ddz + (sr.off[2][j] - oi[2]);
                    } else {
                        d[0] = sr.x[0][j] - xi[0];
                        d[1] = sr.x[1][j] - xi[1];
                        d[2] = sr.x[2][j] - xi[2];
                    }
                    ++cand;
                    hits += (r2_of<real>(d) < R2) ? 1u : 0u;
                }
            }
        }
    }
    // wavefront sums, one atomic per wavefront (integer: order-independent)
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        cand += __shfl_down(cand, off, kWave);
        hits += __shfl_down(hits, off, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicAdd(&counts[0], cand);
        atomicAdd(&counts[1], hits);
    }
}

template <typename real, int PASS, bool SOLID>
hipError_t go(const Params &P, const Grid &g, const sph_particles &tg, const uint32_t *tidx,
              const uint32_t *nt, const sph_particles &sr, const uint32_t *sstart, bool self, int zero_first,
              const sph_rates &r, hipStream_t s)
{
    uint32_t blocks = div_up(tg.n, kBlock);
    if (blocks == 0) return hipSuccess;
    if (self)
        k_interact<real, PASS, SOLID, true><<<blocks, kBlock, 0, s>>>(P, g, view<real>(tg), tidx, nt,
                                                                      view<real>(sr), sstart, zero_first,
                                                                      view<real>(r));
    else
        k_interact<real, PASS, SOLID, false><<<blocks, kBlock, 0, s>>>(P, g, view<real>(tg), tidx, nt,
                                                                       view<real>(sr), sstart, zero_first,
                                                                       view<real>(r));
    return hipGetLastError();
}

template <typename real>
hipError_t go_prec(const Params &P, const Grid &g, int pass, const sph_particles &tg, const uint32_t *tidx,
                   const uint32_t *nt, const sph_particles &sr, const uint32_t *sstart, bool self,
                   int zero_first, const sph_rates &r, hipStream_t s)
{
    if (pass == SPH_PASS_GRADIENT)
        return go<real, SPH_PASS_GRADIENT, false>(P, g, tg, tidx, nt, sr, sstart, self, zero_first, r, s);
    if (P.material == SPH_SOLID_J2)
        return go<real, SPH_PASS_FORCE, true>(P, g, tg, tidx, nt, sr, sstart, self, zero_first, r, s);
    return go<real, SPH_PASS_FORCE, false>(P, g, tg, tidx, nt, sr, sstart, self, zero_first, r, s);
}

}  // namespace

hipError_t launch_count_pairs(const Params &P, const Grid &g, int prec, const sph_particles &tg,
                              const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr,
                              const uint32_t *sstart, bool self, uint64_t *counts, hipStream_t s)
{
    uint32_t blocks = div_up(tg.n, kBlock);
    if (blocks == 0) return hipSuccess;
    auto *c = reinterpret_cast<unsigned long long *>(counts);
    if (prec == SPH_FP64) {
        if (self)
            k_count<double, true><<<blocks, kBlock, 0, s>>>(P, g, view<double>(tg), tidx, nt, view<double>(sr),
                                                            sstart, c);
        else
            k_count<double, false><<<blocks, kBlock, 0, s>>>(P, g, view<double>(tg), tidx, nt, view<double>(sr),
                                                             sstart, c);
    } else {
        if (self)
            k_count<float, true><<<blocks, kBlock, 0, s>>>(P, g, view<float>(tg), tidx, nt, view<float>(sr),
                                                           sstart, c);
        else
            k_count<float, false><<<blocks, kBlock, 0, s>>>(P, g, view<float>(tg), tidx, nt, view<float>(sr),
                                                            sstart, c);
    }
    return hipGetLastError();
}

hipError_t launch_interact(const Params &P, const Grid &g, int prec, int pass, const sph_particles &tg,
                           const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr,
                           const uint32_t *sstart, bool self, int zero_first, const sph_rates &r, hipStream_t s)
{
    if (prec == SPH_FP64)
        return go_prec<double>(P, g, pass, tg, tidx, nt, sr, sstart, self, zero_first, r, s);
    return go_prec<float>(P, g, pass, tg, tidx, nt, sr, sstart, self, zero_first, r, s);
}

}  // namespace sph
