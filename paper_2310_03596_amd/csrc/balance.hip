// Periodic particle swapping between two GPUs (Section III.A), the part one
// GPU computes: the centre of gravity of its particles, each particle's
// balancing hash towards the other GPU's centre, the selection of the
// k = min(n+_own, n+_other) particles of largest hash (a stable sort by
// descending hash, reusing the bucket-sort machinery), and the pairwise
// exchange of the selected particles between two particle arrays (the
// single-device stand-in for the send/receive between the GPUs).
//
// The balancing hash, with e = Cg_other - Cg_own and M the midpoint: the
// projection of x - M on e, measured in half distances, scaled to hmax:
//   t = ((x0 - M0) e0 + (x1 - M1) e1) + (x2 - M2) e2,  ee = |e|^2,
//   v = hmax (2 t / ee),  hash = t > 0 ? min(ceil(v), hmax) : 0,
// in IEEE binary64 without contraction, so every particle's integer hash is
// decided exactly as a plain CPU evaluation of the same expression decides it.
#include "radix.hpp"

namespace sph {

namespace {

constexpr int kCg = 4;   // sum m x, sum m y, sum m z, sum m

// Sums of one block in a fixed order (wavefront butterfly, then waves in turn).
__device__ inline void block_sum4(double r[kCg], double *out)
{
    __shared__ double sh[kCg][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kCg; ++k) {
        double v = r[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
        if (lane == 0) sh[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kCg; ++k) {
            double v = sh[k][0];
            for (int w = 1; w < kBlock / kWave; ++w) v += sh[k][w];
            out[k] = v;
        }
    }
}

constexpr uint32_t kCgBlocks = 1024;   // fixed partial count: the sum order depends on n only

// Each thread sums the particles i = t, t + T, t + 2T, ... (T = grid threads)
// in that order, then the block folds its threads in a fixed order.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_cg_partial(PV<real> s, double *__restrict__ partials)
{
    double r[kCg] = {0.0, 0.0, 0.0, 0.0};
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < s.n; i += stride) {
        const double m = (double)s.m[i];
        r[0] += m * s.x[0][i];
        r[1] += m * s.x[1][i];
        r[2] += m * s.x[2][i];
        r[3] += m;
    }
    block_sum4(r, partials + (size_t)blockIdx.x * kDiagPartial);
}

__global__ __launch_bounds__(kBlock) void k_cg_final(const double *__restrict__ partials, uint32_t nblocks,
                                                     double *__restrict__ cg)
{
    double r[kCg] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
        for (int k = 0; k < kCg; ++k) r[k] += partials[(size_t)b * kDiagPartial + k];
    }
    __shared__ double out[kCg];
    block_sum4(r, out);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sm = out[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) cg[d] = sm > 0.0 ? out[d] / sm : 0.0;
        cg[3] = sm;
    }
}

__device__ inline uint32_t balance_hash(const double x[3], const double e[3], const double M[3], double ee,
                                        uint32_t hmax)
{
#pragma clang fp contract(off)
    if (!(ee > 0.0)) return 0u;
    const double t = ((x[0] - M[0]) * e[0] + (x[1] - M[1]) * e[1]) + (x[2] - M[2]) * e[2];
    if (!(t > 0.0)) return 0u;
    const double v = (double)hmax * ((t + t) / ee);
    return v >= (double)hmax ? hmax : (uint32_t)ceil(v);
}

// Balancing hash of every particle and the per-block count of positive hashes.
__global__ __launch_bounds__(kBlock) void k_bhash(uint32_t n, const double *__restrict__ x0,
                                                  const double *__restrict__ x1, const double *__restrict__ x2,
                                                  const double *__restrict__ cg_own,
                                                  const double *__restrict__ cg_other, uint32_t hmax,
                                                  uint32_t *__restrict__ bhash, uint32_t *__restrict__ counts)
{
    double e[3], M[3];
    {
#pragma clang fp contract(off)
        for (int d = 0; d < 3; ++d) {
            e[d] = cg_other[d] - cg_own[d];
            M[d] = 0.5 * (cg_own[d] + cg_other[d]);
        }
    }
    double ee;
    {
#pragma clang fp contract(off)
        ee = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
    }
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    uint32_t h = 0;
    if (i < n) {
        const double x[3] = {x0[i], x1[i], x2[i]};
        h = balance_hash(x, e, M, ee, hmax);
        bhash[i] = h;
    }
    // positive hashes of this block (integer: the total is order-independent)
    __shared__ uint32_t wc[kBlock / kWave];
    const uint64_t b = __ballot(i < n && h > 0);
    if ((threadIdx.x & (kWave - 1)) == 0) wc[threadIdx.x / kWave] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int w = 0; w < kBlock / kWave; ++w) c += wc[w];
        counts[blockIdx.x] = c;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_counts(const uint32_t *__restrict__ counts, uint32_t nblocks,
                                                       uint32_t *__restrict__ total)
{
    __shared__ uint32_t sh[kBlock];
    uint32_t c = 0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += kBlock) c += counts[b];
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = sh[0];
}

// Sort key hmax - hash (an ascending sort puts the largest hashes first,
// ties in index order) and the identity index.
__global__ __launch_bounds__(kBlock) void k_sel_keys(uint32_t n, const uint32_t *__restrict__ bhash, uint32_t hmax,
                                                     uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t h = bhash[i];
    keys[i] = hmax - (h < hmax ? h : hmax);
    vals[i] = i;
}

// k = min(own, other) (both at most n); the first k sorted indices.
__global__ __launch_bounds__(kBlock) void k_select(uint32_t n, const uint32_t *__restrict__ sorted_vals,
                                                   const uint32_t *__restrict__ npos_own,
                                                   const uint32_t *__restrict__ npos_other,
                                                   uint32_t *__restrict__ sel, uint32_t *__restrict__ k_out)
{
    uint32_t k = *npos_own < *npos_other ? *npos_own : *npos_other;
    k = k < n ? k : n;
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t < k) sel[t] = sorted_vals[t];
    if (t == 0) *k_out = k;
}

// A field of both selected particles, read before any write (the two
// arrays could alias as far as the compiler knows, and a read issued after a
// write would wait out the write's round trip); absent fields stay absent.
template <typename T>
struct FieldPair {
    T a, b;
};
template <typename T>
__device__ inline FieldPair<T> read_pair(const T *a, uint32_t i, const T *b, uint32_t j)
{
    FieldPair<T> r{T(0), T(0)};
    if (a && b) {
        r.a = a[i];
        r.b = b[j];
    }
    return r;
}
template <typename T>
__device__ inline void write_swapped(T *a, uint32_t i, T *b, uint32_t j, const FieldPair<T> &q)
{
    if (a && b) {
        a[i] = q.b;
        b[j] = q.a;
    }
}

// Exchange particle sel_a[t] of a with particle sel_b[t] of b, every field.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_swap(PV<real> a, const uint32_t *__restrict__ sel_a, PV<real> b,
                                                 const uint32_t *__restrict__ sel_b,
                                                 const uint32_t *__restrict__ k_dev, uint32_t k_max)
{
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    uint32_t k = *k_dev;
    k = k < k_max ? k : k_max;
    if (t >= k) return;
    const uint32_t i = sel_a[t], j = sel_b[t];
    if (i >= a.n || j >= b.n) return;   // out-of-range selections are ignored
    FieldPair<double> x[3];
    FieldPair<float> off[3];
    FieldPair<real> v[3], S[6];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        x[d] = read_pair(a.x[d], i, b.x[d], j);
        off[d] = read_pair(a.off[d], i, b.off[d], j);
        v[d] = read_pair(a.v[d], i, b.v[d], j);
    }
    const FieldPair<uint32_t> hash = read_pair(a.hash, i, b.hash, j), id = read_pair(a.id, i, b.id, j);
    const FieldPair<real> m = read_pair(a.m, i, b.m, j), w = read_pair(a.w, i, b.w, j);
    const FieldPair<real> rho = read_pair(a.rho, i, b.rho, j), p = read_pair(a.p, i, b.p, j);
    const FieldPair<real> c = read_pair(a.c, i, b.c, j), e = read_pair(a.e, i, b.e, j);
    const FieldPair<double> E = read_pair(a.E, i, b.E, j);
#pragma unroll
    for (int q = 0; q < 6; ++q) S[q] = read_pair(a.S[q], i, b.S[q], j);
    const FieldPair<real> ep = read_pair(a.ep, i, b.ep, j);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        write_swapped(a.x[d], i, b.x[d], j, x[d]);
        write_swapped(a.off[d], i, b.off[d], j, off[d]);
        write_swapped(a.v[d], i, b.v[d], j, v[d]);
    }
    write_swapped(a.hash, i, b.hash, j, hash);
    write_swapped(a.id, i, b.id, j, id);
    write_swapped(a.m, i, b.m, j, m);
    write_swapped(a.w, i, b.w, j, w);
    write_swapped(a.rho, i, b.rho, j, rho);
    write_swapped(a.p, i, b.p, j, p);
    write_swapped(a.c, i, b.c, j, c);
    write_swapped(a.e, i, b.e, j, e);
    write_swapped(a.E, i, b.E, j, E);
#pragma unroll
    for (int q = 0; q < 6; ++q) write_swapped(a.S[q], i, b.S[q], j, S[q]);
    write_swapped(a.ep, i, b.ep, j, ep);
}

// ------------------------------------------------ several particle types
// Section III.B: every type is balanced on its own with the single-type rule,
// towards biased centres Cg'_t = alpha Cg_all + (1 - alpha) Cg_t (the paper
// takes alpha = 0.1), which pull the decomposition of each type towards that
// of all the particles.  Particles whose type is ntypes or more take no part
// (no centre, hash 0, never selected).

constexpr int kTypeRec = kCg * (kMaxTypes + 1);   // per type, then all types
static_assert(8 * kTypeRec * (kSortTile / kBlock) <= 4 * kMaxRadixBins,
              "per-block type partials fit the sort-histogram area of the workspace");

// Each thread sums its particles (i = t, t + T, ...) into the sums of every
// type, adding an exact zero to the types other than its own, so each type's
// sum runs over its own particles in index order; the block then folds its
// threads in a fixed order.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_cgt_partial(PV<real> s, const uint8_t *__restrict__ type, uint32_t ntypes,
                                                        double *__restrict__ partials)
{
    double r[kMaxTypes + 1][kCg] = {};
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < s.n; i += stride) {
        const uint32_t t = type[i];
        if (t >= ntypes) continue;
        const double m = (double)s.m[i];
        const double q[kCg] = {m * s.x[0][i], m * s.x[1][i], m * s.x[2][i], m};
#pragma unroll
        for (int u = 0; u < kMaxTypes; ++u) {
#pragma unroll
            for (int k = 0; k < kCg; ++k) r[u][k] += (uint32_t)u == t ? q[k] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kCg; ++k) r[kMaxTypes][k] += q[k];
    }
    __shared__ double sh[kMaxTypes + 1][kCg][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int u = 0; u <= kMaxTypes; ++u) {
#pragma unroll
        for (int k = 0; k < kCg; ++k) {
            double v = r[u][k];
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
            if (lane == 0) sh[u][k][wave] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kTypeRec) {
        const int u = threadIdx.x / kCg, k = threadIdx.x % kCg;
        double v = sh[u][k][0];
        for (int w = 1; w < kBlock / kWave; ++w) v += sh[u][k][w];
        partials[(size_t)blockIdx.x * kTypeRec + threadIdx.x] = v;
    }
}

// Folds the block records (thread j takes blocks j, j + kBlock, ... in turn,
// then a fixed tree) and forms the centres: record t < ntypes holds Cg'_t and
// the type's mass (zeros for a type without mass), record ntypes holds Cg_all
// and the total mass.
__global__ __launch_bounds__(kBlock) void k_cgt_final(const double *__restrict__ partials, uint32_t nblocks,
                                                      uint32_t ntypes, double alpha, double *__restrict__ cg)
{
    __shared__ double tot[kTypeRec];
    __shared__ double sh[kTypeRec][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    double a[kTypeRec] = {};
    for (uint32_t b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
        for (int v = 0; v < kTypeRec; ++v) a[v] += partials[(size_t)b * kTypeRec + v];
    }
#pragma unroll
    for (int v = 0; v < kTypeRec; ++v) {
        double x = a[v];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_down(x, off, kWave);
        if (lane == 0) sh[v][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < kTypeRec) {
        double t = sh[threadIdx.x][0];
        for (int w = 1; w < kBlock / kWave; ++w) t += sh[threadIdx.x][w];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x <= ntypes) {
#pragma clang fp contract(off)
        const uint32_t u = threadIdx.x;
        const double *all = tot + kCg * kMaxTypes;
        const double *own = u < ntypes ? tot + kCg * u : all;
        const double ma = all[3], mo = own[3];
        double *out = cg + (size_t)kCg * u;
        for (int d = 0; d < 3; ++d) {
            const double ca = ma > 0.0 ? all[d] / ma : 0.0;
            const double co = mo > 0.0 ? own[d] / mo : 0.0;
            out[d] = u == ntypes ? ca : (mo > 0.0 ? alpha * ca + (1.0 - alpha) * co : 0.0);
        }
        out[3] = mo;
    }
}

// Balancing hash of every particle towards its type's centres, and the
// per-block count of positive hashes of every type.
__global__ __launch_bounds__(kBlock) void k_bhash_types(uint32_t n, const double *__restrict__ x0,
                                                        const double *__restrict__ x1,
                                                        const double *__restrict__ x2,
                                                        const uint8_t *__restrict__ type, uint32_t ntypes,
                                                        const double *__restrict__ cg_own,
                                                        const double *__restrict__ cg_other, uint32_t hmax,
                                                        uint32_t *__restrict__ bhash, uint32_t *__restrict__ counts)
{
    __shared__ double se[kMaxTypes][3], sm[kMaxTypes][3], see[kMaxTypes];
    __shared__ uint32_t cnt[kMaxTypes];
    if (threadIdx.x < ntypes) {
#pragma clang fp contract(off)
        const int u = threadIdx.x;
        for (int d = 0; d < 3; ++d) {
            se[u][d] = cg_other[kCg * u + d] - cg_own[kCg * u + d];
            sm[u][d] = 0.5 * (cg_own[kCg * u + d] + cg_other[kCg * u + d]);
        }
        see[u] = (se[u][0] * se[u][0] + se[u][1] * se[u][1]) + se[u][2] * se[u][2];
        cnt[u] = 0;
    }
    __syncthreads();
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const uint32_t t = type[i];
        uint32_t h = 0;
        if (t < ntypes) {
            const double x[3] = {x0[i], x1[i], x2[i]};
            h = balance_hash(x, se[t], sm[t], see[t], hmax);
            if (h > 0) atomicAdd(&cnt[t], 1u);   // integer counts: order-independent
        }
        bhash[i] = h;
    }
    __syncthreads();
    if (threadIdx.x < ntypes) counts[(size_t)blockIdx.x * ntypes + threadIdx.x] = cnt[threadIdx.x];
}

// One workgroup per type: the sum of its per-block counts.
__global__ __launch_bounds__(kBlock) void k_sum_type_counts(const uint32_t *__restrict__ counts, uint32_t nblocks,
                                                            uint32_t ntypes, uint32_t *__restrict__ total)
{
    __shared__ uint32_t sh[kBlock];
    const uint32_t u = blockIdx.x;
    uint32_t c = 0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += kBlock) c += counts[(size_t)b * ntypes + u];
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) total[u] = sh[0];
}

// Sort key type (hmax + 1) + (hmax - hash): an ascending sort groups the
// types in order, the largest hashes first within each, ties in index order;
// particles without a valid type sort last.
__global__ __launch_bounds__(kBlock) void k_sel_keys_types(uint32_t n, const uint32_t *__restrict__ bhash,
                                                           const uint8_t *__restrict__ type, uint32_t ntypes,
                                                           uint32_t hmax, uint32_t *__restrict__ keys,
                                                           uint32_t *__restrict__ vals)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = type[i];
    const uint32_t h = bhash[i];
    keys[i] = t < ntypes ? t * (hmax + 1) + (hmax - (h < hmax ? h : hmax)) : ntypes * (hmax + 1);
    vals[i] = i;
}

// start[t] = first sorted position of type t, for t = 0 .. ntypes (start[ntypes]
// = the number of particles with a valid type).
__global__ __launch_bounds__(kBlock) void k_type_start(const uint32_t *__restrict__ keys, uint32_t n, uint32_t hmax,
                                                       uint32_t ntypes, uint32_t *__restrict__ start)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i > n) return;
    auto type_at = [&](uint32_t k) {
        const uint32_t t = keys[k] / (hmax + 1);
        return t < ntypes ? t : ntypes;
    };
    const int prev = i == 0 ? -1 : (int)type_at(i - 1);
    const int cur = i == n ? (int)ntypes : (int)type_at(i);
    for (int t = prev + 1; t <= cur; ++t) start[t] = i;
}

// k_t = min(n+_own[t], n+_other[t], count_t) and the exclusive offsets of the
// per-type selections (off[ntypes] = their total).
__global__ void k_type_offsets(const uint32_t *__restrict__ start, const uint32_t *__restrict__ npos_own,
                               const uint32_t *__restrict__ npos_other, uint32_t ntypes,
                               uint32_t *__restrict__ k_out, uint32_t *__restrict__ off)
{
    if (threadIdx.x != 0) return;
    uint32_t o = 0;
    for (uint32_t t = 0; t < ntypes; ++t) {
        uint32_t k = npos_own[t] < npos_other[t] ? npos_own[t] : npos_other[t];
        const uint32_t c = start[t + 1] - start[t];
        k = k < c ? k : c;
        k_out[t] = k;
        off[t] = o;
        o += k;
    }
    off[ntypes] = o;
}

// The first k_t sorted indices of every type, one after another.
__global__ __launch_bounds__(kBlock) void k_select_types(uint32_t n, const uint32_t *__restrict__ keys,
                                                         const uint32_t *__restrict__ vals, uint32_t hmax,
                                                         uint32_t ntypes, const uint32_t *__restrict__ start,
                                                         const uint32_t *__restrict__ k_t,
                                                         const uint32_t *__restrict__ off,
                                                         uint32_t *__restrict__ sel)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = keys[i] / (hmax + 1);
    if (t >= ntypes) return;
    const uint32_t q = i - start[t];
    if (q < k_t[t]) sel[off[t] + q] = vals[i];
}

}  // namespace

hipError_t launch_centroid(int prec, const sph_particles &p, double *cg, const Workspace &ws, hipStream_t s)
{
    uint32_t blocks = div_up(p.n > 0 ? p.n : 1, kBlock);
    blocks = blocks < kCgBlocks ? blocks : kCgBlocks;   // the workspace holds one record per kBlock particles
    if (prec == SPH_FP64)
        k_cg_partial<double><<<blocks, kBlock, 0, s>>>(view<double>(p), ws.partials);
    else
        k_cg_partial<float><<<blocks, kBlock, 0, s>>>(view<float>(p), ws.partials);
    k_cg_final<<<1, kBlock, 0, s>>>(ws.partials, blocks, cg);
    return hipGetLastError();
}

hipError_t launch_balance_hash(const sph_particles &p, const double *cg_own, const double *cg_other,
                               uint32_t hmax, uint32_t *bhash, uint32_t *npos, const Workspace &ws, hipStream_t s)
{
    const uint32_t blocks = div_up(p.n > 0 ? p.n : 1, kBlock);
    k_bhash<<<blocks, kBlock, 0, s>>>(p.n, p.x[0], p.x[1], p.x[2], cg_own, cg_other, hmax, bhash, ws.counts);
    k_sum_counts<<<1, kBlock, 0, s>>>(ws.counts, blocks, npos);
    return hipGetLastError();
}

hipError_t launch_balance_select(uint32_t n, const uint32_t *bhash, uint32_t hmax, const uint32_t *npos_own,
                                 const uint32_t *npos_other, uint32_t *sel, uint32_t *k_out, const Workspace &ws,
                                 hipStream_t s)
{
    const uint32_t blocks = div_up(n > 0 ? n : 1, kBlock);
    int cur = 0;
    if (n > 0) {
        k_sel_keys<<<blocks, kBlock, 0, s>>>(n, bhash, hmax, ws.keys[0], ws.vals[0]);
        cur = radix_sort(ws, n, hmax + 1, s);
    }
    k_select<<<blocks, kBlock, 0, s>>>(n, ws.vals[cur], npos_own, npos_other, sel, k_out);
    return hipGetLastError();
}

hipError_t launch_swap(int prec, const sph_particles &a, const uint32_t *sel_a, const sph_particles &b,
                       const uint32_t *sel_b, const uint32_t *k_dev, uint32_t k_max, hipStream_t s)
{
    if (k_max == 0) return hipSuccess;
    const uint32_t blocks = div_up(k_max, kBlock);
    if (prec == SPH_FP64)
        k_swap<double><<<blocks, kBlock, 0, s>>>(view<double>(a), sel_a, view<double>(b), sel_b, k_dev, k_max);
    else
        k_swap<float><<<blocks, kBlock, 0, s>>>(view<float>(a), sel_a, view<float>(b), sel_b, k_dev, k_max);
    return hipGetLastError();
}

hipError_t launch_centroid_types(int prec, const sph_particles &p, const uint8_t *type, uint32_t ntypes, double alpha,
                                 double *cg, const Workspace &ws, hipStream_t s)
{
    uint32_t blocks = div_up(p.n > 0 ? p.n : 1, kBlock);
    blocks = blocks < kCgBlocks ? blocks : kCgBlocks;
    double *partials = reinterpret_cast<double *>(ws.hist);
    if (prec == SPH_FP64)
        k_cgt_partial<double><<<blocks, kBlock, 0, s>>>(view<double>(p), type, ntypes, partials);
    else
        k_cgt_partial<float><<<blocks, kBlock, 0, s>>>(view<float>(p), type, ntypes, partials);
    k_cgt_final<<<1, kBlock, 0, s>>>(partials, blocks, ntypes, alpha, cg);
    return hipGetLastError();
}

hipError_t launch_balance_hash_types(const sph_particles &p, const uint8_t *type, uint32_t ntypes,
                                     const double *cg_own, const double *cg_other, uint32_t hmax, uint32_t *bhash,
                                     uint32_t *npos, const Workspace &ws, hipStream_t s)
{
    const uint32_t blocks = div_up(p.n > 0 ? p.n : 1, kBlock);
    k_bhash_types<<<blocks, kBlock, 0, s>>>(p.n, p.x[0], p.x[1], p.x[2], type, ntypes, cg_own, cg_other, hmax,
                                            bhash, ws.hist);
    k_sum_type_counts<<<ntypes, kBlock, 0, s>>>(ws.hist, blocks, ntypes, npos);
    return hipGetLastError();
}

hipError_t launch_balance_select_types(uint32_t n, const uint8_t *type, uint32_t ntypes, const uint32_t *bhash,
                                       uint32_t hmax, const uint32_t *npos_own, const uint32_t *npos_other,
                                       uint32_t *sel, uint32_t *k_out, uint32_t *off, const Workspace &ws,
                                       hipStream_t s)
{
    const uint32_t blocks = div_up(n > 0 ? n : 1, kBlock);
    int cur = 0;
    if (n > 0) {
        k_sel_keys_types<<<blocks, kBlock, 0, s>>>(n, bhash, type, ntypes, hmax, ws.keys[0], ws.vals[0]);
        cur = radix_sort(ws, n, ntypes * (hmax + 1) + 1, s);
    }
    uint32_t *start = ws.totals;   // free once the sort has run
    k_type_start<<<div_up((uint64_t)n + 1, kBlock), kBlock, 0, s>>>(ws.keys[cur], n, hmax, ntypes, start);
    k_type_offsets<<<1, kWave, 0, s>>>(start, npos_own, npos_other, ntypes, k_out, off);
    if (n > 0)
        k_select_types<<<blocks, kBlock, 0, s>>>(n, ws.keys[cur], ws.vals[cur], hmax, ntypes, start, k_out, off,
                                                 sel);
    return hipGetLastError();
}

}  // namespace sph
