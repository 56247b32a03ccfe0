// Bucket hashing, stable radix sort, reorder, bucket table (Section I and
// step a of Section II), communication hash and boundary compaction (step c)
// and the boundary payload packing for step d.  The sort itself is in
// radix.hpp.
#include <mutex>

#include "radix.hpp"

namespace sph {

namespace {

__device__ inline int cell_coord(double x, double o, double L, int n)
{
    double t = floor((x - o) / L);
    if (!(t >= 0.0)) return 0;
    if (t > (double)(n - 1)) return n - 1;
    return (int)t;
}

__device__ inline uint32_t bucket_of(const Grid &g, double x, double y, double z)
{
    const int cx = cell_coord(x, g.o[0], g.L, g.nx);
    const int cy = cell_coord(y, g.o[1], g.L, g.ny);
    const int cz = cell_coord(z, g.o[2], g.L, g.nz);
    return (uint32_t)cx + (uint32_t)g.nx * ((uint32_t)cy + (uint32_t)g.ny * (uint32_t)cz);
}

// Bucket hash of every particle (keys, with values the particle indices),
// and in the same pass the first radix pass's per-tile counts of the lowest
// D-bit digit (same tiles and tile order as the histogram kernel), so the
// sort starts at its digit scan.  A tile of 2,048 or 4,096 keys is one
// workgroup of 1,024 threads (a column-sized sort has only a few hundred
// tiles, so the sort's own 256-thread workgroups would leave the chip short
// of wavefronts).  Also clears the count of long empty-bucket runs that the
// bucket table queues for the reorder.
constexpr int kHashBlock = 1024;
template <int D>
__global__ __launch_bounds__(kHashBlock) void k_hash_hist(Grid g, uint32_t n, const double *__restrict__ x0,
                                                          const double *__restrict__ x1,
                                                          const double *__restrict__ x2,
                                                          uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                          uint32_t *__restrict__ hist, uint32_t tiles,
                                                          uint32_t *__restrict__ ngaps)
{
    constexpr int BINS = 1 << D;
    constexpr int TILE = kBlock * sort_items<D>;
    static_assert(TILE % kHashBlock == 0, "a tile is whole rounds of the workgroup");
    constexpr int IT = TILE / kHashBlock;
    __shared__ uint32_t h[BINS];
    for (int b = threadIdx.x; b < BINS; b += kHashBlock) h[b] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ngaps = 0u;
    __syncthreads();
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t base = tile * (uint32_t)TILE;
    double p[IT][3];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t e = base + it * kHashBlock + threadIdx.x;
        const bool valid = e < n;
        p[it][0] = valid ? x0[e] : 0.0;
        p[it][1] = valid ? x1[e] : 0.0;
        p[it][2] = valid ? x2[e] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t e = base + it * kHashBlock + threadIdx.x;
        const bool valid = e < n;
        const uint32_t key = bucket_of(g, p[it][0], p[it][1], p[it][2]);
        if (valid) {
            keys[e] = key;
            vals[e] = e;
        }
        hist_chunk<D>(h, valid ? key & (BINS - 1) : (uint32_t)BINS, valid);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < BINS; b += kHashBlock) hist[(size_t)b * tiles + tile] = h[b];
}

// Float offset from the bucket corner, ((x - o) - c L) evaluated in IEEE
// double without contraction, rounded once to float.
__device__ inline float corner_offset(double x, double o, uint32_t c, double L)
{
#pragma clang fp contract(off)
    return (float)((x - o) - (double)c * L);
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_gather(Grid g, PV<real> in, PV<real> out,
                                                   const uint32_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ vals,
                                                   uint32_t *__restrict__ perm, int split,
                                                   uint32_t *__restrict__ start,
                                                   const uint32_t *__restrict__ ngaps,
                                                   const uint3 *__restrict__ gaps, uint32_t gap_cap)
{
    uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    {
        // the bucket table's long runs of empty buckets, each spread over
        // every thread of the grid
        uint32_t m = *ngaps;
        m = m < gap_cap ? m : gap_cap;
        const uint32_t T = gridDim.x * kBlock;
        for (uint32_t r = 0; r < m; ++r) {
            const uint3 gp = gaps[r];
            for (uint64_t c = (uint64_t)gp.x + k; c <= gp.y; c += T) start[c] = gp.z;   // no wrap near 2^32
        }
    }
    if (k >= in.n) return;
    const uint32_t s = vals[k];
    const uint32_t h = keys[k];
    // every read is issued before the first write: the writes could alias
    // the reads as far as the compiler knows, and a read issued after a write
    // would wait for the write's round trip
    const uint32_t id = in.id[s];
    double x[3];
    real v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        x[d] = in.x[d][s];
        v[d] = in.v[d][s];
    }
    const real m = in.m[s], w = in.w[s], rho = in.rho[s], p = in.p[s], c = in.c[s], e = in.e[s];
    const double E = in.E[s];
    const bool solid = in.S[0] != nullptr;
    real S[6] = {}, ep = 0;
    if (solid) {
#pragma unroll
        for (int q = 0; q < 6; ++q) S[q] = in.S[q][s];
        ep = in.ep[s];
    }
    perm[k] = s;
    out.hash[k] = h;
    out.id[k] = id;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        out.x[d][k] = x[d];
        out.v[d][k] = v[d];
    }
    out.m[k] = m;
    out.w[k] = w;
    out.rho[k] = rho;
    out.p[k] = p;
    out.c[k] = c;
    out.e[k] = e;
    out.E[k] = E;
    if (solid) {
#pragma unroll
        for (int q = 0; q < 6; ++q) out.S[q][k] = S[q];
        out.ep[k] = ep;
    }
    if (split) {
        uint32_t cx = h % (uint32_t)g.nx;
        uint32_t cy = (h / (uint32_t)g.nx) % (uint32_t)g.ny;
        uint32_t cz = h / ((uint32_t)g.nx * (uint32_t)g.ny);
        out.off[0][k] = corner_offset(x[0], g.o[0], cx, g.L);
        out.off[1][k] = corner_offset(x[1], g.o[1], cy, g.L);
        out.off[2][k] = corner_offset(x[2], g.o[2], cz, g.L);
    }
}

// Bucket table from the sorted keys: start[c] is the number of keys below c,
// so the buckets c with keys[i-1] < c <= keys[i] all start at i (with
// keys[-1] = -1 and keys[n] = ncells).  Each thread takes kStartItems values
// of i (its keys loaded at once) and writes the starts of their runs of
// buckets: short runs itself, longer ones with its workgroup, and runs of
// more than kLongRun empty buckets (wide empty regions of the box) go to a
// list that the reorder kernel, launched next, fills with all its threads;
// if the list is full the workgroup fills the run.  Every start[c] is
// written exactly once, and no thread walks a long run alone.
constexpr uint32_t kShortRun = 8;
constexpr uint32_t kLongRun = 16 * kBlock;
constexpr int kStartItems = 2;
__global__ __launch_bounds__(kBlock) void k_cell_start(const uint32_t *__restrict__ keys, uint32_t n,
                                                       uint32_t ncells, uint32_t *__restrict__ start,
                                                       uint32_t *__restrict__ ngaps, uint3 *__restrict__ gaps,
                                                       uint32_t gap_cap)
{
    __shared__ uint3 q[kBlock * kStartItems];
    __shared__ uint32_t nq;
    if (threadIdx.x == 0) nq = 0;
    // consecutive key ranges on one XCD: the starts they write side by side
    // fill whole lines in one L2
    const uint32_t base = xcd_tile(blockIdx.x, gridDim.x) * (uint32_t)(kBlock * kStartItems);
    uint32_t kp[kStartItems], kc[kStartItems];
#pragma unroll
    for (int it = 0; it < kStartItems; ++it) {
        const uint32_t i = base + it * kBlock + threadIdx.x;
        kp[it] = i >= 1 && i <= n ? keys[i - 1] : 0u;
        kc[it] = i < n ? keys[i] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kStartItems; ++it) {
        const uint32_t i = base + it * kBlock + threadIdx.x;
        if (i > n) break;
        const uint32_t lo = i == 0 ? 0u : kp[it] + 1u;
        const uint32_t hi = i == n ? ncells : kc[it];   // buckets lo..hi start at i
        if (lo > hi) continue;
        const uint32_t len = hi - lo + 1u;
        if (len <= kShortRun) {
            for (uint32_t c = lo; c <= hi; ++c) start[c] = i;
            continue;
        }
        bool listed = false;
        if (len > kLongRun) {
            const uint32_t k = atomicAdd(ngaps, 1u);
            if (k < gap_cap) {
                gaps[k] = make_uint3(lo, hi, i);
                listed = true;
            }
        }
        if (!listed) q[atomicAdd(&nq, 1u)] = make_uint3(lo, hi, i);
    }
    __syncthreads();
    const uint32_t m = nq;
    for (uint32_t k = 0; k < m; ++k) {
        const uint3 r = q[k];
        // 64-bit index: the stride must not wrap past r.y near 2^32
        for (uint64_t c = (uint64_t)r.x + threadIdx.x; c <= r.y; c += kBlock) start[c] = r.z;
    }
}

// start[0..ncells] = 0 (no particles).
__global__ __launch_bounds__(kBlock) void k_start_empty(uint32_t ncells, uint32_t *__restrict__ start)
{
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c <= ncells) start[c] = 0u;
}

// ------------------------------------------------------------ step c: mark

__global__ __launch_bounds__(kBlock) void k_mark(Grid g, uint32_t n, const uint32_t *__restrict__ hash,
                                                 const uint32_t *__restrict__ rstart,
                                                 uint32_t *__restrict__ comm, uint32_t *__restrict__ counts)
{
    __shared__ uint32_t wc[kBlock / kWave];
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    bool flag = false;
    if (i < n) {
        const uint32_t h = hash[i];
        const uint32_t nx = (uint32_t)g.nx, nxy = nx * (uint32_t)g.ny;
        const uint32_t cz = h / nxy, rz = h - cz * nxy;
        const uint32_t cy = rz / nx, cx = rz - cy * nx;
        // Row (dy, dz) of the target's 27 buckets spans the source range
        // [start[h + dy nx + dz nxy - (cx > 0)], start[h + dy nx + dz nxy + 1
        // + (cx + 1 < nx)]) (up to three adjacent buckets); it is occupied iff
        // that range is non-empty.  The bounds of all nine rows are loaded
        // before any is tested, so the test costs one memory round trip; a row
        // outside the grid reads start[0] instead and is ignored.
        const uint32_t a = h - (cx > 0 ? 1u : 0u), b = h + 1u + (cx + 1u < nx ? 1u : 0u);
        const bool yin[3] = {cy > 0, true, cy + 1u < (uint32_t)g.ny};
        const bool zin[3] = {cz > 0 && cz <= (uint32_t)g.nz, cz < (uint32_t)g.nz, cz + 1u < (uint32_t)g.nz};
        uint32_t lo[9], hi[9];
        bool inside[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const int dz = r / 3 - 1, dy = r % 3 - 1;
            inside[r] = zin[dz + 1] && yin[dy + 1];
            const uint32_t off = (uint32_t)dy * nx + (uint32_t)dz * nxy;   // modular: dy, dz may be -1
            lo[r] = rstart[inside[r] ? a + off : 0u];
            hi[r] = rstart[inside[r] ? b + off : 0u];
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) flag = flag || (inside[r] && hi[r] > lo[r]);
        comm[i] = flag ? h : g.ncells;
    }
    uint64_t m = __ballot(flag);
    if ((threadIdx.x & (kWave - 1)) == 0) wc[threadIdx.x / kWave] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += wc[w];
        counts[blockIdx.x] = t;
    }
}

// Single workgroup: exclusive scan of block counts, total to *nb.
constexpr int kScanBlock = 1024;
// nb: the entries the compaction writes (at most cap), the count the list's
// consumers read; nflag (optional): every flagged particle, above *nb when
// the list overflows.
__global__ __launch_bounds__(kScanBlock) void k_scan_counts(uint32_t *__restrict__ counts, uint32_t nblocks,
                                                            uint32_t *__restrict__ nb, uint32_t cap,
                                                            uint32_t *__restrict__ nflag)
{
    const uint32_t tot = block_scan_row<kScanBlock, 8>(counts, nblocks);
    if (threadIdx.x == 0) {
        *nb = tot < cap ? tot : cap;
        if (nflag) *nflag = tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_compact(uint32_t n, uint32_t G, const uint32_t *__restrict__ comm,
                                                    const uint32_t *__restrict__ counts,
                                                    uint32_t *__restrict__ bidx, uint32_t cap)
{
    __shared__ uint32_t wc[kBlock / kWave];
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    bool flag = i < n && comm[i] != G;
    uint64_t m = __ballot(flag);
    if (lane == 0) wc[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t pre = counts[blockIdx.x];
    for (int w = 0; w < wave; ++w) pre += wc[w];
    uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t k = pre + (uint32_t)__popcll(m & below);
    if (flag && k < cap) bidx[k] = i;
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_pack(PV<real> in, const uint32_t *__restrict__ bidx,
                                                 const uint32_t *__restrict__ nb, PV<real> out)
{
    uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    uint32_t cnt = *nb;
    if (k >= out.n || k >= cnt) return;
    const uint32_t s = bidx[k];
    if (s >= in.n) return;   // a listed index outside the array names no particle
    // every field is read before the first write (the payload could alias
    // the particles as far as the compiler knows, and a read issued after a
    // write would wait out the write's round trip)
    double x[3] = {0.0, 0.0, 0.0};
    real off[3] = {0, 0, 0}, v[3] = {0, 0, 0}, S[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (out.x[d]) x[d] = in.x[d][s];
        if (out.off[d]) off[d] = in.off[d][s];
        if (out.v[d]) v[d] = in.v[d][s];
    }
    const uint32_t hash = out.hash ? in.hash[s] : 0u, id = out.id ? in.id[s] : 0u;
    const real m = out.m ? in.m[s] : real(0), w = out.w ? in.w[s] : real(0);
    const real rho = out.rho ? in.rho[s] : real(0), p = out.p ? in.p[s] : real(0);
    const real c = out.c ? in.c[s] : real(0), e = out.e ? in.e[s] : real(0);
    const double E = out.E ? in.E[s] : 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (out.S[q]) S[q] = in.S[q][s];
    const real ep = out.ep ? in.ep[s] : real(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (out.x[d]) out.x[d][k] = x[d];
        if (out.off[d]) out.off[d][k] = off[d];
        if (out.v[d]) out.v[d][k] = v[d];
    }
    if (out.hash) out.hash[k] = hash;
    if (out.id) out.id[k] = id;
    if (out.m) out.m[k] = m;
    if (out.w) out.w[k] = w;
    if (out.rho) out.rho[k] = rho;
    if (out.p) out.p[k] = p;
    if (out.c) out.c[k] = c;
    if (out.e) out.e[k] = e;
    if (out.E) out.E[k] = E;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (out.S[q]) out.S[q][k] = S[q];
    if (out.ep) out.ep[k] = ep;
}

}  // namespace

hipError_t launch_build_cells(const Grid &g, int prec, const sph_particles &in, const sph_particles &out,
                              uint32_t *perm, uint32_t *start, const Workspace &ws, hipStream_t s)
{
    uint32_t n = in.n;
    uint32_t blocks = div_up(n, kBlock);
    if (n > 0) {
        // the list of long empty-bucket runs takes the histogram area once the
        // sort is done; its count sits in the first entry of counts
        uint32_t *ngaps = ws.counts;
        uint3 *gaps = reinterpret_cast<uint3 *>(ws.hist);
        const uint32_t gap_cap = (uint32_t)(((uint64_t)kMaxRadixBins * div_up(n, kSortTile)) / 3u);
        const int D = radix_digit_bits(g.ncells);
        if (D == 8)
            k_hash_hist<8><<<sort_tiles<8>(n), kHashBlock, 0, s>>>(g, n, in.x[0], in.x[1], in.x[2], ws.keys[0],
                                                               ws.vals[0], ws.hist, sort_tiles<8>(n), ngaps);
        else if (D == 9)
            k_hash_hist<9><<<sort_tiles<9>(n), kHashBlock, 0, s>>>(g, n, in.x[0], in.x[1], in.x[2], ws.keys[0],
                                                               ws.vals[0], ws.hist, sort_tiles<9>(n), ngaps);
        else
            k_hash_hist<10><<<sort_tiles<10>(n), kHashBlock, 0, s>>>(g, n, in.x[0], in.x[1], in.x[2], ws.keys[0],
                                                                 ws.vals[0], ws.hist, sort_tiles<10>(n), ngaps);
        const int cur = radix_sort(ws, n, g.ncells, s, true);
        // the reorder also fills the long empty runs: enough threads that each
        // takes at most 16 buckets of the longest, whatever n
        const uint64_t gblocks64 = div_up((uint64_t)g.ncells + 1, (uint64_t)kBlock * 16u);
        const uint32_t gblocks = blocks > gblocks64 ? blocks : (uint32_t)gblocks64;
        k_cell_start<<<div_up((uint64_t)n + 1, (uint64_t)kBlock * kStartItems), kBlock, 0, s>>>(
            ws.keys[cur], n, g.ncells, start, ngaps, gaps, gap_cap);
        if (prec == SPH_FP64)
            k_gather<double><<<gblocks, kBlock, 0, s>>>(g, view<double>(in), view<double>(out), ws.keys[cur],
                                                        ws.vals[cur], perm, 0, start, ngaps, gaps, gap_cap);
        else
            k_gather<float><<<gblocks, kBlock, 0, s>>>(g, view<float>(in), view<float>(out), ws.keys[cur],
                                                       ws.vals[cur], perm, 1, start, ngaps, gaps, gap_cap);
    } else {
        k_start_empty<<<div_up((uint64_t)g.ncells + 1, kBlock), kBlock, 0, s>>>(g.ncells, start);
    }
    return hipGetLastError();
}

hipError_t launch_mark_boundary(const Grid &g, const sph_particles &local, const uint32_t *rstart,
                                uint32_t *comm, uint32_t *bidx, uint32_t cap, uint32_t *nb, uint32_t *nflag,
                                const Workspace &ws, hipStream_t s)
{
    uint32_t n = local.n;
    uint32_t blocks = div_up(n > 0 ? n : 1, kBlock);
    k_mark<<<blocks, kBlock, 0, s>>>(g, n, local.hash, rstart, comm, ws.counts);
    k_scan_counts<<<1, kScanBlock, 0, s>>>(ws.counts, blocks, nb, cap, nflag);
    k_compact<<<blocks, kBlock, 0, s>>>(n, g.ncells, comm, ws.counts, bidx, cap);
    return hipGetLastError();
}

// Block counts of the mark and compaction for callers that cannot allocate
// (sph_mark_boundary_noalloc): one copy per GPU, held until the process
// ends.  k_mark writes every entry the scan and the compaction read, so
// nothing needs clearing between calls; calls that overlap on one GPU race.
static __device__ __align__(256) uint32_t scratch[kNoAllocMarkMax / kBlock + 1];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_dev[kMaxDevices] = {};

// The address of this GPU's copy of `scratch`, looked up once per device with
// that device current (the host-side name is not a device address).
hipError_t scratch_of_current_device(uint32_t **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}
}  // namespace

hipError_t launch_mark_boundary_noalloc(const Grid &g, const sph_particles &local, const uint32_t *rstart,
                                        uint32_t *comm, uint32_t *bidx, uint32_t cap, uint32_t *nb,
                                        uint32_t *nflag, hipStream_t s)
{
    uint32_t *counts = nullptr;
    hipError_t e = scratch_of_current_device(&counts);
    if (e != hipSuccess) return e;
    Workspace ws{};
    ws.counts = counts;
    return launch_mark_boundary(g, local, rstart, comm, bidx, cap, nb, nflag, ws, s);
}

hipError_t launch_pack(int prec, const sph_particles &local, const uint32_t *bidx, const uint32_t *nb,
                       const sph_particles &payload, hipStream_t s)
{
    uint32_t blocks = div_up(payload.n, kBlock);
    if (blocks == 0) return hipSuccess;
    if (prec == SPH_FP64)
        k_pack<double><<<blocks, kBlock, 0, s>>>(view<double>(local), bidx, nb, view<double>(payload));
    else
        k_pack<float><<<blocks, kBlock, 0, s>>>(view<float>(local), bidx, nb, view<float>(payload));
    return hipGetLastError();
}

}  // namespace sph
