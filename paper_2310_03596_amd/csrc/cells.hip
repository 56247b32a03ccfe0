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

__global__ __launch_bounds__(kBlock) void k_hash(Grid g, uint32_t n, const double *__restrict__ x0,
                                                 const double *__restrict__ x1,
                                                 const double *__restrict__ x2, uint32_t *keys,
                                                 uint32_t *vals)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(x0[i], g.o[0], g.L, g.nx);
    int cy = cell_coord(x1[i], g.o[1], g.L, g.ny);
    int cz = cell_coord(x2[i], g.o[2], g.L, g.nz);
    keys[i] = (uint32_t)cx + (uint32_t)g.nx * ((uint32_t)cy + (uint32_t)g.ny * (uint32_t)cz);
    vals[i] = i;
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
                                                   uint32_t *__restrict__ perm, int split)
{
    uint32_t k = blockIdx.x * kBlock + threadIdx.x;
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

// start[c] = lower bound of c in the sorted keys, c = 0..ncells.
__global__ __launch_bounds__(kBlock) void k_cell_start(const uint32_t *__restrict__ keys, uint32_t n,
                                                       uint32_t ncells, uint32_t *__restrict__ start)
{
    uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c > ncells) return;
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    start[c] = lo;
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
__global__ __launch_bounds__(kScanBlock) void k_scan_counts(uint32_t *__restrict__ counts, uint32_t nblocks,
                                                            uint32_t *__restrict__ nb)
{
    const uint32_t tot = block_scan_row<kScanBlock, 8>(counts, nblocks);
    if (threadIdx.x == 0) *nb = tot;
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
    uint32_t s = bidx[k];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (out.x[d]) out.x[d][k] = in.x[d][s];
        if (out.off[d]) out.off[d][k] = in.off[d][s];
        if (out.v[d]) out.v[d][k] = in.v[d][s];
    }
    if (out.hash) out.hash[k] = in.hash[s];
    if (out.id) out.id[k] = in.id[s];
    if (out.m) out.m[k] = in.m[s];
    if (out.w) out.w[k] = in.w[s];
    if (out.rho) out.rho[k] = in.rho[s];
    if (out.p) out.p[k] = in.p[s];
    if (out.c) out.c[k] = in.c[s];
    if (out.e) out.e[k] = in.e[s];
    if (out.E) out.E[k] = in.E[s];
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (out.S[q]) out.S[q][k] = in.S[q][s];
    if (out.ep) out.ep[k] = in.ep[s];
}

}  // namespace

hipError_t launch_build_cells(const Grid &g, int prec, const sph_particles &in, const sph_particles &out,
                              uint32_t *perm, uint32_t *start, const Workspace &ws, hipStream_t s)
{
    uint32_t n = in.n;
    uint32_t blocks = div_up(n, kBlock);
    if (n > 0) {
        k_hash<<<blocks, kBlock, 0, s>>>(g, n, in.x[0], in.x[1], in.x[2], ws.keys[0], ws.vals[0]);
        const int cur = radix_sort(ws, n, g.ncells, s);
        if (prec == SPH_FP64)
            k_gather<double><<<blocks, kBlock, 0, s>>>(g, view<double>(in), view<double>(out), ws.keys[cur],
                                                       ws.vals[cur], perm, 0);
        else
            k_gather<float><<<blocks, kBlock, 0, s>>>(g, view<float>(in), view<float>(out), ws.keys[cur],
                                                      ws.vals[cur], perm, 1);
        k_cell_start<<<div_up((uint64_t)g.ncells + 1, kBlock), kBlock, 0, s>>>(ws.keys[cur], n, g.ncells,
                                                                                start);
    } else {
        k_cell_start<<<div_up((uint64_t)g.ncells + 1, kBlock), kBlock, 0, s>>>(ws.keys[0], 0, g.ncells, start);
    }
    return hipGetLastError();
}

hipError_t launch_mark_boundary(const Grid &g, const sph_particles &local, const uint32_t *rstart,
                                uint32_t *comm, uint32_t *bidx, uint32_t cap, uint32_t *nb,
                                const Workspace &ws, hipStream_t s)
{
    uint32_t n = local.n;
    uint32_t blocks = div_up(n > 0 ? n : 1, kBlock);
    k_mark<<<blocks, kBlock, 0, s>>>(g, n, local.hash, rstart, comm, ws.counts);
    k_scan_counts<<<1, kScanBlock, 0, s>>>(ws.counts, blocks, nb);
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
                                        uint32_t *comm, uint32_t *bidx, uint32_t cap, uint32_t *nb, hipStream_t s)
{
    uint32_t *counts = nullptr;
    hipError_t e = scratch_of_current_device(&counts);
    if (e != hipSuccess) return e;
    Workspace ws{};
    ws.counts = counts;
    return launch_mark_boundary(g, local, rstart, comm, bidx, cap, nb, ws, s);
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
