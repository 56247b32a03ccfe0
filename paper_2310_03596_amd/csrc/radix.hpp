// Stable least-significant-digit radix sort of (key, index) pairs held in the
// workspace, with digits of 8 to 10 bits chosen so that a key takes as few
// passes as possible (two for keys of up to 20 bits).  Each pass: (1)
// per-tile digit histograms in LDS, (2) one workgroup per digit scans that
// digit's counts over tiles, (3) each tile ranks its keys stably with
// wavefront ballots (one ballot per digit bit gives every lane the mask of
// lanes holding the same digit; popcount of the lanes below gives the rank
// inside the wavefront) and scatters.  Used for the bucket sort (Section I)
// and the sort by balancing hash (Section III.A).
#pragma once
#include "common.hpp"

namespace sph {

namespace {

#ifndef SPH_SORT_WIDE
#define SPH_SORT_WIDE 2
#endif
// Keys per thread of a tile: 10-bit digits take tiles SPH_SORT_WIDE times as
// long, so the per-tile work that scales with the 1024 digits (clearing and
// writing the tile's histogram, reading it back for the scatter) stays small
// next to the keys (measured on 8 M + 2 M keys: 2 and 4 equal, both 5 %
// faster than 1).
template <int D>
constexpr int sort_items = D >= 10 ? SPH_SORT_WIDE * kSortItems : kSortItems;

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan over the NT threads of a block; every thread gets `total`.
template <int NT = kBlock>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t &total)
{
    __shared__ uint32_t wsum[NT / kWave];
    int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        uint32_t s = wsum[w];
        before += (w < wave) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

// In-place exclusive scan of row[0, len) by one block of NT threads; returns
// the row's total.  The row is taken in tiles of NT * B entries: a tile is
// loaded with coalesced reads (all in flight at once) into LDS, each thread
// then scans B consecutive entries of it (entry e sits at e + e / B, so the
// threads' strided LDS reads hit distinct banks), one block scan gives every
// thread its offset, and the tile is written back coalesced.  A tile costs
// one memory round trip and one block scan, where a scan 256 entries at a
// time costs one of each per 256 entries.
template <int NT, int B>
__device__ inline uint32_t block_scan_row(uint32_t *__restrict__ row, uint32_t len)
{
    constexpr uint32_t T = (uint32_t)NT * B;
    __shared__ uint32_t sh[T + T / B];
    const uint32_t tid = threadIdx.x;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < len; base += T) {
        uint32_t q[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const uint32_t e = (uint32_t)k * NT + tid;
            q[k] = base + e < len ? row[base + e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const uint32_t e = (uint32_t)k * NT + tid;
            sh[e + e / B] = q[k];
        }
        __syncthreads();
        uint32_t v[B];
        uint32_t sum = 0;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            v[u] = sh[tid * (B + 1) + u];
            sum += v[u];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl_scan<NT>(sum, tot);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            sh[tid * (B + 1) + u] = run;
            run += v[u];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const uint32_t e = (uint32_t)k * NT + tid;
            if (base + e < len) row[base + e] = sh[e + e / B];
        }
        carry += tot;
        __syncthreads();   // the next tile overwrites the LDS copy
    }
    return carry;
}

// Adds one chunk of a tile (the kBlock keys' digits d, BINS for no key) to
// the tile's histogram h in LDS.  Runs of equal digits in consecutive lanes
// add their length once (the keys arrive nearly sorted, step after step, so
// runs are long and the LDS atomics do not serialise on one address).
template <int D>
__device__ inline void hist_chunk(uint32_t *h, uint32_t d, bool valid)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t prev = __shfl_up(d, 1, kWave);
    const bool head = lane == 0 || d != prev;
    const uint64_t heads = __ballot(head);
    const uint64_t above = heads & ~((2ull << lane) - 1ull);   // heads past this lane (2 << 63 wraps to 0)
    const int next = above ? __ffsll((unsigned long long)above) - 1 : kWave;
    if (valid && head) atomicAdd(&h[d], (uint32_t)(next - lane));
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_upsweep(const uint32_t *__restrict__ keys, uint32_t n, int shift,
                                                    uint32_t *__restrict__ hist, uint32_t tiles)
{
    constexpr int BINS = 1 << D;
    __shared__ uint32_t h[BINS];
    for (int b = threadIdx.x; b < BINS; b += kBlock) h[b] = 0;
    __syncthreads();
    constexpr int IT = sort_items<D>;
    // Consecutive tiles run on one XCD: a digit's counts of 32 consecutive
    // tiles share one 128-byte line of hist, which is then written (here)
    // and read (in the scatter) through a single L2 instead of eight.
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t base = tile * (kBlock * IT);
    uint32_t keyv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t e = base + it * kBlock + threadIdx.x;
        keyv[it] = e < n ? keys[e] : 0u;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t e = base + it * kBlock + threadIdx.x;
        const bool valid = e < n;
        hist_chunk<D>(h, valid ? (keyv[it] >> shift) & (BINS - 1) : (uint32_t)BINS, valid);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < BINS; b += kBlock) hist[(size_t)b * tiles + tile] = h[b];
}

// One workgroup per digit: exclusive scan of that digit's tile counts.
__global__ __launch_bounds__(kBlock) void k_scan_digit(uint32_t *__restrict__ hist, uint32_t tiles,
                                                       uint32_t *__restrict__ totals)
{
    const uint32_t tot = block_scan_row<kBlock, 16>(hist + (size_t)blockIdx.x * tiles, tiles);
    if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_downsweep(const uint32_t *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin,
                                                      uint32_t *__restrict__ kout,
                                                      uint32_t *__restrict__ vout, uint32_t n, int shift,
                                                      const uint32_t *__restrict__ hist, uint32_t tiles,
                                                      const uint32_t *__restrict__ totals)
{
    constexpr int BINS = 1 << D;
    constexpr int PT = BINS / kBlock;   // digits per thread in the bookkeeping
    static_assert(BINS % kBlock == 0, "digits must cover the block");
    constexpr int NW = kBlock / kWave;
    __shared__ uint32_t dbase[BINS];
    __shared__ uint32_t run[BINS];
    __shared__ uint32_t cnt[NW][BINS];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    // the tile's keys and values are read first: their loads overlap the
    // digit-base bookkeeping below and each other (a load issued inside the
    // loop would wait out a full round trip behind every barrier)
    constexpr int IT = sort_items<D>;
    // the tile order of the histogram pass (same XCD for consecutive tiles,
    // so the runs they write side by side in each digit's range fill whole
    // lines in one L2)
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t base = tile * (kBlock * IT);
    uint32_t keyv[IT], valv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t e = base + it * kBlock + tid;
        keyv[it] = e < n ? kin[e] : 0u;
        valv[it] = e < n ? vin[e] : 0u;
    }
    // digit bases of this tile: exclusive scan of the digit totals (each
    // thread holds PT consecutive digits) plus the tile's offset in its digit
    uint32_t loc[PT];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        loc[k] = sum;
        sum += totals[tid * PT + k];
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(sum, tot);
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int d = tid * PT + k;
        dbase[d] = ex + loc[k] + hist[(size_t)d * tiles + tile];
        run[d] = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) cnt[w][d] = 0;
    }
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t e = base + it * kBlock + tid;
        const bool valid = e < n;
        const uint32_t key = keyv[it];
        const uint32_t val = valv[it];
        uint32_t d = (key >> shift) & (BINS - 1);
        // Rank among the lanes of this wavefront with the same digit.  When the
        // valid lanes' digits do not decrease (the usual case: the keys arrive
        // nearly sorted), each digit is one run of lanes and the rank is the
        // distance from the run's first lane; otherwise one ballot per digit
        // bit gives each lane the mask of lanes holding its digit.
        const uint32_t prev = __shfl_up(d, 1, kWave);
        const uint64_t vmask = __ballot(valid);
        uint32_t rank, count;
        bool leader;
        if (__ballot(valid && lane > 0 && d < prev) == 0ull) {
            const bool head = valid && (lane == 0 || d != prev);
            const uint64_t heads = __ballot(head) | ~vmask;   // invalid lanes end the last run
            const uint64_t upto = heads & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull));
            const int start = 63 - __clzll((long long)upto);
            const uint64_t above = heads & ~(lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull));
            const int next = above ? __ffsll((unsigned long long)above) - 1 : kWave;
            rank = (uint32_t)(lane - start);
            count = (uint32_t)(next - start);
            leader = valid && next == lane + 1;
        } else {
            uint64_t mask = vmask;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                bool bit = (d >> b) & 1u;
                uint64_t bm = __ballot(bit);
                mask &= bit ? bm : ~bm;
            }
            rank = (uint32_t)__popcll(mask & below);
            count = (uint32_t)__popcll(mask);
            leader = valid && ((mask >> lane) == 1ull);
        }
        if (leader) cnt[wave][d] = count;
        __syncthreads();
        if (valid) {
            uint32_t pre = run[d];
            for (int w = 0; w < wave; ++w) pre += cnt[w][d];
            uint32_t pos = dbase[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const int b = tid * PT + k;
            uint32_t add = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                add += cnt[w][b];
                cnt[w][b] = 0;
            }
            run[b] += add;
        }
        __syncthreads();
    }
}

// Keys per tile and tiles of a pass with D-bit digits over n keys.
template <int D>
inline uint32_t sort_tiles(uint32_t n)
{
    return div_up(n, (uint64_t)kBlock * sort_items<D>);   // at most the workspace's tiles
}

// One LSD pass with D-bit digits starting at bit `shift`; with hist_ready the
// per-tile digit counts are already in ws.hist (written by the kernel that
// produced the keys, over the same tiles).
template <int D>
void sort_pass(const Workspace &ws, uint32_t n, int shift, int cur, hipStream_t s, bool hist_ready = false)
{
    const uint32_t tiles = sort_tiles<D>(n);
    if (!hist_ready) k_upsweep<D><<<tiles, kBlock, 0, s>>>(ws.keys[cur], n, shift, ws.hist, tiles);
    k_scan_digit<<<1u << D, kBlock, 0, s>>>(ws.hist, tiles, ws.totals);
    k_downsweep<D><<<tiles, kBlock, 0, s>>>(ws.keys[cur], ws.vals[cur], ws.keys[cur ^ 1], ws.vals[cur ^ 1], n,
                                            shift, ws.hist, tiles, ws.totals);
}

// Number of bits needed for keys below nkeys.
inline int key_bits(uint32_t nkeys)
{
    int b = 0;
    while (b < 32 && (uint64_t(1) << b) < nkeys) ++b;
    return b;
}

// Digit width (8 to 10 bits) of a sort of keys below nkeys, in as few passes
// as possible.
inline int radix_digit_bits(uint32_t nkeys)
{
    const int bits = key_bits(nkeys);
    const int passes = bits > 0 ? (bits + kMaxRadixBits - 1) / kMaxRadixBits : 1;
    const int dbits = (bits + passes - 1) / passes;
    return dbits < 8 ? 8 : dbits;
}

// Sorts (ws.keys[0], ws.vals[0]) of n entries, keys below nkeys; returns the
// index of the key/value buffer pair that holds the result.  With
// first_hist, the first pass's per-tile digit counts are already in ws.hist.
inline int radix_sort(const Workspace &ws, uint32_t n, uint32_t nkeys, hipStream_t s, bool first_hist = false)
{
    const int bits = key_bits(nkeys);
    const int passes = bits > 0 ? (bits + kMaxRadixBits - 1) / kMaxRadixBits : 1;
    const int dbits = radix_digit_bits(nkeys);
    int cur = 0;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = ps * dbits;
        const bool ready = first_hist && ps == 0;
        if (dbits == 8)
            sort_pass<8>(ws, n, shift, cur, s, ready);
        else if (dbits == 9)
            sort_pass<9>(ws, n, shift, cur, s, ready);
        else
            sort_pass<10>(ws, n, shift, cur, s, ready);
        cur ^= 1;
    }
    return cur;
}

}  // namespace

}  // namespace sph
