// Interaction loops: steps e (local-local) and f (local x received boundary
// particles) of Section II, FORCE and GRADIENT passes, FP64 and FP32-split.
//
// Neighbour search (Section I): the 27 buckets around a target are 9 rows of
// up to 3 buckets that are contiguous in hash order (the hash runs
// x-fastest), so each row is one contiguous range of the sorted sources.
//
// Work mapping (one lane per target, sources sorted by hash):
//   * the lanes of a wavefront are split into groups that share a bucket row
//     (cy, cz); consecutive sorted targets almost always do;
//   * for each of the 9 neighbour rows the group's candidates form one
//     contiguous source range (the union of the lanes' 3-bucket ranges); the
//     wavefront stages it in LDS with coalesced loads (in pages when it is
//     long), and then each lane walks its OWN 3-bucket range inside the page
//     (a per-lane LDS offset), all lanes in step, so a lane tests about its
//     27 buckets' worth of candidates instead of the whole union (about half
//     as many on the column workload);
//   * hits go to a per-lane list in LDS; when any lane's list is nearly full
//     (and at the end of the group) every lane evaluates the pair terms of its
//     listed hits.  Only ~1 candidate in 6 is a neighbour, so separating the
//     cheap test from the pair body (about a hundred operations) keeps the
//     body dense.
// A candidate outside a lane's own 3-bucket range is farther than one bucket
// side >= 2h on some axis and fails the distance test, so the lanes that run
// past the end of their range while the longest one finishes change no
// neighbour set.  Hits are listed, and summed, in ascending source index.  A
// pair with r = 0 (the target itself, or a coincident particle) adds
// nothing: its terms all carry F(0) = 0.
//
// The FP64 form's fluid FORCE pass over every target (and its census) runs
// k_pairs_mx instead: the same frame, bound, staging and pair body, with the
// candidate tests of 32 sources x 32 targets done as one matrix product on
// the matrix cores and two lanes per target, each summing every other run of
// four sources in ascending index; the two sums are then added.
//
// In the FP32-split form the position difference is rebuilt from bucket
// indices and float offsets, d = (c_j - c_i) L + (off_j - off_i), which is
// exactly odd under i <-> j and never cancels the way a difference of large
// float positions would; its pair sums accumulate in FP64 (full rate on
// gfx950: a convert and an add per term) and are stored as a float (hi, lo)
// pair.
#include <atomic>

#include "pair.hpp"

namespace sph {

namespace {

// Events recorded around every pair-kernel launch when set (sph_set_pair_events).
std::atomic<void *> g_pair_events[2] = {nullptr, nullptr};

#ifndef SPH_PAIR_BLOCK
#define SPH_PAIR_BLOCK 256
#endif
constexpr int kPairBlock = SPH_PAIR_BLOCK;  // targets per workgroup
constexpr int kWaves = kPairBlock / kWave;
// wavefronts whose list entries share one dword (so that a wavefront's 64
// lanes touch 64 different dwords)
constexpr int kHitWaves = kWaves < 4 ? kWaves : 4;
static_assert(kWaves % kHitWaves == 0 && kWaves % 2 == 0, "whole wavefront groups");
#ifndef SPH_PAIR_SUB
#define SPH_PAIR_SUB 4   // measured best of 4, 8, 16 on the 810k column (fewer live VGPRs)
#endif
constexpr int kSub = SPH_PAIR_SUB;         // candidates tested between list-fill checks
constexpr int kMaxWin = 12;                // staged pages whose hits a list can hold at once
// Per precision: source records staged per page (one neighbour row of a
// group, split into pages when longer) and listed hits per lane (u8 entries:
// the index inside the page).  A lane's hits arrive unevenly over the 9 rows
// (its position inside its bucket favours some rows), so a list that fills
// before the group ends forces every lane to evaluate while most lists are
// part full; lists longer than the ~80 neighbours of a particle at h = 1.3 dx
// are emptied once per group.  Sizes keep a workgroup's LDS (lists, page
// marks, pages, page tables) within 40 KB, four workgroups per CU; the page
// covers the row union of a group in about 97 % (FP32) and 70 % (FP64) of
// the cases on the column workload.
#ifndef SPH_PAIR_PAGE_F32
#define SPH_PAIR_PAGE_F32 160
#endif
#ifndef SPH_PAIR_CAP_F32
#define SPH_PAIR_CAP_F32 88
#endif
template <typename real>
struct Tune {
    static constexpr int page = sizeof(real) == 4 ? SPH_PAIR_PAGE_F32 : 160;
    static constexpr int cap = sizeof(real) == 4 ? SPH_PAIR_CAP_F32 : 88;
};
static_assert(Tune<float>::page + kSub <= 256 && Tune<double>::page + kSub <= 256, "page index must fit a u8 entry");
static_assert(Tune<float>::page % kSub == 0 && Tune<double>::page % kSub == 0, "reads stay below page + kSub");
static_assert(Tune<float>::cap <= 255 && Tune<double>::cap <= 255 && kMaxWin <= 255, "marks hold a u8 fill and slot");
constexpr int kPassAdjoint = 2;            // reverse mode of the FORCE pass
constexpr int kPassGradAdjoint = 4;        // reverse mode of the GRADIENT pass
constexpr int kPassCensus = 3;             // neighbour census of a FORCE or GRADIENT pass

// Census outputs: per target, the number of sources the pass evaluates
// (r^2 < (2h)^2 on the rebuilt d, the pairs at r = 0 included) and the sum,
// modulo 2^64, of mix64 of their ids; sid is the sources' id array.
struct Census {
    uint32_t *count;
    unsigned long long *sum;
    const uint32_t *sid;
};

// SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", 2014): a bijection of 64-bit words whose
// sums over two different id sets differ with overwhelming probability.
__device__ inline unsigned long long mix64(uint32_t id)
{
    unsigned long long z = (unsigned long long)id + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
#ifndef SPH_PAIR_MX
#define SPH_PAIR_MX 1   // the FP64 fluid FORCE pass over every target filters on the matrix cores (k_pairs_mx)
#endif
// Wavefronts per SIMD of the solid FORCE pass: at 4 (FP32) and 3 (FP64) its
// registers spilled (4 and 33); measured on the cylinder and the impact
// (steps, ms): FP32 4.69 -> 4.53 and 8.30 -> 8.07 at 3, FP64 7.90 -> 7.46
// and 14.27 -> 13.63 at 2.
// The FP64 solid FORCE reverse needs about 380 registers: at two wavefronts
// per SIMD it spilled 244 to scratch, at one it keeps them (256 plus 120
// accumulation registers); backward pass of a 64,000-particle block 12.6 ->
// 8.6 ms.
#ifndef SPH_PAIR_EU_SOLID_ADJ_F64
#define SPH_PAIR_EU_SOLID_ADJ_F64 1
#endif
#ifndef SPH_PAIR_EU_SOLID_F32
#define SPH_PAIR_EU_SOLID_F32 3
#endif
#ifndef SPH_PAIR_EU_SOLID_F64
#define SPH_PAIR_EU_SOLID_F64 2
#endif
#ifndef SPH_PAIR_WAVES_PER_EU
#define SPH_PAIR_WAVES_PER_EU 4
#endif
// Occupancy target (waves per SIMD; caps VGPRs at 512 / target) per
// variant: the LDS of a workgroup allows four per SIMD, which the fluid
// passes and the FP32 solid pass reach; the FP64 solid body fits 3, the
// fluid adjoint body (11 cotangents) 3 (FP32) and 2 (FP64), the solid
// adjoint body (17) 2, the GRADIENT reverse 3 and 2.
template <typename real, bool SOLID, int PASS>
struct PairOccupancy {
    static constexpr bool ADJ = PASS == kPassAdjoint || PASS == kPassGradAdjoint;
    static constexpr int fp32 = ADJ ? ((SOLID && PASS == kPassAdjoint) ? 2 : 3)
                                    : (SOLID && PASS == SPH_PASS_FORCE ? SPH_PAIR_EU_SOLID_F32
                                                                       : (SOLID ? 4 : SPH_PAIR_WAVES_PER_EU));
    // measured: the FP64 fluid passes run faster at 3 than at 4 (no spills)
    static constexpr int fp64 = ADJ ? ((SOLID && PASS == kPassAdjoint) ? SPH_PAIR_EU_SOLID_ADJ_F64 : 2)
                                    : (SOLID && PASS == SPH_PASS_FORCE ? SPH_PAIR_EU_SOLID_F64 : 3);
    static constexpr int value = sizeof(real) == 4 ? fp32 : fp64;
};

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

// Orders this wavefront's LDS writes before its following LDS reads.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave-uniform double held in scalar registers (it is an operand of
// vector instructions, so it takes no vector registers of its own).
__device__ inline double uniform_double(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ inline int wave_min(int v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return __builtin_amdgcn_readfirstlane(v);   // equal in every lane
}

// Largest value over the wavefront of a v in [0, 256), by eight ballots
// (no cross-lane data movement: the page loop's bound costs no LDS round
// trips; 1.5 % off the FP32 column FORCE pass with the page prefetch below).
__device__ inline int wave_max_u8(int v)
{
    int r = 0;
#pragma unroll
    for (int b = 7; b >= 0; --b) {
        const int c = r | (1 << b);
        if (__ballot(v >= c)) r = c;
    }
    return r;
}

__device__ inline int wave_max(int v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return __builtin_amdgcn_readfirstlane(v);   // equal in every lane
}

// Row-aligned wavefronts: the targets of one bucket row (cy, cz) are one
// contiguous range of the sorted array, and a wavefront whose targets span
// two rows walks the neighbour rows of each in turn with the other lanes
// idle.  For a pass over every target of a sorted array, one workgroup
// lists (first target, count) for wavefronts that each take up to 64
// targets of a single row, rows in order (on the column workload: 13,183 row
// walks instead of 14,243).  plan holds at most ceil(n / 64) + rows entries;
// *nplan receives their number.  The staging kernel runs this as its first
// workgroup, so the plan's latency hides behind the staging.
constexpr int kPlanBlock = kBlock;
constexpr int kPlanRows = 8;   // consecutive rows per thread in one chunk of the plan
__device__ inline void wave_plan_block(const Grid &g, const uint32_t *__restrict__ start, uint2 *__restrict__ plan,
                                       uint32_t *__restrict__ nplan)
{
    __shared__ uint32_t wsum[kPlanBlock / kWave];
    const uint32_t nx = (uint32_t)g.nx, nrows = (uint32_t)g.ny * (uint32_t)g.nz;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t carry = 0;
    for (uint32_t r0 = 0; r0 < nrows; r0 += kPlanBlock * kPlanRows) {
        // the thread's rows rb .. rb + kPlanRows - 1: their kPlanRows + 1
        // boundaries are all loaded before the first is used (one memory
        // round trip per chunk; rows past the last start and end at n)
        const uint32_t rb = r0 + (uint32_t)threadIdx.x * kPlanRows;
        uint32_t bnd[kPlanRows + 1];
#pragma unroll
        for (int k = 0; k <= kPlanRows; ++k) {
            const uint32_t r = rb + (uint32_t)k < nrows ? rb + (uint32_t)k : nrows;
            bnd[k] = start[(size_t)r * nx];
        }
        uint32_t w = 0;
#pragma unroll
        for (int k = 0; k < kPlanRows; ++k) w += (bnd[k + 1] - bnd[k] + kWave - 1) / kWave;
        // exclusive scan of w over the block (wavefront scan, then wavefront totals)
        uint32_t inc = w;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t v = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += v;
        }
        if (lane == kWave - 1) wsum[wave] = inc;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int k = 0; k < kPlanBlock / kWave; ++k) {
            const uint32_t s = wsum[k];
            before += k < wave ? s : 0u;
            tot += s;
        }
        __syncthreads();
        uint32_t q = carry + before + inc - w;
#pragma unroll
        for (int k = 0; k < kPlanRows; ++k) {
            const uint32_t b = bnd[k], len = bnd[k + 1] - bnd[k];
            for (uint32_t m = 0; m * (uint32_t)kWave < len; ++m) {
                const uint32_t left = len - m * (uint32_t)kWave;
                plan[q++] = make_uint2(b + m * (uint32_t)kWave, left < (uint32_t)kWave ? left : (uint32_t)kWave);
            }
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *nplan = carry;
}

// Packs the pair inputs of every source particle (see Stage).
template <typename real, bool SOLID>
__global__ __launch_bounds__(kBlock) void k_stage(Grid g, PV<real> s, Stage<real> st, const uint32_t *pstart,
                                                  uint2 *plan, uint32_t *nplan)
{
    constexpr bool SPLIT = sizeof(real) == 4;
    if (plan && blockIdx.x == 0) {
        wave_plan_block(g, pstart, plan, nplan);
        return;
    }
    uint32_t j = (blockIdx.x - (plan ? 1u : 0u)) * kBlock + threadIdx.x;
    if (j >= s.n) return;
    using v4 = typename Vec4<real>::type;
    // every field is read before the first record is written: the records
    // could alias the fields as far as the compiler knows, and a read issued
    // after a write would wait out the write's round trip
    v4 pos, a, b, c0, c1;
    const uint32_t hj = s.hash[j];
    if constexpr (SPLIT) {
        pos.x = s.off[0][j];
        pos.y = s.off[1][j];
        pos.z = s.off[2][j];
    } else {
        pos.x = s.x[0][j];
        pos.y = s.x[1][j];
        pos.z = s.x[2][j];
    }
    a.x = s.v[0][j];
    a.y = s.v[1][j];
    a.z = s.v[2][j];
    a.w = s.w[j];
    b.x = s.rho[j];
    b.y = s.p[j];
    b.z = s.c[j];
    b.w = s.e[j];
    if constexpr (SOLID) {
        c0.x = s.S[0][j];
        c0.y = s.S[1][j];
        c0.z = s.S[2][j];
        c0.w = s.S[3][j];
        c1.x = s.S[4][j];
        c1.y = s.S[5][j];
        c1.z = 0;
        c1.w = 0;
    }
    pos.w = (real)(hj % (uint32_t)g.nx);
    st.pos[j] = pos;
    st.va[rec_stride<real> * j] = a;
    st.vb[rec_stride<real> * j] = b;
    if constexpr (SOLID) {
        st.s0[rec_stride<real> * j] = c0;
        st.s1[rec_stride<real> * j] = c1;
    }
}

// Target position: bucket offsets and bucket x index (split), or x (FP64).
template <typename real>
struct TargetPos {
    real o[3];
    double x[3];
    real cxf;
    real Lf;
};

// d = x_j - x_i for a staged source record p in neighbour row (ddy, ddz).
template <typename real>
__device__ inline void diff(const TargetPos<real> &T, const typename Vec4<real>::type &p, real ddy, real ddz,
                            real d[3])
{
    if constexpr (sizeof(real) == 4) {
        d[0] = (p.w - T.cxf) * T.Lf + (p.x - T.o[0]);
        d[1] = ddy + (p.y - T.o[1]);
        d[2] = ddz + (p.z - T.o[2]);
    } else {
        d[0] = p.x - T.x[0];
        d[1] = p.y - T.x[1];
        d[2] = p.z - T.x[2];
    }
}

// Pair-sum accumulator: FP64 in both forms.
struct Acc {
    double s;
    __device__ inline void add(float x) { s += (double)x; }
    __device__ inline void add(double x) { s += x; }
};

template <typename real, int PASS, bool SOLID, bool SELF>
__global__ __launch_bounds__(kPairBlock)
__attribute__((amdgpu_waves_per_eu(PairOccupancy<real, SOLID, PASS>::value)))
void k_pairs(Params P, Grid g, PV<real> tg, const uint32_t *__restrict__ tidx, const uint32_t *__restrict__ ntdev,
             Stage<real> src, const uint32_t *__restrict__ sstart, int zero_first, RV<real> R, AV<real> B,
             const uint2 *__restrict__ plan, const uint32_t *__restrict__ nplan, Census cz)
{
    using v4 = typename Vec4<real>::type;
    constexpr bool SPLIT = sizeof(real) == 4;
    constexpr bool ADJ = PASS == kPassAdjoint;
    constexpr bool GADJ = PASS == kPassGradAdjoint;
    constexpr bool CENSUS = PASS == kPassCensus;
    constexpr int NOUT = PASS == SPH_PASS_FORCE ? 6 : (ADJ ? (SOLID ? 17 : 11) : (GADJ ? 7 : (CENSUS ? 1 : 9)));
    constexpr int kPage = Tune<real>::page;
    constexpr int kHitCap = Tune<real>::cap;
    // List entries and marks are laid out so that the 64 lanes of a wavefront
    // always touch 64 different dwords (the wavefronts of the workgroup share
    // each dword), whatever each lane's fill: no LDS bank conflicts.
    __shared__ uint8_t hits[kHitCap][kWaves / kHitWaves][kWave][kHitWaves];   // index inside the page
    // per lane, one mark per page in which it has hits: (slot << 8) | list fill
    // at the end of that page's hits
    __shared__ uint16_t marks[kMaxWin][kWaves / 2][kWave][2];
    __shared__ float4 stage[kWaves][kPage + kSub];   // a page, then far sentinels
    // per staged page: its first source index and (c_j - c_i) L in y and z of
    // its row (split form; the FP64 form works on absolute positions), side by
    // side so that one address serves the three reads
    struct alignas(16) Win {
        uint32_t base;
        float dy, dz, pad;
    };
    __shared__ Win win[kWaves][kMaxWin];

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);   // neighbouring tiles share sources
    bool valid;
    uint32_t i;
    if (plan) {
        // row-aligned wavefronts (k_wave_plan), the plan's tiles shared evenly
        // by the XCDs (the grid is sized for the plan's bound); whole
        // wavefronts beyond the plan leave
        const uint32_t np = *nplan;
        if (!xcd_tile_active(blockIdx.x, (np + kWaves - 1) / kWaves, tile)) return;
        const uint32_t wid = tile * kWaves + wave;
        if (wid >= np) return;
        const uint2 d = plan[wid];
        valid = (uint32_t)lane < d.y;
        i = valid ? d.x + (uint32_t)lane : 0u;
    } else {
        uint32_t nt = tg.n;
        if (tidx) {
            // a target list's count is on the device and the grid is sized for
            // the whole array: the list's tiles shared evenly by the XCDs
            uint32_t c = *ntdev;
            nt = c < nt ? c : nt;
            if (!xcd_tile_active(blockIdx.x, (nt + kPairBlock - 1) / kPairBlock, tile)) return;
        }
        const uint32_t t = tile * kPairBlock + tid;
        // whole wavefronts beyond the targets leave; partial ones keep idle lanes
        if (tile * kPairBlock + wave * kWave >= nt) return;
        valid = t < nt;
        i = valid ? (tidx ? tidx[t] : t) : 0u;
        // a listed index outside the target array names no target
        valid = valid && i < tg.n;
        i = valid ? i : 0u;
    }

    const PairK<real> K = make_pair_k<real>(P);
    const real R2 = (real)P.R2;

    const uint32_t h = valid ? tg.hash[i] : 0u;
    const int cx = (int)(h % (uint32_t)g.nx);
    const uint32_t rowkey = valid ? h / (uint32_t)g.nx : 0xFFFFFFFFu;   // cy + ny cz
    const int x0 = cx > 0 ? cx - 1 : 0;
    const int x1 = cx + 1 < g.nx ? cx + 1 : g.nx - 1;

    TargetPos<real> T;
    T.cxf = (real)cx;
    T.Lf = SPLIT ? (real)g.Lf : real(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if constexpr (SPLIT) {
            T.o[d] = valid ? tg.off[d][i] : real(0);
            T.x[d] = 0.0;
        } else {
            T.x[d] = valid ? tg.x[d][i] : 0.0;
            T.o[d] = real(0);
        }
    }
    Part<real, SOLID> I;
    real rbi[GADJ ? 9 : 6];   // adjoint: the target's rate (or velocity-gradient) cotangents
    if constexpr (PASS == SPH_PASS_FORCE || ADJ) {
        load_part<real, SOLID>(tg, i, I);
    } else if constexpr (!CENSUS) {
#pragma unroll
        for (int d = 0; d < 3; ++d) I.v[d] = tg.v[d][i];
        if constexpr (GADJ) I.w = tg.w[i];
    }
    if constexpr (ADJ) {
#pragma unroll
        for (int k = 0; k < 6; ++k) rbi[k] = R.hi[0] ? R.hi[k][i] : real(0);
    }
    if constexpr (GADJ) {
#pragma unroll
        for (int k = 0; k < 9; ++k) rbi[k] = R.Lhi[0] ? R.Lhi[k][i] : real(0);
    }

    Acc acc[NOUT];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        double s0 = 0.0;
        if constexpr (!ADJ && !GADJ && !CENSUS) {
            real *hi = PASS == SPH_PASS_FORCE ? R.hi[k] : R.Lhi[k];
            real *lo = PASS == SPH_PASS_FORCE ? R.lo[k] : R.Llo[k];
            if (!zero_first && valid) {
                s0 = (double)hi[i];
                if (SPLIT) s0 += (double)lo[i];
            }
        }
        acc[k].s = s0;
    }

    uint32_t ncen = 0;             // census: pairs evaluated
    unsigned long long scen = 0;   // census: sum of mix64 of their ids
    int cnt = 0;   // entries in the lane's list
    // Records of one listed hit; the next hit's are loaded while the current
    // pair is evaluated (software pipelining hides the L2 latency).
    struct Rec {
        v4 p, a, b, s0, s1, r0, r1;
        real qy, qz;
        uint32_t j;
    };
    // entry s of the lane's list; (mk, nb) walk the lane's marks as s ascends
    // (each mark covers at least one entry, so one step suffices)
    auto fetch = [&](int s, int &mk, int &nb) {
        Rec q;
        mk += s >= nb ? 1 : 0;
        const uint32_t m = marks[mk][wave >> 1][lane][wave & 1];
        nb = (int)(m & 0xFFu);
        const uint32_t slot = m >> 8;
        const Win &wn = win[wave][slot];
        const uint32_t jj = wn.base + (uint32_t)hits[s][wave / kHitWaves][lane][wave % kHitWaves];
        q.qy = SPLIT ? (real)wn.dy : real(0);
        q.qz = SPLIT ? (real)wn.dz : real(0);
        // a 32-bit byte offset from each array's base (sources are fewer than
        // 2^27, and a source's records span at most 32 bytes per array), so
        // the loads take the scalar-base form
        const uint32_t ob = jj * (uint32_t)sizeof(v4);
        auto at = [&](const v4 *base, uint32_t o) { return *reinterpret_cast<const v4 *>(reinterpret_cast<const char *>(base) + o); };
        q.p = at(src.pos, ob);
        q.j = jj;
        if constexpr (CENSUS) return q;
        const uint32_t ob2 = ob * rec_stride<real>;
        q.a = at(src.va, ob2);
        if constexpr (PASS == SPH_PASS_FORCE || ADJ || GADJ) q.b = at(src.vb, ob2);
        if constexpr ((PASS == SPH_PASS_FORCE || ADJ) && SOLID) {
            q.s0 = at(src.s0, ob2);
            q.s1 = at(src.s1, ob2);
        }
        if constexpr (ADJ || GADJ) {
            q.r0 = at(src.r0, ob2);
            q.r1 = at(src.r1, ob2);
        }
        return q;
    };
    // the pair terms of one listed hit, added to the lane's sums
    auto eval = [&](const Rec &cur) {
            real d[3];
            diff<real>(T, cur.p, cur.qy, cur.qz, d);
            const real r2 = r2_of<real>(d);
            // the neighbour predicate, on the exact and odd d (so a pair is in or
            // out for both of its particles); the filter's shortlist is wider
            if (!(r2 < R2)) {
                // outside the support: nothing to add
            } else if constexpr (CENSUS) {
                ++ncen;
                scen += mix64(cz.sid[cur.j]);
            } else if constexpr (PASS == SPH_PASS_FORCE) {
                const v4 b = cur.b;
                Part<real, SOLID> J;
                J.v[0] = cur.a.x;
                J.v[1] = cur.a.y;
                J.v[2] = cur.a.z;
                J.w = cur.a.w;
                J.rho = b.x;
                J.p = b.y;
                J.c = b.z;
                J.e = b.w;
                if constexpr (SOLID) {
                    J.S[0] = cur.s0.x;
                    J.S[1] = cur.s0.y;
                    J.S[2] = cur.s0.z;
                    J.S[3] = cur.s0.w;
                    J.S[4] = cur.s1.x;
                    J.S[5] = cur.s1.y;
                }
                real o[6];
                pair_force<real, SOLID>(d, r2, I, J, K, o);
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[k].add(o[k]);
            } else if constexpr (ADJ) {
                Part<real, SOLID> J;
                J.v[0] = cur.a.x;
                J.v[1] = cur.a.y;
                J.v[2] = cur.a.z;
                J.w = cur.a.w;
                J.rho = cur.b.x;
                J.p = cur.b.y;
                J.c = cur.b.z;
                J.e = cur.b.w;
                if constexpr (SOLID) {
                    J.S[0] = cur.s0.x;
                    J.S[1] = cur.s0.y;
                    J.S[2] = cur.s0.z;
                    J.S[3] = cur.s0.w;
                    J.S[4] = cur.s1.x;
                    J.S[5] = cur.s1.y;
                }
                // T(s_j, s_i) = sigma T(s_i, s_j): mass, momentum and energy terms
                // are odd (sigma = -1), the volume term even (+1)
                const real rbj[6] = {cur.r0.x, cur.r0.y, cur.r0.z, cur.r0.w, cur.r1.x, cur.r1.y};
                real wb[6];
#pragma unroll
                for (int k = 0; k < 5; ++k) wb[k] = rbi[k] - rbj[k];
                wb[5] = rbi[5] + rbj[5];
                real o[NOUT];
#pragma unroll
                for (int k = 0; k < NOUT; ++k) o[k] = real(0);
                pair_force_vjp<real, SOLID>(d, r2, I, J, K, wb, o);
#pragma unroll
                for (int k = 0; k < NOUT; ++k) acc[k].add(o[k]);
            } else if constexpr (GADJ) {
                const real vj[3] = {cur.a.x, cur.a.y, cur.a.z};
                const real Lj[9] = {cur.b.x, cur.b.y, cur.b.z, cur.b.w, cur.r0.x, cur.r0.y, cur.r0.z, cur.r0.w,
                                    cur.r1.x};
                real o[7] = {0, 0, 0, 0, 0, 0, 0};
                pair_grad_vjp<real>(d, r2, I.v, vj, I.w, cur.a.w, rbi, Lj, K, o);
#pragma unroll
                for (int k = 0; k < 7; ++k) acc[k].add(o[k]);
            } else {
                const real vj[3] = {cur.a.x, cur.a.y, cur.a.z};
                real o[9];
                pair_grad<real>(d, r2, I.v, vj, cur.a.w, K, o);
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[k].add(o[k]);
            }
    };
    // Evaluate the pair terms of every listed hit, two at a time: the records
    // of the next two are loaded while the current two are evaluated, into
    // alternating buffers (no register copies); indices past the list end are
    // clamped to its last entry, so every load reads a listed record.  Every
    // page with hits must be marked first (close_page); the last mark ends at
    // cnt, so the walk over the marks stays inside them.
    int cnt0 = 0;   // list fill when the current page started
    int npg = 0;    // marks written since the lists were last emptied
    auto close_page = [&](int slot) {
        if (cnt != cnt0) marks[npg++][wave >> 1][lane][wave & 1] = (uint16_t)(((uint32_t)slot << 8) | (uint32_t)cnt);
        cnt0 = cnt;
    };
    auto flush = [&]() {
        if (cnt > 0) {
            const int last = cnt - 1;
            int mk = 0, nb = (int)(marks[0][wave >> 1][lane][wave & 1] & 0xFFu);
            Rec A = fetch(0, mk, nb);
            Rec B = fetch(last < 1 ? last : 1, mk, nb);
            for (int s = 0; s < cnt; s += 2) {
                eval(A);
                A = fetch(s + 2 < last ? s + 2 : last, mk, nb);
                if (s + 1 < cnt) eval(B);
                B = fetch(s + 3 < last ? s + 3 : last, mk, nb);
            }
        }
        cnt = 0;
        cnt0 = 0;
        npg = 0;
    };

    const float kFar = 1e30f;

    uint64_t pending = __ballot(valid);
    while (pending) {
        // the next group: lanes whose target shares the first pending lane's bucket row
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const uint32_t key = __builtin_amdgcn_readfirstlane(__shfl(rowkey, leader, kWave));
        const bool in = valid && rowkey == key;
        pending &= ~__ballot(in);
        const int gx0 = wave_min(in ? x0 : 0x7FFFFFFF);
        const int gx1 = wave_max(in ? x1 : -1);
        // Filter frame, in FP32 in both forms: positions relative to the
        // corner of bucket (gx0, gy, gz); split form ((c - gx0) L + off) in x
        // and (dy L + off) in y, z; FP64 form (x - corner) in FP64, rounded
        // once to float.  The test is the expanded form
        // |q|^2 - 2 q.f < R2 - |f|^2, with (2q, |q|^2) staged for each record,
        // so a candidate costs three FMAs and a compare.  For a candidate
        // within 2h of the target (|q| <= |f| + 2h) its rounding, with that of
        // the frame, stays below 2^-18 (|f| + 2h)^2; the bound is widened by
        // four times that, and in FP64 also by 2^-46 X (|f| + 2h) with
        // X = |corner|_1 + |f| + 2h, over ten times the rounding of the FP64
        // differences.  So the shortlist keeps every neighbour, and the FP64
        // form's sums are those an FP64 filter would give.  The pair body
        // applies the neighbour predicate itself, on the exact, odd d.
        float fo[3];
        const int gy = (int)(key % (uint32_t)g.ny), gz = (int)(key / (uint32_t)g.ny);
        const float gx0f = (float)gx0;
        double corner[3] = {0.0, 0.0, 0.0};
        if constexpr (SPLIT) {
            fo[0] = (T.cxf - gx0f) * T.Lf + T.o[0];
            fo[1] = T.o[1];
            fo[2] = T.o[2];
        } else {
            corner[0] = uniform_double(g.o[0] + (double)gx0 * g.L);
            corner[1] = uniform_double(g.o[1] + (double)gy * g.L);
            corner[2] = uniform_double(g.o[2] + (double)gz * g.L);
#pragma unroll
            for (int d = 0; d < 3; ++d) fo[d] = (float)(T.x[d] - corner[d]);
        }
        const float f2 = fo[0] * fo[0] + fo[1] * fo[1] + fo[2] * fo[2];
        const float fl = sqrtf(f2) + (float)(2.0 * P.h);
        float margin = 0x1p-16f * fl * fl;
        if constexpr (!SPLIT) {
            const float X = (float)(fabs(corner[0]) + fabs(corner[1]) + fabs(corner[2])) + fl;
            margin += 0x1p-46f * X * fl;
        }
        const float Tl = in ? ((float)R2 - f2) + margin : -kFar;
        int nwin = 0;
        for (int r = 0; r < 9; ++r) {
            const int dz = r / 3 - 1, dy = r % 3 - 1;
            const int z = gz + dz, y = gy + dy;
            if (z < 0 || z >= g.nz || y < 0 || y >= g.ny) continue;
            const uint32_t row = (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
            const uint32_t ub = sstart[row + gx0], ue = sstart[row + gx1 + 1];
            if (ub >= ue) continue;
            // the lane's own 3-bucket range of this row (a sub-range of [ub, ue))
            const uint32_t lo = in ? sstart[row + x0] : ub;
            const uint32_t hi = in ? sstart[row + x1 + 1] : ub;
            const real ddy = (real)dy * T.Lf, ddz = (real)dz * T.Lf;
            for (uint32_t pb = ub; pb < ue; pb += (uint32_t)kPage) {
                const uint32_t len = ue - pb < (uint32_t)kPage ? ue - pb : (uint32_t)kPage;
                if (nwin == kMaxWin) {
                    flush();
                    nwin = 0;
                }
                int slot = nwin++;
                if (lane == 0) {
                    win[wave][slot] = Win{pb, (float)ddy, (float)ddz, 0.0f};
                }
                wave_lds_sync();   // earlier reads of the stage are done
                // the page in the group's filter frame, then far sentinels up to
                // kPage + kSub so that every read below stays in the array and
                // nothing past the page can pass a test
                {
                    // every lane's records of the page in flight at once, then
                    // staged (one memory round trip per page instead of three)
                    constexpr int kIt = (kPage + kSub + kWave - 1) / kWave;
                    v4 sp[kIt];
#pragma unroll
                    for (int it = 0; it < kIt; ++it) {
                        const uint32_t u = (uint32_t)lane + (uint32_t)(it * kWave);
                        if (u < len) sp[it] = src.pos[pb + u];
                    }
#pragma unroll
                    for (int it = 0; it < kIt; ++it) {
                        const uint32_t u = (uint32_t)lane + (uint32_t)(it * kWave);
                        if (u >= (uint32_t)(kPage + kSub)) continue;
                        float4 rec;
                        if (u < len) {
                            if constexpr (SPLIT) {
                                rec.x = (sp[it].w - gx0f) * T.Lf + sp[it].x;
                                rec.y = ddy + sp[it].y;
                                rec.z = ddz + sp[it].z;
                            } else {
                                rec.x = (float)(sp[it].x - corner[0]);
                                rec.y = (float)(sp[it].y - corner[1]);
                                rec.z = (float)(sp[it].z - corner[2]);
                            }
                            rec.w = rec.x * rec.x + rec.y * rec.y + rec.z * rec.z;
                            rec.x *= 2.0f;
                            rec.y *= 2.0f;
                            rec.z *= 2.0f;
                        } else {
                            rec.x = rec.y = rec.z = 0.0f;
                            rec.w = kFar;
                        }
                        stage[wave][u] = rec;
                    }
                }
                wave_lds_sync();
                // Each lane walks its own range clipped to the page.  Lanes whose
                // range is shorter than the longest keep reading past its end:
                // those records lie in farther buckets of the same row (or are
                // sentinels) and are more than one bucket side away, so no lane
                // needs a bound check per candidate.
                const uint32_t pe = pb + len;
                const uint32_t la = lo > pb ? lo - pb : 0u;
                const uint32_t hc = hi < pe ? hi : pe;
                const uint32_t le = hc > pb ? hc - pb : 0u;
                const int nl = le > la ? (int)(le - la) : 0;
                const int nmax = wave_max_u8(nl);   // nl <= kPage < 256
                // every lane reads `span` records from a; moving a lane's start
                // back (to records before its own range: nearer buckets of the
                // row, also more than one bucket side away) keeps the reads
                // inside the array
                const int span = (nmax + kSub - 1) / kSub * kSub;
                const int a = (int)la < kPage + kSub - span ? (int)la : kPage + kSub - span;
                for (int k0 = 0; k0 < nmax; k0 += kSub) {
                    // at most kSub more entries per lane before the next check
                    if (__ballot(cnt > kHitCap - kSub)) {
                        // empty the lists mid-page; the page keeps going as slot 0
                        close_page(slot);
                        flush();
                        if (lane == 0) {
                            win[wave][0] = Win{pb, (float)ddy, (float)ddz, 0.0f};
                        }
                        slot = 0;
                        nwin = 1;
                    }
                    const int base = a + k0;
#pragma unroll
                    for (int m = 0; m < kSub; ++m) {
                        const float4 q = stage[wave][base + m];
                        const float t = fmaf(-q.z, fo[2], fmaf(-q.y, fo[1], fmaf(-q.x, fo[0], q.w)));
                        // the entry is written always and kept only when it is a hit
                        hits[cnt][wave / kHitWaves][lane][wave % kHitWaves] = (uint8_t)(base + m);
                        cnt += (t < Tl) ? 1 : 0;
                    }
                }
                close_page(slot);
            }
        }
        flush();
    }
    if (!valid) return;
    if constexpr (CENSUS) {
        cz.count[i] = ncen;
        cz.sum[i] = scen;
    } else if constexpr (ADJ) {
        // accumulate the cotangents of x, v, omega, rho, p, c, e (and S)
        real *out[17] = {B.x[0], B.x[1], B.x[2], B.v[0], B.v[1], B.v[2], B.w, B.rho, B.p, B.c, B.e,
                         B.S[0], B.S[1], B.S[2], B.S[3], B.S[4], B.S[5]};
#pragma unroll
        for (int k = 0; k < NOUT; ++k) out[k][i] = (real)((double)out[k][i] + acc[k].s);
    } else if constexpr (GADJ) {
        // accumulate the cotangents of x, v, omega
        real *out[7] = {B.x[0], B.x[1], B.x[2], B.v[0], B.v[1], B.v[2], B.w};
#pragma unroll
        for (int k = 0; k < 7; ++k) out[k][i] = (real)((double)out[k][i] + acc[k].s);
    } else {
#pragma unroll
        for (int k = 0; k < NOUT; ++k) {
            real *hi = PASS == SPH_PASS_FORCE ? R.hi[k] : R.Lhi[k];
            real *lo = PASS == SPH_PASS_FORCE ? R.lo[k] : R.Llo[k];
            const real hv = (real)acc[k].s;
            hi[i] = hv;
            if (SPLIT) lo[i] = (real)(acc[k].s - (double)hv);
        }
    }
}

// The FORCE pass of a fluid over every target of a sorted array, with the
// neighbour filter on the matrix cores.  A wavefront takes up to 32 targets
// of one bucket row (one half of an entry of the row-aligned plan), two lanes
// per target: lane t and lane t + 32.  For each of the 9 neighbour rows the
// sources of the union of its targets' buckets are tested 32 at a time: the
// shortlist value |q|^2 - 2 q.f of every (source, target) pair of a block is
// one 32 x 32 x 4 matrix product, two v_mfma_f32_32x32x2f32 (A: the sources'
// (-2q, |q|^2), B: the targets' (f, 1)), in the FP32 frame of the VALU
// filter and against the same widened bound (the product's rounding, within
// two units of 2^-24 of the sum of the terms' magnitudes when measured, is
// far inside that margin).  Lane (t, h) receives the values of the block's
// sources 8m + 4h + r (m, r < 4) for target t and keeps one bit for each;
// the hits are evaluated from these bit masks in one flat loop per lane (so
// a lane's hits in different rows do not wait for each other), and the two
// lanes of a target add their sums at the end.  No per-candidate LDS traffic
// and about three vector instructions per 64 candidate tests, where the VALU
// filter spends eight and a page read; but every target is tested against
// the union of the wavefront's buckets (about 1.8 times its own 27), and two
// lanes per target balance their hits less evenly than one, so it pays in
// the FP64 form only (whose pair evaluation and staging cost more per hit).
// Measured on the FP64 column (FORCE launch, median of 60): 4 wavefronts
// per workgroup 0.570 ms, 2 0.569, 8 0.665; 3 wavefronts per SIMD as set,
// 4 spills ten registers and takes 0.646.
#ifndef SPH_PAIR_MX_WAVES
#define SPH_PAIR_MX_WAVES 4
#endif
#ifndef SPH_PAIR_MX_EU_F64
#define SPH_PAIR_MX_EU_F64 3
#endif
constexpr int kMxWaves = SPH_PAIR_MX_WAVES;   // wavefronts per workgroup
constexpr int kMxTargets = 32;   // targets per wavefront
constexpr int kMxWords = 24;     // bit-mask words a lane holds before its hits are evaluated
typedef float mx16 __attribute__((ext_vector_type(16)));

template <typename real, bool CENSUS>
__global__ __launch_bounds__(kMxWaves * kWave)
__attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? SPH_PAIR_WAVES_PER_EU : SPH_PAIR_MX_EU_F64)))
void k_pairs_mx(Params P, Grid g, PV<real> tg, Stage<real> src, const uint32_t *__restrict__ sstart,
                int zero_first, RV<real> R, const uint2 *__restrict__ plan, const uint32_t *__restrict__ nplan,
                Census cz)
{
    using v4 = typename Vec4<real>::type;
    constexpr bool SPLIT = sizeof(real) == 4;
    constexpr int NOUT = CENSUS ? 1 : 6;
    // one word of a lane's bit masks covers two blocks of one row: the first
    // block's first source and the row's (c_j - c_i) L in y and z
    struct alignas(16) Slot {
        uint32_t base;
        float dy, dz, pad;
    };
    __shared__ uint32_t bits[kMxWaves][kMxWords][kWave];
    __shared__ Slot slots[kMxWaves][kMxWords];

    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int tl = lane & (kMxTargets - 1), half = lane / kMxTargets;
    // wavefront w takes half w % 2 of the plan's entry w / 2 (up to 64
    // targets of one row); wavefronts beyond the plan, or on the empty second
    // half of a short entry, leave whole
    // (the plan's tiles shared evenly by the XCDs: the grid is sized for the
    // plan's bound)
    const uint32_t np = *nplan;
    uint32_t tile;
    if (!xcd_tile_active(blockIdx.x, (2u * np + kMxWaves - 1) / kMxWaves, tile)) return;
    const uint32_t wid = tile * kMxWaves + wave;
    if (wid / 2u >= np) return;
    const uint2 pe = plan[wid / 2u];
    const uint32_t off = (wid & 1u) * (uint32_t)kMxTargets;
    if (pe.y <= off) return;
    const uint2 pd = make_uint2(pe.x + off, pe.y - off < (uint32_t)kMxTargets ? pe.y - off : (uint32_t)kMxTargets);
    const bool valid = (uint32_t)tl < pd.y;
    const uint32_t i = pd.x + (valid ? (uint32_t)tl : 0u);   // idle lanes shadow the first target

    const PairK<real> K = make_pair_k<real>(P);
    const real R2 = (real)P.R2;
    const uint32_t h = tg.hash[i];
    const int cx = (int)(h % (uint32_t)g.nx);
    // one row for the whole wavefront, its targets in ascending x bucket
    const uint32_t key = __builtin_amdgcn_readfirstlane(h / (uint32_t)g.nx);
    const int gx0 = __builtin_amdgcn_readfirstlane(cx);
    const int gx1 = wave_max(valid ? cx : gx0);
    const int gy = (int)(key % (uint32_t)g.ny), gz = (int)(key / (uint32_t)g.ny);

    TargetPos<real> T;
    T.cxf = (real)cx;
    T.Lf = SPLIT ? (real)g.Lf : real(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if constexpr (SPLIT) {
            T.o[d] = tg.off[d][i];
            T.x[d] = 0.0;
        } else {
            T.x[d] = tg.x[d][i];
            T.o[d] = real(0);
        }
    }
    Part<real, false> I;
    if constexpr (!CENSUS) load_part<real, false>(tg, i, I);
    Acc acc[NOUT];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        double s0 = 0.0;
        if constexpr (!CENSUS) {
            if (!zero_first && valid && half == 0) {
                s0 = (double)R.hi[k][i];
                if (SPLIT) s0 += (double)R.lo[k][i];
            }
        }
        acc[k].s = s0;
    }
    uint32_t ncen = 0;             // census: pairs evaluated
    unsigned long long scen = 0;   // census: sum of mix64 of their ids

    // the filter frame, margin and bound of the VALU filter (k_pairs)
    const float kFar = 1e30f;
    float fo[3];
    const float gx0f = (float)gx0;
    double corner[3] = {0.0, 0.0, 0.0};
    if constexpr (SPLIT) {
        fo[0] = (T.cxf - gx0f) * T.Lf + T.o[0];
        fo[1] = T.o[1];
        fo[2] = T.o[2];
    } else {
        corner[0] = uniform_double(g.o[0] + (double)gx0 * g.L);
        corner[1] = uniform_double(g.o[1] + (double)gy * g.L);
        corner[2] = uniform_double(g.o[2] + (double)gz * g.L);
#pragma unroll
        for (int d = 0; d < 3; ++d) fo[d] = (float)(T.x[d] - corner[d]);
    }
    const float f2 = fo[0] * fo[0] + fo[1] * fo[1] + fo[2] * fo[2];
    const float fl = sqrtf(f2) + (float)(2.0 * P.h);
    float margin = 0x1p-16f * fl * fl;
    if constexpr (!SPLIT) {
        const float X = (float)(fabs(corner[0]) + fabs(corner[1]) + fabs(corner[2])) + fl;
        margin += 0x1p-46f * X * fl;
    }
    const float Tl = valid ? ((float)R2 - f2) + margin : -kFar;
    // B operands: component h, then 2 + h, of the lane's target (f, 1)
    const float b1 = half ? fo[1] : fo[0];
    const float b2 = half ? 1.0f : fo[2];

    // Records of one hit; the next hit's are loaded while the current pair
    // is evaluated.
    struct Rec {
        v4 p, a, b;
        real qy, qz;
        uint32_t j;
    };
    int nslot = 0;   // words recorded (the same in every lane)
    int cnt = 0;     // hits recorded by this lane
    // the lane's walk over its recorded bits: current word and what is left
    int cs = -1, left = 0;
    uint32_t w = 0, jlast = i;
    float dylast = 0.0f, dzlast = 0.0f;
    auto fetch = [&]() {
        if (left > 0) {
            while (w == 0) w = bits[wave][++cs][lane];   // a later word holds the next hit
            const int p = __builtin_ctz(w);
            w &= w - 1u;
            --left;
            const Slot sl = slots[wave][cs];
            const int rr = p & 15;
            jlast = sl.base + 32u * (uint32_t)(p >> 4) + 8u * (uint32_t)(rr >> 2) + 4u * (uint32_t)half +
                    (uint32_t)(rr & 3);
            dylast = sl.dy;
            dzlast = sl.dz;
        }
        // past the lane's last hit the last record is read again (never evaluated)
        Rec q;
        q.j = jlast;
        q.qy = SPLIT ? (real)dylast : real(0);
        q.qz = SPLIT ? (real)dzlast : real(0);
        const uint32_t ob = jlast * (uint32_t)sizeof(v4);
        auto at = [&](const v4 *base, uint32_t o) { return *reinterpret_cast<const v4 *>(reinterpret_cast<const char *>(base) + o); };
        q.p = at(src.pos, ob);
        if constexpr (!CENSUS) {
            const uint32_t ob2 = ob * rec_stride<real>;
            q.a = at(src.va, ob2);
            q.b = at(src.vb, ob2);
        }
        return q;
    };
    auto eval = [&](const Rec &cur) {
        real d[3];
        diff<real>(T, cur.p, cur.qy, cur.qz, d);
        const real r2 = r2_of<real>(d);
        if (!(r2 < R2)) {
            // outside the support: nothing to add
        } else if constexpr (CENSUS) {
            ++ncen;
            scen += mix64(cz.sid[cur.j]);
        } else {
            Part<real, false> J;
            J.v[0] = cur.a.x;
            J.v[1] = cur.a.y;
            J.v[2] = cur.a.z;
            J.w = cur.a.w;
            J.rho = cur.b.x;
            J.p = cur.b.y;
            J.c = cur.b.z;
            J.e = cur.b.w;
            real o[6];
            pair_force<real, false>(d, r2, I, J, K, o);
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[k].add(o[k]);
        }
    };
    // evaluate every recorded hit, two at a time in flight, then start over
    auto flush = [&]() {
        wave_lds_sync();   // the words and slots written are visible to every lane
        const int nmax = wave_max(cnt);
        if (nmax > 0) {
            cs = -1;
            left = cnt;
            w = 0;
            Rec A = fetch();
            Rec B = fetch();
            for (int s = 0; s < nmax; s += 2) {
                if (s < cnt) eval(A);
                A = fetch();
                if (s + 1 < cnt) eval(B);
                B = fetch();
            }
        }
        cnt = 0;
        nslot = 0;
        wave_lds_sync();   // every read of the words is done before they are rewritten
    };

    uint32_t word = 0, wbase = 0;
    bool open = false;   // a word holds one block and waits for the next
    float wdy = 0.0f, wdz = 0.0f;
    auto commit = [&]() {
        bits[wave][nslot][lane] = word;
        if (lane == 0) slots[wave][nslot] = Slot{wbase, wdy, wdz, 0.0f};
        cnt += __popc(word);
        ++nslot;
        open = false;
    };
    const int xa = gx0 > 0 ? gx0 - 1 : 0;
    const int xb = gx1 + 1 < g.nx ? gx1 + 1 : g.nx - 1;
    for (int r = 0; r < 9; ++r) {
        const int dz = r / 3 - 1, dy = r % 3 - 1;
        const int z = gz + dz, y = gy + dy;
        if (z < 0 || z >= g.nz || y < 0 || y >= g.ny) continue;
        const uint32_t row = (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
        const uint32_t ub = sstart[row + xa], ue = sstart[row + xb + 1];
        const float ddy = SPLIT ? (float)((real)dy * T.Lf) : 0.0f;
        const float ddz = SPLIT ? (float)((real)dz * T.Lf) : 0.0f;
        for (uint32_t b0 = ub; b0 < ue; b0 += 32u) {
            // A operands: component h, then 2 + h, of source b0 + t's (-2q, |q|^2);
            // past the row's end a far sentinel that no target takes
            const uint32_t sj = b0 + (uint32_t)tl;
            float a1 = 0.0f, a2 = half ? kFar : 0.0f;
            if (sj < ue) {
                const v4 pp = src.pos[sj];
                float q0, q1, q2;
                if constexpr (SPLIT) {
                    q0 = (pp.w - gx0f) * T.Lf + pp.x;
                    q1 = ddy + pp.y;
                    q2 = ddz + pp.z;
                } else {
                    q0 = (float)(pp.x - corner[0]);
                    q1 = (float)(pp.y - corner[1]);
                    q2 = (float)(pp.z - corner[2]);
                }
                a1 = -2.0f * (half ? q1 : q0);
                a2 = half ? q0 * q0 + q1 * q1 + q2 * q2 : -2.0f * q2;
            }
            mx16 c = {};
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, b2, c, 0, 0, 0);
            uint32_t m16 = 0;
#pragma unroll
            for (int k = 15; k >= 0; --k) m16 = m16 + m16 + (c[k] < Tl ? 1u : 0u);
            if (!open) {
                if (nslot == kMxWords) flush();
                word = m16;
                wbase = b0;
                wdy = ddy;
                wdz = ddz;
                open = true;
            } else {
                word |= m16 << 16;
                commit();
            }
        }
        if (open) commit();
    }
    flush();

    // the two lanes of a target add their sums; lane t writes
    if constexpr (CENSUS) {
        ncen += __shfl_xor(ncen, kMxTargets, kWave);
        scen += __shfl_xor(scen, kMxTargets, kWave);
        if (valid && half == 0) {
            cz.count[i] = ncen;
            cz.sum[i] = scen;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k].s += __shfl_xor(acc[k].s, kMxTargets, kWave);
        if (valid && half == 0) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const real hv = (real)acc[k].s;
                R.hi[k][i] = hv;
                if (SPLIT) R.lo[k][i] = (real)(acc[k].s - (double)hv);
            }
        }
    }
}

// Adjoint pass: the sources' rate cotangents in the two spare records
// (zeros when the sources' rates have no cotangent: rb.hi[0] == NULL).
template <typename real>
__global__ __launch_bounds__(kBlock) void k_stage_rbar(uint32_t n, RV<real> rb, Stage<real> st)
{
    uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    typename Vec4<real>::type a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
    if (rb.hi[0]) {
        a.x = rb.hi[0][j];
        a.y = rb.hi[1][j];
        a.z = rb.hi[2][j];
        a.w = rb.hi[3][j];
        b.x = rb.hi[4][j];
        b.y = rb.hi[5][j];
    }
    st.r0[rec_stride<real> * j] = a;
    st.r1[rec_stride<real> * j] = b;
}

// GRADIENT reverse: the sources' velocity-gradient cotangents in vb (0..3),
// r0 (4..7) and r1.x (8) (zeros when rb.Lhi[0] == NULL).
template <typename real>
__global__ __launch_bounds__(kBlock) void k_stage_lbar(uint32_t n, RV<real> rb, Stage<real> st)
{
    uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    real L[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) L[k] = rb.Lhi[0] ? rb.Lhi[k][j] : real(0);
    typename Vec4<real>::type a = {L[0], L[1], L[2], L[3]}, b = {L[4], L[5], L[6], L[7]}, c = {L[8], 0, 0, 0};
    st.vb[rec_stride<real> * j] = a;
    st.r0[rec_stride<real> * j] = b;
    st.r1[rec_stride<real> * j] = c;
}

// Candidates and hits of one pass, with the predicate of the pair kernel.
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
    const uint32_t i = t < nt ? (tidx ? tidx[t] : t) : tg.n;
    if (i < tg.n) {   // a listed index outside the target array names no target
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
                    const real r2 = r2_of<real>(d);
                    hits += (r2 < R2 && r2 > real(0)) ? 1u : 0u;
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

// One pass.  The census (PASS = kPassCensus) runs the staging, wavefront
// mapping, filter and lists of the FORCE pass of the same material (SOLID),
// or of the GRADIENT pass when census_of_gradient is set.
template <typename real, int PASS, bool SOLID>
hipError_t go(const Params &P, const Grid &g, const sph_particles &tg, const uint32_t *tidx,
              const uint32_t *nt, const sph_particles &sr, const uint32_t *sstart, bool self, int zero_first,
              const sph_rates &r, const sph_adjoint &bar, const Workspace &ws, hipStream_t s,
              const Census cz = Census{}, bool census_of_gradient = false, const sph_rates *rsrc = nullptr)
{
    if (tg.n == 0) return hipSuccess;
    constexpr bool ADJ = PASS == kPassAdjoint || PASS == kPassGradAdjoint;
    Stage<real> st = stage_view<real>(ws, sr.n, SOLID, ADJ);
    uint32_t blocks = div_up(tg.n, kPairBlock);
    uint2 *plan = nullptr;
    uint32_t *nplan = nullptr;
    // A pass over every target of a sorted array (targets = sources, whose
    // bucket table is at hand) takes row-aligned wavefronts; the plan lives in
    // the sort's key buffers, free during a pass, when it fits there.
    // (Measured: the FP32 column's FORCE pass 5 % faster; with the plan's
    // tiles shared evenly by the XCDs, the solid steps too: cylinder 4.87 ->
    // 4.70 ms FP32, 8.68 -> 7.93 FP64; impact 8.46 -> 8.33, 14.73 -> 14.30.)
    // The FP64 form's fluid FORCE pass (and its census) over every target
    // takes the matrix-core filter (k_pairs_mx: two lanes per target, two
    // wavefronts per plan entry).  Measured on the column: FP64 605 us against 651 with the VALU
    // filter; FP32 361 against 353, so the FP32 form keeps the VALU filter.
    constexpr bool MX_PASS = !SOLID && (PASS == SPH_PASS_FORCE || PASS == kPassCensus) && sizeof(real) == 8 &&
                             SPH_PAIR_MX;
    const bool mx = MX_PASS && !census_of_gradient && self && !tidx;
    const uint64_t nrows = (uint64_t)g.ny * (uint64_t)g.nz;
    const uint64_t pmax = div_up(tg.n, kWave) + nrows;
    // (the workspace's key buffers hold 4 bytes for each of the sources->n
    // particles it was sized for)
    if (self && !tidx && pmax * sizeof(uint2) <= 4ull * sr.n) {
        plan = reinterpret_cast<uint2 *>(ws.keys[0]);
        nplan = ws.keys[1];
        blocks = mx ? div_up(2 * pmax, kMxWaves) : div_up(pmax, kWaves);   // k_pairs_mx: two wavefronts per entry
    }
    const bool use_mx = mx && plan;
    if (sr.n > 0) {
        // one more workgroup (the first) builds the wavefront plan
        k_stage<real, SOLID><<<div_up(sr.n, kBlock) + (plan ? 1 : 0), kBlock, 0, s>>>(g, view<real>(sr), st, sstart,
                                                                                    plan, nplan);
        if constexpr (ADJ) {
            const sph_rates none{};
            const RV<real> rs = view<real>(rsrc ? *rsrc : none);
            if constexpr (PASS == kPassGradAdjoint)
                k_stage_lbar<real><<<div_up(sr.n, kBlock), kBlock, 0, s>>>(sr.n, rs, st);
            else
                k_stage_rbar<real><<<div_up(sr.n, kBlock), kBlock, 0, s>>>(sr.n, rs, st);
        }
    }
    hipEvent_t ev_begin = static_cast<hipEvent_t>(g_pair_events[0].load());
    hipEvent_t ev_end = static_cast<hipEvent_t>(g_pair_events[1].load());
    if (ev_begin && ev_end) {
        const hipError_t e = hipEventRecord(ev_begin, s);
        if (e != hipSuccess) return e;
    }
    if constexpr (MX_PASS) {
        if (use_mx) {
            k_pairs_mx<real, PASS == kPassCensus><<<blocks, kMxWaves * kWave, 0, s>>>(
                P, g, view<real>(tg), st, sstart, zero_first, view<real>(r), plan, nplan, cz);
            const hipError_t le = hipGetLastError();
            if (le != hipSuccess) return le;
            if (ev_begin && ev_end) return hipEventRecord(ev_end, s);
            return hipSuccess;
        }
    }
    if (self)
        k_pairs<real, PASS, SOLID, true><<<blocks, kPairBlock, 0, s>>>(P, g, view<real>(tg), tidx, nt, st, sstart,
                                                                     zero_first, view<real>(r), view<real>(bar),
                                                                     plan, nplan, cz);
    else
        k_pairs<real, PASS, SOLID, false><<<blocks, kPairBlock, 0, s>>>(P, g, view<real>(tg), tidx, nt, st, sstart,
                                                                      zero_first, view<real>(r), view<real>(bar),
                                                                      plan, nplan, cz);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return le;
    if (ev_begin && ev_end) return hipEventRecord(ev_end, s);
    return hipSuccess;
}

template <typename real>
hipError_t go_prec(const Params &P, const Grid &g, int pass, const sph_particles &tg, const uint32_t *tidx,
                   const uint32_t *nt, const sph_particles &sr, const uint32_t *sstart, bool self,
                   int zero_first, const sph_rates &r, const Workspace &ws, hipStream_t s)
{
    const sph_adjoint none{};
    if (pass == SPH_PASS_GRADIENT)
        return go<real, SPH_PASS_GRADIENT, false>(P, g, tg, tidx, nt, sr, sstart, self, zero_first, r, none, ws, s);
    if (P.material == SPH_SOLID_J2)
        return go<real, SPH_PASS_FORCE, true>(P, g, tg, tidx, nt, sr, sstart, self, zero_first, r, none, ws, s);
    return go<real, SPH_PASS_FORCE, false>(P, g, tg, tidx, nt, sr, sstart, self, zero_first, r, none, ws, s);
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

hipError_t launch_census(const Params &P, const Grid &g, int prec, int pass, const sph_particles &tg,
                         const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr, const uint32_t *sstart,
                         bool self, uint32_t *count, uint64_t *sum, const Workspace &ws, hipStream_t s)
{
    const sph_rates none{};
    const sph_adjoint nobar{};
    const Census cz{count, reinterpret_cast<unsigned long long *>(sum), sr.id};
    const bool grad = pass == SPH_PASS_GRADIENT;
    const bool solid = !grad && P.material == SPH_SOLID_J2;
    if (prec == SPH_FP64) {
        if (solid)
            return go<double, kPassCensus, true>(P, g, tg, tidx, nt, sr, sstart, self, 1, none, nobar, ws, s, cz);
        return go<double, kPassCensus, false>(P, g, tg, tidx, nt, sr, sstart, self, 1, none, nobar, ws, s, cz, grad);
    }
    if (solid) return go<float, kPassCensus, true>(P, g, tg, tidx, nt, sr, sstart, self, 1, none, nobar, ws, s, cz);
    return go<float, kPassCensus, false>(P, g, tg, tidx, nt, sr, sstart, self, 1, none, nobar, ws, s, cz, grad);
}

hipError_t launch_interact_adjoint(const Params &P, const Grid &g, int prec, int pass, const sph_particles &tg,
                                   const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr,
                                   const uint32_t *sstart, bool self, const sph_rates &rbar_t,
                                   const sph_rates &rbar_s, const sph_adjoint &bar, const Workspace &ws,
                                   hipStream_t s)
{
    const bool solid = P.material == SPH_SOLID_J2;
    if (prec == SPH_FP64) {
        if (pass == SPH_PASS_GRADIENT)
            return go<double, kPassGradAdjoint, false>(P, g, tg, tidx, nt, sr, sstart, self, 0, rbar_t, bar, ws, s,
                                                       Census{}, false, &rbar_s);
        if (solid)
            return go<double, kPassAdjoint, true>(P, g, tg, tidx, nt, sr, sstart, self, 0, rbar_t, bar, ws, s,
                                                  Census{}, false, &rbar_s);
        return go<double, kPassAdjoint, false>(P, g, tg, tidx, nt, sr, sstart, self, 0, rbar_t, bar, ws, s, Census{},
                                               false, &rbar_s);
    }
    if (pass == SPH_PASS_GRADIENT)
        return go<float, kPassGradAdjoint, false>(P, g, tg, tidx, nt, sr, sstart, self, 0, rbar_t, bar, ws, s,
                                                  Census{}, false, &rbar_s);
    if (solid)
        return go<float, kPassAdjoint, true>(P, g, tg, tidx, nt, sr, sstart, self, 0, rbar_t, bar, ws, s, Census{},
                                             false, &rbar_s);
    return go<float, kPassAdjoint, false>(P, g, tg, tidx, nt, sr, sstart, self, 0, rbar_t, bar, ws, s, Census{},
                                          false, &rbar_s);
}

hipError_t launch_interact(const Params &P, const Grid &g, int prec, int pass, const sph_particles &tg,
                           const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr,
                           const uint32_t *sstart, bool self, int zero_first, const sph_rates &r,
                           const Workspace &ws, hipStream_t s)
{
    if (prec == SPH_FP64)
        return go_prec<double>(P, g, pass, tg, tidx, nt, sr, sstart, self, zero_first, r, ws, s);
    return go_prec<float>(P, g, pass, tg, tidx, nt, sr, sstart, self, zero_first, r, ws, s);
}

void set_pair_events(void *begin, void *end)
{
    g_pair_events[0].store(begin);
    g_pair_events[1].store(end);
}

}  // namespace sph
