// Internal definitions shared by the HIP kernels and the C ABI of libsph.
// gfx950 (CDNA4) only: 64-lane wavefronts, 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph.h"

namespace sph {

constexpr int kBlock = 256;          // threads per workgroup for streaming kernels
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kXcds = 8;             // accelerator dies (XCDs), each with its own L2

// Workgroups are dispatched to the XCDs in turn (workgroup b runs on XCD
// b mod 8).  This maps the launch index to a tile index so that each XCD
// works through one contiguous run of tiles, keeping the data that
// neighbouring tiles share in that XCD's L2.  A bijection on [0, n).
__device__ inline uint32_t xcd_tile(uint32_t b, uint32_t n)
{
    const uint32_t x = b % kXcds, k = b / kXcds;
    const uint32_t q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + k;
}

// The same mapping when only the first `active` tiles of a larger grid have
// work (a grid sized for an upper bound that the device fills in): each XCD
// takes an equal share of the active tiles, one contiguous run, and the
// workgroups past their XCD's share get no tile (false).  With xcd_tile the
// idle tiles would all fall on the last XCDs and leave the others a larger
// share of the work.
__device__ inline bool xcd_tile_active(uint32_t b, uint32_t active, uint32_t &tile)
{
    const uint32_t x = b % kXcds, k = b / kXcds;
    const uint32_t q = active / kXcds, r = active % kXcds;
    if (k >= q + (x < r ? 1u : 0u)) return false;
    tile = x * q + (x < r ? x : r) + k;
    return true;
}
#ifndef SPH_SORT_ITEMS
#define SPH_SORT_ITEMS 8
#endif
constexpr int kSortItems = SPH_SORT_ITEMS;   // keys per thread in a radix-sort tile
constexpr int kSortTile = kBlock * kSortItems;
constexpr int kMaxRadixBits = 10;     // digits of 8 to 10 bits: keys up to 20 bits sort in two passes
constexpr int kMaxRadixBins = 1 << kMaxRadixBits;
constexpr int kDiag = 8;             // integrate diagnostics (next dt, totals, non-finite count)
constexpr int kDiagPartial = 8;      // per-block partial record (doubles)
static_assert(kDiag <= kDiagPartial, "a partial record holds the diagnostics");
constexpr int kMaxTypes = SPH_MAX_TYPES;   // particle types balanced separately

// Device view of the grid: origin, bucket side and its float copy.
struct Grid {
    double o[3];
    double L;
    float Lf;
    int nx, ny, nz;
    uint32_t ncells;
};

// Constants the kernels read, precomputed on the host.
struct Params {
    double h, rho0, c0, gamma, K, G, Y0, H, beta, cfl;
    double g[3], wlo[3], whi[3];
    uint32_t wall_mask;
    int material;
    double R2;            // (2h)^2, the neighbour predicate bound
    double hinv;          // 1 / h
    double Fc;            // 1 / (pi h^4): F = Fc f(q)
    double B;             // Tait stiffness rho0 c0^2 / gamma
    double c_solid;       // solid sound speed (linear EOS)
    int eos;              // sph_solid_eos
    double mg_s, mg_gamma0, p_cut;
    int gamma_odd;        // gamma when it is an odd integer in [1, 15] (powers by products), else 0
};

// s^k for 0 <= k < 16 by repeated squaring (k is uniform across the launch).
__device__ inline double ipow(double s, int k)
{
    double r = 1.0, b = s;
    for (; k > 0; k >>= 1) {
        if (k & 1) r *= b;
        b *= b;
    }
    return r;
}

// Tait EOS factors s^gamma and s^((gamma - 1) / 2), s = rho / rho0.  The
// FP32-split form (real = float) takes products for an odd integer gamma:
// within a few ulp of pow in FP64, invisible once stored as float, and far
// cheaper.  The FP64 form keeps pow, the plain definition, so that its
// near-zero differences (p = B (s^gamma - 1) with s close to 1) round as
// the oracle's do.
template <typename real>
__device__ inline void tait_powers(const Params &P, double s, double &sg, double &sh)
{
    if (sizeof(real) == 4 && P.gamma_odd) {
        sh = ipow(s, (P.gamma_odd - 1) / 2);
        sg = sh * sh * s;
    } else {
        sg = pow(s, P.gamma);
        sh = pow(s, 0.5 * (P.gamma - 1.0));
    }
}

// Particle array with typed pointers.  real = float (FP32 split) or double.
template <typename real>
struct PV {
    uint32_t n;
    double *x[3];
    float *off[3];
    uint32_t *hash;
    uint32_t *id;
    real *v[3];
    real *m, *w, *rho, *p, *c, *e;
    double *E;
    real *S[6];
    real *ep;
};

template <typename real>
inline PV<real> view(const sph_particles &s)
{
    PV<real> o;
    o.n = s.n;
    for (int d = 0; d < 3; ++d) {
        o.x[d] = s.x[d];
        o.off[d] = s.off[d];
        o.v[d] = static_cast<real *>(s.v[d]);
    }
    o.hash = s.hash;
    o.id = s.id;
    o.m = static_cast<real *>(s.m);
    o.w = static_cast<real *>(s.omega);
    o.rho = static_cast<real *>(s.rho);
    o.p = static_cast<real *>(s.p);
    o.c = static_cast<real *>(s.c);
    o.e = static_cast<real *>(s.e);
    o.E = s.E;
    for (int k = 0; k < 6; ++k) o.S[k] = static_cast<real *>(s.S[k]);
    o.ep = static_cast<real *>(s.eps_p);
    return o;
}

template <typename real>
struct RV {
    real *hi[6];
    real *lo[6];
    real *Lhi[9];
    real *Llo[9];
};

template <typename real>
inline RV<real> view(const sph_rates &r)
{
    RV<real> o;
    for (int k = 0; k < 6; ++k) {
        o.hi[k] = static_cast<real *>(r.hi[k]);
        o.lo[k] = static_cast<real *>(r.lo[k]);
    }
    for (int k = 0; k < 9; ++k) {
        o.Lhi[k] = static_cast<real *>(r.Lhi[k]);
        o.Llo[k] = static_cast<real *>(r.Llo[k]);
    }
    return o;
}

template <typename real>
struct AV {
    real *x[3];
    real *v[3];
    real *m, *w, *E, *rho, *p, *c, *e;
    real *S[6];
    real *ep;
};

template <typename real>
inline AV<real> view(const sph_adjoint &a)
{
    AV<real> o;
    for (int d = 0; d < 3; ++d) {
        o.x[d] = static_cast<real *>(a.x[d]);
        o.v[d] = static_cast<real *>(a.v[d]);
    }
    o.m = static_cast<real *>(a.m);
    o.w = static_cast<real *>(a.omega);
    o.E = static_cast<real *>(a.E);
    o.rho = static_cast<real *>(a.rho);
    o.p = static_cast<real *>(a.p);
    o.c = static_cast<real *>(a.c);
    o.e = static_cast<real *>(a.e);
    for (int k = 0; k < 6; ++k) o.S[k] = static_cast<real *>(a.S[k]);
    o.ep = static_cast<real *>(a.eps_p);
    return o;
}

// Packed pair inputs of the source particles, one record per particle so a
// candidate costs one 16-byte load (FP32) and a pair two more:
//   pos = (position or bucket offset x, y, z, bucket x index), va = (v, omega),
//   vb = (rho, p, c, e), solids s0 = (S xx yy zz xy), s1 = (S xz yz, 0, 0).
template <typename real>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

// In the FP32 form the two records of a source that the pair body reads
// together (va and vb; s0 and s1) sit side by side in one 32-byte pair, so a
// hit touches two cache lines instead of three (measured: 4 % off the FORCE
// pass on the column); the FP64 form's 32-byte records stay in separate
// arrays (paired they were 1.5 % slower).
template <typename real>
constexpr uint32_t rec_stride = sizeof(real) == 4 ? 2 : 1;

// Adjoint passes add two records of cotangents: r0 = (rbar 0..3) and
// r1 = (rbar 4, 5, 0, 0) of the sources' rates (FORCE), or, for the
// GRADIENT reverse, the velocity-gradient cotangent Lbar in vb (0..3), r0
// (4..7) and r1.x (8).
template <typename real>
struct Stage {
    using v4 = typename Vec4<real>::type;
    v4 *pos, *va, *vb, *s0, *s1, *r0, *r1;   // all but pos: record j at [rec_stride<real> j]
};

// Bytes per source particle of the packed records: three for a fluid pass,
// seven for material SPH_SOLID_J2 (the solid pass's two stress records and
// the adjoint passes' two cotangent records).
inline size_t stage_bytes(int prec, int material)
{
    size_t rec = prec == SPH_FP64 ? 32 : 16;
    return rec * (material == SPH_SOLID_J2 ? 7 : 3);
}

// Workspace layout for n particles (256-byte aligned pieces).  The packed
// source records come last; calls other than sph_interact never touch them.
struct Workspace {
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *hist;        // kMaxRadixBins * sort tiles
    uint32_t *totals;      // kMaxRadixBins
    uint32_t *counts;      // compaction block counts (+1)
    double *partials;      // kDiagPartial * reduction blocks
    char *stage;           // n * stage bytes
    size_t bytes;
};

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

inline Workspace carve(void *base, uint32_t n, size_t stage_per_particle)
{
    Workspace w;
    uint64_t nn = n > 0 ? n : 1;
    uint32_t tiles = div_up(nn, kSortTile);
    uint32_t blocks = div_up(nn, kBlock);
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t b) {
        char *r = p ? p + off : nullptr;
        off += align256(b);
        return r;
    };
    for (int k = 0; k < 2; ++k) {
        w.keys[k] = reinterpret_cast<uint32_t *>(take(4 * nn));
        w.vals[k] = reinterpret_cast<uint32_t *>(take(4 * nn));
    }
    w.hist = reinterpret_cast<uint32_t *>(take(4ull * kMaxRadixBins * tiles));
    w.totals = reinterpret_cast<uint32_t *>(take(4ull * kMaxRadixBins));
    w.counts = reinterpret_cast<uint32_t *>(take(4ull * (blocks + 1)));
    w.partials = reinterpret_cast<double *>(take(8ull * kDiagPartial * blocks));
    w.stage = take(stage_per_particle * nn);
    w.bytes = off;
    return w;
}

// Records 0 (pos), 1-2 (va, vb), 3-4 (s0, s1 for solids), then the adjoint's
// (r0, r1): records 3-4 of a fluid adjoint, 5-6 of a solid one.
template <typename real>
inline Stage<real> stage_view(const Workspace &w, uint32_t n, bool solid, bool adj = false)
{
    using v4 = typename Vec4<real>::type;
    Stage<real> s;
    v4 *b = reinterpret_cast<v4 *>(w.stage);
    size_t nn = n > 0 ? n : 1;
    auto pair_at = [&](size_t rec, v4 *&first, v4 *&second) {
        first = b + rec * nn;
        second = rec_stride<real> == 2 ? first + 1 : b + (rec + 1) * nn;
    };
    s.pos = b;
    pair_at(1, s.va, s.vb);
    s.s0 = s.s1 = s.r0 = s.r1 = nullptr;
    if (solid) pair_at(3, s.s0, s.s1);
    if (adj) pair_at(solid ? 5 : 3, s.r0, s.r1);
    return s;
}

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error; arguments were validated.

void set_pair_events(void *begin, void *end);
hipError_t launch_build_cells(const Grid &g, int prec, const sph_particles &in, const sph_particles &out,
                              uint32_t *perm, uint32_t *start, const Workspace &ws, hipStream_t s);
// Largest local array sph_mark_boundary_noalloc takes (its block counts live
// in a fixed device array of kNoAllocMarkMax / kBlock + 1 words, 1 MiB).
constexpr uint32_t kNoAllocMarkMax = 1u << 26;
hipError_t launch_mark_boundary_noalloc(const Grid &g, const sph_particles &local, const uint32_t *rstart,
                                        uint32_t *comm, uint32_t *bidx, uint32_t cap, uint32_t *nb,
                                        uint32_t *nflag, hipStream_t s);
hipError_t launch_mark_boundary(const Grid &g, const sph_particles &local, const uint32_t *rstart,
                                uint32_t *comm, uint32_t *bidx, uint32_t cap, uint32_t *nb, uint32_t *nflag,
                                const Workspace &ws, hipStream_t s);
hipError_t launch_pack(int prec, const sph_particles &local, const uint32_t *bidx, const uint32_t *nb,
                       const sph_particles &payload, hipStream_t s);
hipError_t launch_interact(const Params &P, const Grid &g, int prec, int pass, const sph_particles &tg,
                           const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr,
                           const uint32_t *sstart, bool self, int zero_first, const sph_rates &r,
                           const Workspace &ws, hipStream_t s);
hipError_t launch_census(const Params &P, const Grid &g, int prec, int pass, const sph_particles &tg,
                         const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr, const uint32_t *sstart,
                         bool self, uint32_t *count, uint64_t *sum, const Workspace &ws, hipStream_t s);
hipError_t launch_count_pairs(const Params &P, const Grid &g, int prec, const sph_particles &tg,
                              const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr,
                              const uint32_t *sstart, bool self, uint64_t *counts, hipStream_t s);
hipError_t launch_integrate(const Params &P, int prec, int stage, const sph_particles &p,
                            const sph_rates &r, const double *dt, double *diag, const Workspace &ws,
                            hipStream_t s);
hipError_t launch_interact_adjoint(const Params &P, const Grid &g, int prec, int pass, const sph_particles &tg,
                                   const uint32_t *tidx, const uint32_t *nt, const sph_particles &sr,
                                   const uint32_t *sstart, bool self, const sph_rates &rbar_t,
                                   const sph_rates &rbar_s, const sph_adjoint &bar, const Workspace &ws,
                                   hipStream_t s);
hipError_t launch_integrate_adjoint(const Params &P, int prec, int stage, const sph_particles &p,
                                    const sph_rates &r, const double *dt, const sph_adjoint &bar,
                                    const sph_rates &rbar, double *pbar, const Workspace &ws,
                                    hipStream_t s);
hipError_t launch_centroid(int prec, const sph_particles &p, double *cg, const Workspace &ws, hipStream_t s);
hipError_t launch_balance_hash(const sph_particles &p, const double *cg_own, const double *cg_other,
                               uint32_t hmax, uint32_t *bhash, uint32_t *npos, const Workspace &ws, hipStream_t s);
hipError_t launch_balance_select(uint32_t n, const uint32_t *bhash, uint32_t hmax, const uint32_t *npos_own,
                                 const uint32_t *npos_other, uint32_t *sel, uint32_t *k_out, const Workspace &ws,
                                 hipStream_t s);
hipError_t launch_swap(int prec, const sph_particles &a, const uint32_t *sel_a, const sph_particles &b,
                       const uint32_t *sel_b, const uint32_t *k_dev, uint32_t k_max, hipStream_t s);
hipError_t launch_centroid_types(int prec, const sph_particles &p, const uint8_t *type, uint32_t ntypes, double alpha,
                                 double *cg, const Workspace &ws, hipStream_t s);
hipError_t launch_balance_hash_types(const sph_particles &p, const uint8_t *type, uint32_t ntypes,
                                     const double *cg_own, const double *cg_other, uint32_t hmax, uint32_t *bhash,
                                     uint32_t *npos, const Workspace &ws, hipStream_t s);
hipError_t launch_balance_select_types(uint32_t n, const uint8_t *type, uint32_t ntypes, const uint32_t *bhash,
                                       uint32_t hmax, const uint32_t *npos_own, const uint32_t *npos_other,
                                       uint32_t *sel, uint32_t *k_out, uint32_t *off, const Workspace &ws,
                                       hipStream_t s);
hipError_t launch_objective_adjoint(int prec, int objective, const sph_particles &p, const uint8_t *tag,
                                    uint32_t tag_len, uint32_t ntag, double scale, const sph_adjoint &bar,
                                    hipStream_t s);
hipError_t launch_permute_adjoint(int prec, uint32_t n, const uint32_t *perm, const sph_adjoint &in,
                                  const sph_adjoint &out, hipStream_t s);

}  // namespace sph
