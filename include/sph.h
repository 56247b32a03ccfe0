/*
 * libsph: one GPU's share of the particle-decomposition SPH step on MI355X.
 *
 * The paper (Section I) finds SPH neighbours by hashing every particle into
 * cubic buckets of side 2h and radix-sorting by that hash, so a particle's
 * neighbours lie in its own bucket or the 26 surrounding ones.  Section II
 * assigns particles to GPUs regardless of position and runs, per iteration:
 * (a) hash, (b) exchange hashes, (c) communication hash marking the "MGPU
 * boundary" particles that have another GPU's particles in their bucket or
 * the surrounding buckets, (d) send those particles' data, (e) local
 * interactions, (f) interactions of local particles with the received
 * boundary particles, (g) integration.  This library is the per-GPU compute
 * of (a), (c), the packing for (d), (e), (f) and (g), plus a hand-written
 * adjoint of (e) and (g).
 *
 * Conventions shared by every call
 *   - Every pointer inside the structs and every *_dev argument is DEVICE
 *     memory owned by the caller; the structs themselves are host memory and
 *     are read before the call returns.  The library allocates nothing; the
 *     only temporary memory is the caller-provided workspace.
 *   - Calls only enqueue work on `stream` (a hipStream_t; NULL = the default
 *     stream).  They never synchronise and never read device memory on the
 *     host, so device-resident counts (n_boundary, dt) stay on the device.
 *   - Return SPH_OK or a negative sph_status.  Arguments are validated on the
 *     host before anything is enqueued; on an error nothing is enqueued and
 *     sph_last_error() describes it.  A failed kernel launch returns
 *     SPH_ERR_HIP.  n == 0 is a valid no-op.
 *   - Precision: SPH_FP64 keeps every real field in double.  SPH_FP32_SPLIT
 *     keeps positions x and total energy E in double and every other real
 *     field in float; its pair loops run in float on positions held as bucket
 *     index plus a float offset from the bucket corner (so x_j - x_i keeps
 *     its relative precision); pair sums accumulate in double and are
 *     stored as float (hi, lo) pairs whose sum carries the double result.
 *     Fields typed `void*` below are double in SPH_FP64 and float in
 *     SPH_FP32_SPLIT.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum sph_status {
    SPH_OK = 0,
    SPH_ERR_ARG = -1,          /* invalid argument; nothing enqueued            */
    SPH_ERR_WORKSPACE = -2,    /* workspace missing or smaller than required    */
    SPH_ERR_HIP = -3,          /* a HIP launch or runtime call failed           */
    SPH_ERR_UNSUPPORTED = -4   /* combination not provided (e.g. remote adjoint) */
};

enum sph_precision { SPH_FP64 = 0, SPH_FP32_SPLIT = 1 };
enum sph_material { SPH_FLUID_TAIT = 0, SPH_SOLID_J2 = 1 };
enum sph_pass { SPH_PASS_FORCE = 0, SPH_PASS_GRADIENT = 1 };
enum sph_stage { SPH_STAGE_MOTION = 0, SPH_STAGE_STRESS = 1, SPH_STAGE_EOS = 2, SPH_STAGE_INPUT_VELOCITY = 3 };
enum sph_objective { SPH_OBJ_KINETIC_ENERGY = 0, SPH_OBJ_TAGGED_MEAN_Z = 1 };

/* Particle types that the per-type balancing calls (Section III.B) accept. */
#define SPH_MAX_TYPES 8

/* Bucket grid (Section I).  Buckets are cubes of side `cell` >= 2h; bucket
 * (cx, cy, cz) covers origin + [c, c+1) * cell and has hash
 * cx + dims[0] * (cy + dims[1] * cz).  Particles outside the grid are
 * clamped into the edge buckets, which keeps the neighbour search complete.
 * dims[0] * dims[1] * dims[2] must be below 2^32 - 1; its value G = ncells is
 * the "garbage collector" communication hash (Section II). */
typedef struct sph_grid {
    double origin[3];
    double cell;
    int32_t dims[3];
    int32_t reserved;
} sph_grid;

/* Equation of state of a J2 solid (sph_params.eos). */
enum sph_solid_eos { SPH_EOS_LINEAR = 0, SPH_EOS_MIE_GRUNEISEN = 1 };

/* Physical constants.  Smoothing length h is one value for all particles
 * (Section II: equal particle counts balance the work only when h is
 * constant).  Tait fluid: p = rho0 c0^2 / gamma ((rho / rho0)^gamma - 1),
 * c = c0 (rho / rho0)^((gamma - 1) / 2).  J2 solid: yield Y0 + H eps_p
 * (H = 0: the elastic perfectly plastic limit of Johnson-Cook that Section
 * IV.A uses), with eos = SPH_EOS_LINEAR: p = K (rho / rho0 - 1),
 * c = sqrt((K + 4G/3) / rho0); or eos = SPH_EOS_MIE_GRUNEISEN (Section IV.A
 * names a Mie-Gruneisen EOS with a cut-off pressure; the form is the linear
 * shock-velocity one, Us = c0 + mg_s up, with Gamma rho = mg_gamma0 rho0):
 * mu = rho / rho0 - 1, e the specific internal energy,
 *   mu > 0: p = rho0 c0^2 mu (1 + (1 - mg_gamma0 / 2) mu) / D^2 + mg_gamma0 rho0 e,
 *           D = max(1 - (mg_s - 1) mu, 1/16),
 *   mu <= 0: p = rho0 c0^2 mu + mg_gamma0 rho0 e,
 * then p = max(p, p_cut) (spall cut-off, p_cut <= 0); bulk sound speed
 * cb^2 = c0^2 (1 + (2 - mg_gamma0 + mg_s - 1) mu) / D^3 (mu > 0; c0^2 else)
 * + mg_gamma0 rho0 max(p_u, 0) / rho^2 with p_u the pressure before the
 * cut-off, and c = sqrt(cb^2 + 4G / (3 rho)).  K is not read.  beta scales
 * the acoustic Riemann solver's dissipation (1 = the linearised Riemann
 * solution).  Walls: bit 2d of wall_mask reflects at wall_lo[d], bit 2d+1 at
 * wall_hi[d]. */
typedef struct sph_params {
    double h, rho0, c0, gamma, K, G, Y0, H, beta, cfl;
    double gravity[3], wall_lo[3], wall_hi[3];
    uint32_t wall_mask;
    int32_t material;      /* sph_material  */
    int32_t prec;          /* sph_precision */
    int32_t eos;           /* sph_solid_eos (solids; fluids ignore it) */
    double mg_s, mg_gamma0, p_cut;   /* Mie-Gruneisen constants and cut-off */
} sph_params;

/* One particle array in structure-of-arrays form, n entries per field.
 * x: positions (double).  off: float offsets from the bucket corner, written
 * by sph_build_cells in SPH_FP32_SPLIT (NULL in SPH_FP64).  hash: bucket
 * hash, written by sph_build_cells.  id: caller's particle identity, carried
 * through every reorder.  v, m, omega (volume), rho, p, c, e (specific
 * internal energy): real fields.  E: specific total energy (double).  S[6]
 * (xx yy zz xy xz yz) and eps_p: deviatoric stress and equivalent plastic
 * strain, SPH_SOLID_J2 only (NULL for fluids). */
typedef struct sph_particles {
    uint32_t n;
    int32_t prec;          /* sph_precision of the real fields */
    double *x[3];
    float *off[3];
    uint32_t *hash;
    uint32_t *id;
    void *v[3];
    void *m, *omega, *rho, *p, *c, *e;
    double *E;
    void *S[6];
    void *eps_p;
} sph_particles;

/* Bucket table: start[c] = number of particles (in hash order) whose hash is
 * below c, for c = 0..ncells, so bucket c holds [start[c], start[c+1]). */
typedef struct sph_cells {
    uint32_t *start;       /* ncells + 1 entries */
    uint32_t ncells;
    uint32_t reserved;
} sph_cells;

/* Pair-sum outputs, indexed like the target array.  hi[k]: rates of mass,
 * momentum x, y, z, total energy and volume (FORCE pass); L: velocity
 * gradient L_ab = dv_a / dx_b, row-major (GRADIENT pass).  lo / Llo hold the
 * compensation terms in SPH_FP32_SPLIT (the rate is hi + lo) and are NULL in
 * SPH_FP64. */
typedef struct sph_rates {
    void *hi[6];
    void *lo[6];
    void *Lhi[9];
    void *Llo[9];
} sph_rates;

/* Adjoint (cotangent) of a particle state, same precision as the form:
 * x, v, m, omega, E (and, for J2 solids, S and eps_p) are the state variables
 * of one step; rho, p, c, e are the cotangents of the derived fields that the
 * pair terms read.  S and eps_p are NULL for fluids. */
typedef struct sph_adjoint {
    void *x[3];
    void *v[3];
    void *m, *omega, *E;
    void *rho, *p, *c, *e;
    void *S[6];
    void *eps_p;
} sph_adjoint;

/* Library version string (static storage). */
const char *sph_version(void);

/* Description of the last error on the calling thread (static per thread). */
const char *sph_last_error(void);

/* Bytes of workspace the calls below need for arrays of up to n_max
 * particles of precision `prec` (sph_precision) and material `material`
 * (sph_material).  One workspace may be reused by consecutive calls on one
 * stream; calls that overlap on different streams need their own. */
size_t sph_workspace_size(const sph_grid *grid, uint32_t n_max, int prec, int material);

/* Steps (a) and the Section I bucket sort.  Hashes every particle of `in`
 * into `grid`, stable-radix-sorts by hash (ties keep the order of `in`),
 * writes every field present in `in` to `out` in sorted order (plus out->hash
 * and, in SPH_FP32_SPLIT, out->off), perm_out[k] = index in `in` of the
 * particle now at k, and the bucket table.  in and out must not overlap and
 * must have the same n, prec and non-NULL fields.  cells.ncells must equal
 * the grid's bucket count.  Errors: SPH_ERR_ARG (NULL field mismatch, grid
 * too large, cell <= 0), SPH_ERR_WORKSPACE. */
int sph_build_cells(const sph_grid *grid, const sph_particles *in, sph_particles *out,
                    uint32_t *perm_out, sph_cells cells, void *ws, size_t ws_bytes, void *stream);

/* Step (c).  For the hash-sorted `local` array and the bucket table of the
 * separately stored remote particles (other GPUs' particles on the same grid),
 * comm_hash_out[i] = local->hash[i] if a remote particle lies in i's bucket or
 * a surrounding bucket, else G = ncells.  Because `local` is already in hash
 * order, the stable sort by communication hash that isolates the boundary
 * particles reduces to a stable compaction: boundary_idx_out receives the
 * flagged indices in ascending order, at most boundary_cap of them, and
 * *n_boundary_dev (one uint32 on the device) the number it received,
 * min(flagged, boundary_cap): the count that sph_pack_boundary and
 * sph_interact read with this list, so no consumer reads past its end.
 * *n_flagged_dev (one uint32 on the device; may be NULL) receives the number
 * of flagged particles, above *n_boundary_dev when the list overflowed (the
 * caller checks after synchronising, grows the list and marks again).
 * Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
int sph_mark_boundary(const sph_grid *grid, const sph_particles *local, sph_cells remote_cells,
                      uint32_t *comm_hash_out, uint32_t *boundary_idx_out, uint32_t boundary_cap,
                      uint32_t *n_boundary_dev, uint32_t *n_flagged_dev, void *ws, size_t ws_bytes,
                      void *stream);

/* sph_mark_boundary for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same step (c) and the same results, with no workspace
 * argument.  Its temporary block counts live in a fixed array inside the
 * library, one per GPU (1 MiB, held until the process ends), so it takes at
 * most 2^26 = 67,108,864 local particles and calls no allocator.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams or host threads) race and must be ordered by the caller.
 * Errors: SPH_ERR_ARG (as sph_mark_boundary, and local->n above 2^26),
 * SPH_ERR_HIP. */
int sph_mark_boundary_noalloc(const sph_grid *grid, const sph_particles *local, sph_cells remote_cells,
                              uint32_t *comm_hash_out, uint32_t *boundary_idx_out, uint32_t boundary_cap,
                              uint32_t *n_boundary_dev, uint32_t *n_flagged_dev, void *stream);

/* Packing for step (d): payload[k] = local[boundary_idx[k]] for
 * k < min(*n_boundary_dev, payload->n), every field present in payload
 * (payload->n is its capacity; its fields must be a subset of local's).  An
 * index at or above local->n names no particle: its row is left unwritten.
 * Errors: SPH_ERR_ARG. */
int sph_pack_boundary(const sph_particles *local, const uint32_t *boundary_idx,
                      const uint32_t *n_boundary_dev, sph_particles *payload, void *stream);

/* Steps (e) and (f).  For every target i (all of `targets` when target_idx is
 * NULL, else target_idx[k] for k < *n_targets_dev, at most targets->n; an
 * index at or above targets->n names no target), sums
 * the pair terms over sources j with |x_j - x_i| < 2h found through the
 * sources' bucket table.  Pairs with r = 0 (j == i in the local-local pass,
 * step e, or coincident particles) add nothing.  pass = SPH_PASS_FORCE: rates
 * of mass, momentum, energy and volume from the acoustic Riemann solver
 * (solids: Cauchy stress -p I + S); SPH_PASS_GRADIENT: velocity gradient L.
 * zero_first = 1 overwrites the rate entries of the targets, 0 adds to them
 * (the local-remote pass, step f, continues the sums of step e from hi + lo).
 * Summation over j runs in ascending source index (the FP64 fluid FORCE pass
 * over every target: two sums, each over every other run of four sources of
 * a row in ascending index, then added).  Both arrays must be
 * hash-sorted on `grid`.  The workspace receives a packed copy of the
 * sources' pair inputs (sized by sph_workspace_size for sources->n).
 * Errors: SPH_ERR_ARG (precision or material mismatch, missing field,
 * sources->n at or above 2^27 = 134,217,728), SPH_ERR_WORKSPACE. */
int sph_interact(const sph_params *params, const sph_grid *grid, int pass,
                 const sph_particles *targets, const uint32_t *target_idx,
                 const uint32_t *n_targets_dev, const sph_particles *sources, sph_cells source_cells,
                 int zero_first, const sph_rates *rates, void *ws, size_t ws_bytes, void *stream);

/* Step (g).  stage = SPH_STAGE_MOTION: symplectic Euler update of mass,
 * momentum, volume, energy and position with gravity and reflective walls,
 * then the EOS (rho = m / omega, p, c, e).  SPH_STAGE_STRESS (solids): Jaumann
 * rate of S from L, J2 radial return with linear hardening.  SPH_STAGE_EOS:
 * the EOS alone (priming the initial state).  dt_dev: one double on the
 * device.  diag_dev (8 doubles, may be NULL for SPH_STAGE_STRESS): [0] next dt
 * = cfl h / max(c + |v|), [1] total mass, [2..4] total momentum, [5] total
 * energy sum m E, [6] kinetic energy, [7] number of particles with a field
 * that is not finite after the stage (x, v, m, omega, E, rho, p, c: a
 * blow-up guard the caller reads when it synchronises); sums are
 * deterministic.  Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
int sph_integrate(const sph_params *params, int stage, sph_particles *p, const sph_rates *rates,
                  const double *dt_dev, double *diag_dev, void *ws, size_t ws_bytes, void *stream);

/* Work count of one interaction pass (steps e and f), for throughput and
 * roofline figures: adds to counts_dev[0] the number of candidate sources
 * (particles in the 27 surrounding buckets, j != i in a local-local pass) and
 * to counts_dev[1] the number of pairs with |x_j - x_i| < 2h, over the same
 * targets and with the same predicate as sph_interact in params->prec.
 * counts_dev: two uint64 on the device, not cleared.  Errors: SPH_ERR_ARG. */
int sph_count_pairs(const sph_params *params, const sph_grid *grid, const sph_particles *targets,
                    const uint32_t *target_idx, const uint32_t *n_targets_dev,
                    const sph_particles *sources, sph_cells source_cells, uint64_t *counts_dev,
                    void *stream);

/* Measurement hook, not part of the method.  Given two hipEvent_t handles
 * (created by the caller with timing enabled, still owned by the caller),
 * every later call that runs a pair kernel (sph_interact,
 * sph_interact_adjoint, sph_neighbor_census) records begin_event on its
 * stream immediately before launching the pair kernel and end_event
 * immediately after, so that the kernel alone can be timed (the staging of
 * the source records and the wavefront plan run before it in the same
 * call).  NULL, NULL stops the recording.  The setting is process-wide and
 * meant for a benchmark that times one call at a time.
 * Errors: SPH_ERR_ARG when only one of the two handles is given. */
int sph_set_pair_events(void *begin_event, void *end_event);

/* Neighbour census of one interaction pass (Section I: a particle's
 * neighbours lie in its own bucket or the 26 around it).  Takes the arguments
 * of sph_interact without the rates and runs the same staging, wavefront
 * mapping, candidate filter, hit lists and neighbour predicate as that pass
 * would (pass and params->material choose which), but instead of the pair
 * terms it writes, for every target i, count_out[i] = the number of sources
 * j the pass evaluates (r_ij^2 < (2h)^2 on the position difference the pass
 * rebuilds; j == i and coincident particles, whose terms are exactly zero,
 * included) and checksum_out[i] = the sum modulo 2^64 of
 * splitmix64(sources->id[j]) over them, with
 *   splitmix64(k): z = k + 0x9E3779B97F4A7C15;
 *                  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;
 *                  z = (z ^ (z >> 27)) * 0x94D049BB133111EB; return z ^ (z >> 31)
 * (Steele, Lea and Flood 2014), so two neighbour sets are compared by id
 * without listing them.  count_out (u32) and checksum_out (u64) are device
 * arrays indexed like the target array; entries of targets not visited are
 * left as they are.  Test and diagnostic use: it costs about a FORCE pass.
 * Errors: as sph_interact. */
int sph_neighbor_census(const sph_params *params, const sph_grid *grid, int pass,
                        const sph_particles *targets, const uint32_t *target_idx,
                        const uint32_t *n_targets_dev, const sph_particles *sources,
                        sph_cells source_cells, uint32_t *count_out, uint64_t *checksum_out,
                        void *ws, size_t ws_bytes, void *stream);

/* Adjoint of an interaction pass, steps (e) and (f).  The pass being
 * reversed is the sph_interact call with the same pass, targets, target_idx,
 * n_targets_dev, sources and source_cells; every target gathers its
 * cotangent from its own pairs, without atomics.
 *
 * pass = SPH_PASS_FORCE (fluids, and J2 solids with the linear EOS).  Each
 * pair term satisfies T(s_j, s_i) = +-T(s_i, s_j) (odd for mass, momentum
 * and energy, even for volume), so for each target i and source j within 2h
 * it accumulates into `bar` (at i) the cotangent of x, v, omega, rho, p, c,
 * e (and, for solids, S) of target i from the weight
 *   rates_bar_targets[i] + sigma * rates_bar_sources[j],
 * where rates_bar_targets (hi only; NULL = zero) is the cotangent of the
 * targets' rates summed by this pass and rates_bar_sources (hi only; NULL =
 * zero) that of the sources' rates in the mirrored pass, which sums
 * T(s_j, s_i).
 *   - local-local pass (e): targets = sources, both cotangents the same;
 *   - local-remote pass (f), local side: targets = the local array with its
 *     boundary list, sources = the remote array, rates_bar_targets = the
 *     local rates' cotangent, rates_bar_sources = the remote particles' rate
 *     cotangent (from their owner, whose own pass (f) mirrors this one), or
 *     NULL when the remote rates are not differentiated;
 *   - remote side of (f): targets = the remote array, sources = the local
 *     array, rates_bar_targets = NULL, rates_bar_sources = the local rates'
 *     cotangent: the cotangent of the received particles, which their owner
 *     adds to its own.
 * pass = SPH_PASS_GRADIENT (the velocity-gradient loop of solids).  A pair
 * puts w_j (v_j - v_i) (x) g into L_i and w_i (v_j - v_i) (x) g into L_j
 * (g = grad_i W), so with the cotangents Lbar of the targets' and of the
 * sources' L (rates_bar_*->Lhi, 9 row-major entries; NULL = zero) it
 * accumulates the cotangents of x, v and omega of every target.
 *
 * The pair terms read p and c, not c0: d/dc0 comes from the EOS reverse
 * (sph_integrate_adjoint, SPH_STAGE_EOS).  The workspace (sph_workspace_size
 * for sources->n with SPH_SOLID_J2, which has room for the extra staged
 * records) receives packed copies of the sources and their cotangents.
 * Errors: SPH_ERR_ARG (also sources->n at or above 2^27, both cotangents
 * NULL, a solid FORCE pass without S in the particles or in bar),
 * SPH_ERR_WORKSPACE, SPH_ERR_UNSUPPORTED (the Mie-Gruneisen EOS). */
int sph_interact_adjoint(const sph_params *params, const sph_grid *grid, int pass,
                         const sph_particles *targets, const uint32_t *target_idx,
                         const uint32_t *n_targets_dev, const sph_particles *sources,
                         sph_cells source_cells, const sph_rates *rates_bar_targets,
                         const sph_rates *rates_bar_sources, const sph_adjoint *bar, void *ws,
                         size_t ws_bytes, void *stream);

/* Adjoint of step (g) and of the solid stress stage (no walls, no gravity;
 * fluids, and J2 solids with the linear EOS).  stage = SPH_STAGE_MOTION: p is
 * the state BEFORE the update (hash-sorted), rates its FORCE rates; on entry
 * bar holds the cotangent of the state after the update (x, v, m, omega, E),
 * on return the direct cotangent of the state before it, and rates_bar (hi)
 * receives the cotangents of the rates; S and eps_p pass through the update
 * unchanged.  SPH_STAGE_EOS: folds the cotangents of rho, p, c and e into m,
 * omega, v, E (rho = m / omega, p and c from the EOS, e = E - |v|^2 / 2),
 * clears them, and adds d/dc0 to param_bar_dev[0] (deterministic sum; 0 for
 * the linear solid EOS, whose c does not depend on c0).  SPH_STAGE_STRESS
 * (solids): p holds S and eps_p BEFORE the stage and rates->Lhi (and Llo in
 * SPH_FP32_SPLIT) the velocity gradient it used; on entry bar->S and
 * bar->eps_p hold the cotangents of the stage's outputs, on return those of
 * its inputs, and rates_bar->Lhi receives the cotangent of L (overwritten).
 * SPH_STAGE_INPUT_VELOCITY (the end of a reverse pass whose input is the
 * initial velocity at a fixed specific internal energy, E = e + |v|^2 / 2
 * with e held): p is that initial state; bar->v += bar->E v in place, with
 * bar->E left as it is (rates, dt_dev, rates_bar, param_bar_dev and the
 * workspace are not used).
 * Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE, SPH_ERR_UNSUPPORTED (walls,
 * gravity, the Mie-Gruneisen EOS). */
int sph_integrate_adjoint(const sph_params *params, int stage, const sph_particles *p,
                          const sph_rates *rates, const double *dt_dev, const sph_adjoint *bar,
                          const sph_rates *rates_bar, double *param_bar_dev, void *ws,
                          size_t ws_bytes, void *stream);

/* Start of a reverse pass: the cotangent of a scalar objective J of the final
 * state p (any order), times `scale` (the cotangent of J itself; 1 for the
 * plain gradient), written into bar.  Every non-NULL field of bar is
 * overwritten.  SPH_OBJ_KINETIC_ENERGY: J = sum_i m_i |v_i|^2 / 2, so
 * bar->v = scale m v, bar->m = scale |v|^2 / 2 and every other field 0.
 * SPH_OBJ_TAGGED_MEAN_Z: J = the mean z of the ntag particles whose id is
 * tagged (tag: tag_len bytes on the device, tag[id] != 0 for a tagged id; an
 * id at or above tag_len is untagged), so bar->x[2] = scale / ntag on the
 * tagged particles and every other entry and field 0.  Arithmetic in FP64,
 * rounded once to the form's precision.  Needs p->v and p->m (kinetic
 * energy) or p->id (tagged mean z).  Errors: SPH_ERR_ARG. */
int sph_objective_adjoint(int objective, const sph_particles *p, const uint8_t *tag, uint32_t tag_len,
                          uint32_t ntag, double scale, const sph_adjoint *bar, void *stream);

/* Adjoint of the reorder in sph_build_cells: out[perm[k]] = in[k] for every
 * non-NULL field of the state cotangent (x, v, m, omega, E, and for solids S
 * and eps_p), n entries.  Errors: SPH_ERR_ARG. */
int sph_permute_adjoint(int prec, uint32_t n, const uint32_t *perm, const sph_adjoint *in,
                        const sph_adjoint *out, void *stream);

/* ---------------------------------------------------------------------
 * Periodic particle swapping between a pair of GPUs (Section III.A), the
 * part one GPU computes.  A round between GPUs A and B: each computes its
 * centre of gravity (sph_centroid) and, from the other's, the balancing hash
 * of its particles and the count of positive hashes (sph_balance_hash); each
 * selects its k = min(n+_A, n+_B) particles of largest hash
 * (sph_balance_select); the selected particles change GPU pairwise
 * (sph_swap, which exchanges them between two arrays on one device, the
 * stand-in for the send and receive between the GPUs).  Both GPUs keep
 * their particle counts.  The paper runs this every 20 integration loops
 * and repeats it for every GPU pair.  The arrays need not be hash-sorted;
 * after a swap the next sph_build_cells re-sorts them.
 * --------------------------------------------------------------------- */

/* Mass-weighted centre of gravity of p: cg_dev[0..2] = sum m x / sum m,
 * cg_dev[3] = sum m (FP64; a fixed summation order, so repeated calls give
 * identical results; 0 for an empty array).  Reads x and m.  The workspace is
 * sized by sph_workspace_size for p->n.  Errors: SPH_ERR_ARG,
 * SPH_ERR_WORKSPACE. */
int sph_centroid(const sph_particles *p, double *cg_dev, void *ws, size_t ws_bytes, void *stream);

/* Balancing hash of every particle of p (the GPU whose centre is
 * cg_own_dev[0..2]) towards the other GPU's centre cg_other_dev[0..2]: with
 * e = other - own and M their midpoint, t = ((x0 - M0) e0 + (x1 - M1) e1) +
 * (x2 - M2) e2 and ee = (e0 e0 + e1 e1) + e2 e2 (IEEE binary64, no
 * contraction), bhash_out[i] = 0 when t <= 0 or ee = 0, else
 * min(ceil(hmax * ((t + t) / ee)), hmax): 0 on the own side of the midpoint,
 * hmax at or beyond the other centre, proportional in between.
 * *n_positive_dev receives the number of positive hashes.  hmax is the
 * maximum swapping hash (the paper: typically 1000), 1 <= hmax < 2^20.
 * The workspace is sized by sph_workspace_size for p->n.  Errors:
 * SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
int sph_balance_hash(const sph_particles *p, const double *cg_own_dev, const double *cg_other_dev,
                     uint32_t hmax, uint32_t *bhash_out, uint32_t *n_positive_dev, void *ws, size_t ws_bytes,
                     void *stream);

/* Selection for the swap: k = min(*n_positive_own_dev, *n_positive_other_dev,
 * n) is written to *k_dev and sel_out[0..k) receives the indices of the k
 * particles of largest balancing hash, ties in ascending index (a stable
 * sort by descending hash).  bhash holds n hashes, each at most hmax;
 * sel_out has room for n entries.  The workspace is sized by
 * sph_workspace_size for n.  Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
int sph_balance_select(uint32_t n, const uint32_t *bhash, uint32_t hmax, const uint32_t *n_positive_own_dev,
                       const uint32_t *n_positive_other_dev, uint32_t *sel_out, uint32_t *k_dev, void *ws,
                       size_t ws_bytes, void *stream);

/* Pairwise exchange: for t < min(*k_dev, k_max), particle sel_a[t] of a and
 * particle sel_b[t] of b swap every field that both arrays hold (x, off,
 * hash, id, v, m, omega, rho, p, c, e, E, S, eps_p).  The entries of sel_a
 * must be distinct, and so must those of sel_b (sph_balance_select gives
 * such lists); indices out of range are skipped.  k_max bounds the launch
 * (for instance min(a->n, b->n)).  Errors: SPH_ERR_ARG (precisions differ,
 * missing lists). */
int sph_swap(sph_particles *a, const uint32_t *sel_a, sph_particles *b, const uint32_t *sel_b,
             const uint32_t *k_dev, uint32_t k_max, void *stream);

/* ---------------------------------------------------------------------
 * Balancing with several particle types (Section III.B).  Every type is
 * balanced on its own with the rule of Section III.A, and the centres that
 * rule uses are biased towards the centre of all the particles:
 *   Cg'_t = alpha Cg_all + (1 - alpha) Cg_t   (the paper takes alpha = 0.1),
 * so that the decompositions of the types do not drift apart.  A type label
 * per particle (type_dev, u8, n entries on the device) names its type;
 * labels of ntypes or more take no part (in no centre, hash 0, never
 * selected).  1 <= ntypes <= SPH_MAX_TYPES.  One round between GPUs A and B:
 * sph_centroid_types on each, sph_balance_hash_types on each towards the
 * other's centres, sph_balance_select_types on each, then sph_swap with the
 * two selections and k_dev pointing at sel_offset_dev[ntypes] (their total);
 * the selections of a type sit at the same offsets on both sides, so every
 * particle changes GPU against one of its own type and both GPUs keep their
 * count of every type.
 * --------------------------------------------------------------------- */

/* Mass-weighted centres of p by type.  cg_dev receives ntypes + 1 records of
 * four doubles: record t < ntypes holds Cg'_t (above; zeros when type t has
 * no mass in p) and the type's mass, record ntypes holds Cg_all (over the
 * particles of every valid type) and their mass.  0 <= alpha <= 1.  FP64 sums
 * in a fixed order, so repeated calls give identical results.  Reads x, m and
 * type_dev.  The workspace is sized by sph_workspace_size for p->n.  Errors:
 * SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
int sph_centroid_types(const sph_particles *p, const uint8_t *type_dev, uint32_t ntypes, double alpha,
                       double *cg_dev, void *ws, size_t ws_bytes, void *stream);

/* Balancing hash of every particle towards its type's centres: the rule of
 * sph_balance_hash with own = record t of cg_own_dev and other = record t of
 * cg_other_dev (records of four doubles as sph_centroid_types writes them;
 * the fourth is not read).  n_positive_dev[t] receives the number of positive
 * hashes of type t.  1 <= hmax < 2^20.  The workspace is sized by
 * sph_workspace_size for p->n.  Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
int sph_balance_hash_types(const sph_particles *p, const uint8_t *type_dev, uint32_t ntypes,
                           const double *cg_own_dev, const double *cg_other_dev, uint32_t hmax,
                           uint32_t *bhash_out, uint32_t *n_positive_dev, void *ws, size_t ws_bytes,
                           void *stream);

/* Per-type selection: for every type t, k_t = min(n_positive_own_dev[t],
 * n_positive_other_dev[t], number of particles of type t) goes to k_dev[t],
 * and sel_out[sel_offset_dev[t] + q], q < k_t, receives the indices of the
 * k_t particles of type t of largest balancing hash, ties in ascending index
 * (one stable sort by type and descending hash).  sel_offset_dev (ntypes + 1
 * entries) receives the exclusive offsets, sel_offset_dev[ntypes] their
 * total.  sel_out has room for n entries.  The workspace is sized by
 * sph_workspace_size for n.  Errors: SPH_ERR_ARG, SPH_ERR_WORKSPACE. */
int sph_balance_select_types(uint32_t n, const uint8_t *type_dev, uint32_t ntypes, const uint32_t *bhash,
                             uint32_t hmax, const uint32_t *n_positive_own_dev,
                             const uint32_t *n_positive_other_dev, uint32_t *sel_out, uint32_t *k_dev,
                             uint32_t *sel_offset_dev, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
