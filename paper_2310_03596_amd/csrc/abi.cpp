// C ABI of libsph: host-side validation, workspace carving and dispatch to
// the HIP launchers.  Nothing here touches device memory contents.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <cmath>
#include <string>

#include "common.hpp"

using namespace sph;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_status(hipError_t e, const char *what)
{
    if (e == hipSuccess) return SPH_OK;
    return fail(SPH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool make_grid(const sph_grid *sg, Grid &g)
{
    if (!sg) return fail(SPH_ERR_ARG, "grid is NULL"), false;
    if (!(sg->cell > 0.0) || !isfinite(sg->cell)) return fail(SPH_ERR_ARG, "grid cell must be > 0"), false;
    uint64_t nc = 1;
    for (int d = 0; d < 3; ++d) {
        if (sg->dims[d] < 1) return fail(SPH_ERR_ARG, "grid dims[%d] = %d < 1", d, sg->dims[d]), false;
        if (!isfinite(sg->origin[d])) return fail(SPH_ERR_ARG, "grid origin not finite"), false;
        nc *= (uint64_t)sg->dims[d];
    }
    if (nc >= 0xFFFFFFFFull) return fail(SPH_ERR_ARG, "grid has %llu buckets, must be < 2^32 - 1",
                                         (unsigned long long)nc), false;
    for (int d = 0; d < 3; ++d) g.o[d] = sg->origin[d];
    g.L = sg->cell;
    g.Lf = (float)sg->cell;
    g.nx = sg->dims[0];
    g.ny = sg->dims[1];
    g.nz = sg->dims[2];
    g.ncells = (uint32_t)nc;
    return true;
}

bool make_params(const sph_params *sp, const sph_grid *sg, Params &P)
{
    if (!sp) return fail(SPH_ERR_ARG, "params is NULL"), false;
    if (!(sp->h > 0.0)) return fail(SPH_ERR_ARG, "h must be > 0"), false;
    if (sp->prec != SPH_FP64 && sp->prec != SPH_FP32_SPLIT)
        return fail(SPH_ERR_ARG, "unknown precision %d", sp->prec), false;
    if (sp->material != SPH_FLUID_TAIT && sp->material != SPH_SOLID_J2)
        return fail(SPH_ERR_ARG, "unknown material %d", sp->material), false;
    if (!(sp->rho0 > 0.0)) return fail(SPH_ERR_ARG, "rho0 must be > 0"), false;
    if (sp->material == SPH_FLUID_TAIT && !(sp->gamma > 0.0 && sp->c0 > 0.0))
        return fail(SPH_ERR_ARG, "Tait fluid needs gamma > 0 and c0 > 0"), false;
    if (sp->material == SPH_SOLID_J2) {
        if (sp->eos != SPH_EOS_LINEAR && sp->eos != SPH_EOS_MIE_GRUNEISEN)
            return fail(SPH_ERR_ARG, "unknown solid EOS %d", sp->eos), false;
        if (sp->eos == SPH_EOS_LINEAR && !(sp->K > 0.0 && sp->G > 0.0))
            return fail(SPH_ERR_ARG, "J2 solid needs K > 0 and G > 0"), false;
        if (sp->eos == SPH_EOS_MIE_GRUNEISEN &&
            !(sp->c0 > 0.0 && sp->G > 0.0 && sp->mg_s >= 1.0 && sp->mg_gamma0 >= 0.0 && sp->p_cut <= 0.0))
            return fail(SPH_ERR_ARG, "Mie-Gruneisen solid needs c0 > 0, G > 0, mg_s >= 1, mg_gamma0 >= 0, p_cut <= 0"),
                   false;
    }
    double R = 2.0 * sp->h;
    if (sg && sg->cell < R)
        return fail(SPH_ERR_ARG, "bucket side %g is smaller than the support 2h = %g", sg->cell, R), false;
    P.h = sp->h;
    P.rho0 = sp->rho0;
    P.c0 = sp->c0;
    P.gamma = sp->gamma;
    P.K = sp->K;
    P.G = sp->G;
    P.Y0 = sp->Y0;
    P.H = sp->H;
    P.beta = sp->beta;
    P.cfl = sp->cfl;
    for (int d = 0; d < 3; ++d) {
        P.g[d] = sp->gravity[d];
        P.wlo[d] = sp->wall_lo[d];
        P.whi[d] = sp->wall_hi[d];
    }
    P.wall_mask = sp->wall_mask;
    P.material = sp->material;
    P.R2 = R * R;
    P.hinv = 1.0 / sp->h;
    P.Fc = (1.0 / (M_PI * sp->h * sp->h * sp->h)) / sp->h;
    P.B = sp->material == SPH_FLUID_TAIT ? sp->rho0 * sp->c0 * sp->c0 / sp->gamma : 0.0;
    P.c_solid = sp->material == SPH_SOLID_J2 ? sqrt((sp->K + 4.0 * sp->G / 3.0) / sp->rho0) : 0.0;
    P.eos = sp->material == SPH_SOLID_J2 ? sp->eos : SPH_EOS_LINEAR;
    P.mg_s = sp->mg_s;
    P.mg_gamma0 = sp->mg_gamma0;
    P.p_cut = sp->p_cut;
    P.gamma_odd = 0;
    for (int k = 1; k < 16; k += 2)
        if (sp->gamma == (double)k) P.gamma_odd = k;
    return true;
}

// Fields every particle array of the hot path carries.
bool check_particles(const sph_particles *p, const char *name, bool need_off, bool solid)
{
    if (!p) return fail(SPH_ERR_ARG, "%s is NULL", name), false;
    if (p->prec != SPH_FP64 && p->prec != SPH_FP32_SPLIT)
        return fail(SPH_ERR_ARG, "%s: unknown precision %d", name, p->prec), false;
    if (p->n == 0) return true;
    for (int d = 0; d < 3; ++d) {
        if (!p->x[d]) return fail(SPH_ERR_ARG, "%s: x[%d] is NULL", name, d), false;
        if (!p->v[d]) return fail(SPH_ERR_ARG, "%s: v[%d] is NULL", name, d), false;
        if (need_off && p->prec == SPH_FP32_SPLIT && !p->off[d])
            return fail(SPH_ERR_ARG, "%s: off[%d] is NULL in SPH_FP32_SPLIT", name, d), false;
    }
    if (!p->hash || !p->id || !p->m || !p->omega || !p->rho || !p->p || !p->c || !p->e || !p->E)
        return fail(SPH_ERR_ARG, "%s: a required field (hash id m omega rho p c e E) is NULL", name), false;
    if (solid) {
        for (int k = 0; k < 6; ++k)
            if (!p->S[k]) return fail(SPH_ERR_ARG, "%s: S[%d] is NULL for a solid", name, k), false;
        if (!p->eps_p) return fail(SPH_ERR_ARG, "%s: eps_p is NULL for a solid", name), false;
    }
    return true;
}

bool check_ws(void *ws, size_t bytes, uint32_t n, Workspace &w, size_t stage = 0)
{
    size_t need = carve(nullptr, n, stage).bytes;
    if (!ws || bytes < need)
        return fail(SPH_ERR_WORKSPACE, "workspace of %zu bytes, need %zu for n = %u", ws ? bytes : 0, need, n),
               false;
    w = carve(ws, n, stage);
    return true;
}

bool check_rates(const sph_rates *r, int pass, int prec)
{
    if (!r) return fail(SPH_ERR_ARG, "rates is NULL"), false;
    if (pass == SPH_PASS_FORCE) {
        for (int k = 0; k < 6; ++k) {
            if (!r->hi[k]) return fail(SPH_ERR_ARG, "rates.hi[%d] is NULL", k), false;
            if (prec == SPH_FP32_SPLIT && !r->lo[k]) return fail(SPH_ERR_ARG, "rates.lo[%d] is NULL", k), false;
        }
    } else {
        for (int k = 0; k < 9; ++k) {
            if (!r->Lhi[k]) return fail(SPH_ERR_ARG, "rates.Lhi[%d] is NULL", k), false;
            if (prec == SPH_FP32_SPLIT && !r->Llo[k]) return fail(SPH_ERR_ARG, "rates.Llo[%d] is NULL", k), false;
        }
    }
    return true;
}

}  // namespace

extern "C" {

const char *sph_version(void) { return "libsph 0.1 (gfx950, wave64)"; }

const char *sph_last_error(void) { return g_err.c_str(); }

size_t sph_workspace_size(const sph_grid *grid, uint32_t n_max, int prec, int material)
{
    (void)grid;
    return carve(nullptr, n_max, stage_bytes(prec, material)).bytes;
}

int sph_set_pair_events(void *begin_event, void *end_event)
{
    if ((begin_event == nullptr) != (end_event == nullptr))
        return fail(SPH_ERR_ARG, "give both events or neither");
    set_pair_events(begin_event, end_event);
    return SPH_OK;
}

int sph_build_cells(const sph_grid *grid, const sph_particles *in, sph_particles *out, uint32_t *perm_out,
                    sph_cells cells, void *ws, size_t ws_bytes, void *stream)
{
    Grid g;
    if (!make_grid(grid, g)) return SPH_ERR_ARG;
    if (!in || !out) return fail(SPH_ERR_ARG, "in/out is NULL");
    if (in->n != out->n) return fail(SPH_ERR_ARG, "in.n = %u != out.n = %u", in->n, out->n);
    if (in->prec != out->prec) return fail(SPH_ERR_ARG, "in and out precisions differ");
    bool solid = in->S[0] != nullptr;
    if (!check_particles(in, "in", false, solid) || !check_particles(out, "out", true, solid)) return SPH_ERR_ARG;
    if ((out->S[0] != nullptr) != solid) return fail(SPH_ERR_ARG, "in and out disagree on solid fields");
    if (in->n > 0 && in->x[0] == out->x[0]) return fail(SPH_ERR_ARG, "in and out must not overlap");
    if (!cells.start) return fail(SPH_ERR_ARG, "cells.start is NULL");
    if (cells.ncells != g.ncells)
        return fail(SPH_ERR_ARG, "cells.ncells = %u but the grid has %u buckets", cells.ncells, g.ncells);
    if (in->n > 0 && !perm_out) return fail(SPH_ERR_ARG, "perm_out is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, in->n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_build_cells(g, in->prec, *in, *out, perm_out, cells.start, w, (hipStream_t)stream),
                      "sph_build_cells");
}

int sph_mark_boundary(const sph_grid *grid, const sph_particles *local, sph_cells remote_cells,
                      uint32_t *comm_hash_out, uint32_t *boundary_idx_out, uint32_t boundary_cap,
                      uint32_t *n_boundary_dev, uint32_t *n_flagged_dev, void *ws, size_t ws_bytes, void *stream)
{
    Grid g;
    if (!make_grid(grid, g)) return SPH_ERR_ARG;
    if (!local) return fail(SPH_ERR_ARG, "local is NULL");
    if (local->n > 0 && !local->hash) return fail(SPH_ERR_ARG, "local.hash is NULL");
    if (!remote_cells.start || remote_cells.ncells != g.ncells)
        return fail(SPH_ERR_ARG, "remote bucket table missing or not on this grid");
    if (!n_boundary_dev) return fail(SPH_ERR_ARG, "n_boundary_dev is NULL");
    if (local->n > 0 && !comm_hash_out) return fail(SPH_ERR_ARG, "comm_hash_out is NULL");
    if (boundary_cap > 0 && !boundary_idx_out) return fail(SPH_ERR_ARG, "boundary_idx_out is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, local->n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_mark_boundary(g, *local, remote_cells.start, comm_hash_out, boundary_idx_out,
                                           boundary_cap, n_boundary_dev, n_flagged_dev, w, (hipStream_t)stream),
                      "sph_mark_boundary");
}

int sph_mark_boundary_noalloc(const sph_grid *grid, const sph_particles *local, sph_cells remote_cells,
                              uint32_t *comm_hash_out, uint32_t *boundary_idx_out, uint32_t boundary_cap,
                              uint32_t *n_boundary_dev, uint32_t *n_flagged_dev, void *stream)
{
    Grid g;
    if (!make_grid(grid, g)) return SPH_ERR_ARG;
    if (!local) return fail(SPH_ERR_ARG, "local is NULL");
    if (local->n > kNoAllocMarkMax)
        return fail(SPH_ERR_ARG, "local.n = %u exceeds the %u particles sph_mark_boundary_noalloc takes", local->n,
                    kNoAllocMarkMax);
    if (local->n > 0 && !local->hash) return fail(SPH_ERR_ARG, "local.hash is NULL");
    if (!remote_cells.start || remote_cells.ncells != g.ncells)
        return fail(SPH_ERR_ARG, "remote bucket table missing or not on this grid");
    if (!n_boundary_dev) return fail(SPH_ERR_ARG, "n_boundary_dev is NULL");
    if (local->n > 0 && !comm_hash_out) return fail(SPH_ERR_ARG, "comm_hash_out is NULL");
    if (boundary_cap > 0 && !boundary_idx_out) return fail(SPH_ERR_ARG, "boundary_idx_out is NULL");
    return hip_status(launch_mark_boundary_noalloc(g, *local, remote_cells.start, comm_hash_out, boundary_idx_out,
                                                   boundary_cap, n_boundary_dev, n_flagged_dev,
                                                   (hipStream_t)stream),
                      "sph_mark_boundary_noalloc");
}

int sph_pack_boundary(const sph_particles *local, const uint32_t *boundary_idx, const uint32_t *n_boundary_dev,
                      sph_particles *payload, void *stream)
{
    if (!local || !payload) return fail(SPH_ERR_ARG, "local/payload is NULL");
    if (local->prec != payload->prec) return fail(SPH_ERR_ARG, "local and payload precisions differ");
    if (payload->n == 0) return SPH_OK;
    if (!boundary_idx || !n_boundary_dev) return fail(SPH_ERR_ARG, "boundary_idx / n_boundary_dev is NULL");
    // every payload field needs its source
    const void *pf[] = {payload->x[0], payload->x[1], payload->x[2], payload->off[0], payload->off[1],
                        payload->off[2], payload->hash, payload->id, payload->v[0], payload->v[1],
                        payload->v[2], payload->m, payload->omega, payload->rho, payload->p, payload->c,
                        payload->e, payload->E, payload->S[0], payload->S[1], payload->S[2], payload->S[3],
                        payload->S[4], payload->S[5], payload->eps_p};
    const void *lf[] = {local->x[0], local->x[1], local->x[2], local->off[0], local->off[1], local->off[2],
                        local->hash, local->id, local->v[0], local->v[1], local->v[2], local->m, local->omega,
                        local->rho, local->p, local->c, local->e, local->E, local->S[0], local->S[1],
                        local->S[2], local->S[3], local->S[4], local->S[5], local->eps_p};
    for (size_t k = 0; k < sizeof(pf) / sizeof(pf[0]); ++k)
        if (pf[k] && !lf[k]) return fail(SPH_ERR_ARG, "payload field %zu has no source in local", k);
    return hip_status(launch_pack(local->prec, *local, boundary_idx, n_boundary_dev, *payload, (hipStream_t)stream),
                      "sph_pack_boundary");
}

int sph_interact(const sph_params *params, const sph_grid *grid, int pass, const sph_particles *targets,
                 const uint32_t *target_idx, const uint32_t *n_targets_dev, const sph_particles *sources,
                 sph_cells source_cells, int zero_first, const sph_rates *rates, void *ws, size_t ws_bytes,
                 void *stream)
{
    Grid g;
    Params P;
    if (!make_grid(grid, g) || !make_params(params, grid, P)) return SPH_ERR_ARG;
    if (pass != SPH_PASS_FORCE && pass != SPH_PASS_GRADIENT) return fail(SPH_ERR_ARG, "unknown pass %d", pass);
    if (!targets || !sources) return fail(SPH_ERR_ARG, "targets/sources is NULL");
    if (targets->prec != params->prec || sources->prec != params->prec)
        return fail(SPH_ERR_ARG, "particle precision does not match params.prec");
    bool solid_force = pass == SPH_PASS_FORCE && params->material == SPH_SOLID_J2;
    if (!check_particles(targets, "targets", true, solid_force) ||
        !check_particles(sources, "sources", true, solid_force))
        return SPH_ERR_ARG;
    if (target_idx && !n_targets_dev) return fail(SPH_ERR_ARG, "target_idx given without n_targets_dev");
    if (!source_cells.start || source_cells.ncells != g.ncells)
        return fail(SPH_ERR_ARG, "source bucket table missing or not on this grid");
    if (!check_rates(rates, pass, params->prec)) return SPH_ERR_ARG;
    if (targets->n == 0) return SPH_OK;
    // hit records are addressed with 32-bit byte offsets (at most 32 bytes per source and array)
    const uint32_t src_max = 1u << 27;
    if (sources->n >= src_max) return fail(SPH_ERR_ARG, "sources.n = %u must be below %u", sources->n, src_max);
    Workspace w;
    int staged_material = pass == SPH_PASS_FORCE ? params->material : SPH_FLUID_TAIT;
    if (!check_ws(ws, ws_bytes, sources->n, w, stage_bytes(params->prec, staged_material))) return SPH_ERR_WORKSPACE;
    bool self = targets->hash == sources->hash;
    if (self && targets->n != sources->n)
        return fail(SPH_ERR_ARG, "targets and sources share their hash array but not their size");
    return hip_status(launch_interact(P, g, params->prec, pass, *targets, target_idx, n_targets_dev, *sources,
                                      source_cells.start, self, zero_first, *rates, w, (hipStream_t)stream),
                      "sph_interact");
}

int sph_neighbor_census(const sph_params *params, const sph_grid *grid, int pass, const sph_particles *targets,
                        const uint32_t *target_idx, const uint32_t *n_targets_dev, const sph_particles *sources,
                        sph_cells source_cells, uint32_t *count_out, uint64_t *checksum_out, void *ws,
                        size_t ws_bytes, void *stream)
{
    Grid g;
    Params P;
    if (!make_grid(grid, g) || !make_params(params, grid, P)) return SPH_ERR_ARG;
    if (pass != SPH_PASS_FORCE && pass != SPH_PASS_GRADIENT) return fail(SPH_ERR_ARG, "unknown pass %d", pass);
    if (!targets || !sources) return fail(SPH_ERR_ARG, "targets/sources is NULL");
    if (targets->prec != params->prec || sources->prec != params->prec)
        return fail(SPH_ERR_ARG, "particle precision does not match params.prec");
    bool solid_force = pass == SPH_PASS_FORCE && params->material == SPH_SOLID_J2;
    if (!check_particles(targets, "targets", true, solid_force) ||
        !check_particles(sources, "sources", true, solid_force))
        return SPH_ERR_ARG;
    if (target_idx && !n_targets_dev) return fail(SPH_ERR_ARG, "target_idx given without n_targets_dev");
    if (!source_cells.start || source_cells.ncells != g.ncells)
        return fail(SPH_ERR_ARG, "source bucket table missing or not on this grid");
    if (targets->n == 0) return SPH_OK;
    if (!count_out || !checksum_out) return fail(SPH_ERR_ARG, "count_out/checksum_out is NULL");
    const uint32_t src_max = 1u << 27;   // as in sph_interact
    if (sources->n >= src_max) return fail(SPH_ERR_ARG, "sources.n = %u must be below %u", sources->n, src_max);
    Workspace w;
    int staged_material = pass == SPH_PASS_FORCE ? params->material : SPH_FLUID_TAIT;
    if (!check_ws(ws, ws_bytes, sources->n, w, stage_bytes(params->prec, staged_material))) return SPH_ERR_WORKSPACE;
    bool self = targets->hash == sources->hash;
    if (self && targets->n != sources->n)
        return fail(SPH_ERR_ARG, "targets and sources share their hash array but not their size");
    return hip_status(launch_census(P, g, params->prec, pass, *targets, target_idx, n_targets_dev, *sources,
                                    source_cells.start, self, count_out, checksum_out, w, (hipStream_t)stream),
                      "sph_neighbor_census");
}

int sph_count_pairs(const sph_params *params, const sph_grid *grid, const sph_particles *targets,
                    const uint32_t *target_idx, const uint32_t *n_targets_dev, const sph_particles *sources,
                    sph_cells source_cells, uint64_t *counts_dev, void *stream)
{
    Grid g;
    Params P;
    if (!make_grid(grid, g) || !make_params(params, grid, P)) return SPH_ERR_ARG;
    if (!targets || !sources) return fail(SPH_ERR_ARG, "targets/sources is NULL");
    if (targets->prec != params->prec || sources->prec != params->prec)
        return fail(SPH_ERR_ARG, "particle precision does not match params.prec");
    if (!check_particles(targets, "targets", true, false) || !check_particles(sources, "sources", true, false))
        return SPH_ERR_ARG;
    if (target_idx && !n_targets_dev) return fail(SPH_ERR_ARG, "target_idx given without n_targets_dev");
    if (!source_cells.start || source_cells.ncells != g.ncells)
        return fail(SPH_ERR_ARG, "source bucket table missing or not on this grid");
    if (!counts_dev) return fail(SPH_ERR_ARG, "counts_dev is NULL");
    if (targets->n == 0) return SPH_OK;
    bool self = targets->hash == sources->hash;
    if (self && targets->n != sources->n)
        return fail(SPH_ERR_ARG, "targets and sources share their hash array but not their size");
    return hip_status(launch_count_pairs(P, g, params->prec, *targets, target_idx, n_targets_dev, *sources,
                                         source_cells.start, self, counts_dev, (hipStream_t)stream),
                      "sph_count_pairs");
}

int sph_integrate(const sph_params *params, int stage, sph_particles *p, const sph_rates *rates,
                  const double *dt_dev, double *diag_dev, void *ws, size_t ws_bytes, void *stream)
{
    Params P;
    if (!make_params(params, nullptr, P)) return SPH_ERR_ARG;
    if (stage != SPH_STAGE_MOTION && stage != SPH_STAGE_STRESS && stage != SPH_STAGE_EOS)
        return fail(SPH_ERR_ARG, "unknown stage %d", stage);
    if (!p) return fail(SPH_ERR_ARG, "particles is NULL");
    if (p->prec != params->prec) return fail(SPH_ERR_ARG, "particle precision does not match params.prec");
    bool solid = params->material == SPH_SOLID_J2;
    if (stage == SPH_STAGE_STRESS && !solid) return fail(SPH_ERR_ARG, "the stress stage needs a solid");
    if (!check_particles(p, "particles", false, stage == SPH_STAGE_STRESS)) return SPH_ERR_ARG;
    if (stage != SPH_STAGE_EOS) {
        if (!dt_dev) return fail(SPH_ERR_ARG, "dt_dev is NULL");
        if (!check_rates(rates, stage == SPH_STAGE_MOTION ? SPH_PASS_FORCE : SPH_PASS_GRADIENT, params->prec))
            return SPH_ERR_ARG;
    }
    Workspace w{};
    if (stage != SPH_STAGE_STRESS) {
        if (!diag_dev) return fail(SPH_ERR_ARG, "diag_dev is NULL");
        if (!check_ws(ws, ws_bytes, p->n, w)) return SPH_ERR_WORKSPACE;
    }
    sph_rates none{};
    return hip_status(launch_integrate(P, params->prec, stage, *p, rates ? *rates : none, dt_dev, diag_dev, w,
                                       (hipStream_t)stream),
                      "sph_integrate");
}

int sph_interact_adjoint(const sph_params *params, const sph_grid *grid, int pass, const sph_particles *targets,
                         const uint32_t *target_idx, const uint32_t *n_targets_dev, const sph_particles *sources,
                         sph_cells source_cells, const sph_rates *rates_bar_targets,
                         const sph_rates *rates_bar_sources, const sph_adjoint *bar, void *ws, size_t ws_bytes,
                         void *stream)
{
    Grid g;
    Params P;
    if (!make_grid(grid, g) || !make_params(params, grid, P)) return SPH_ERR_ARG;
    if (pass != SPH_PASS_FORCE && pass != SPH_PASS_GRADIENT) return fail(SPH_ERR_ARG, "unknown pass %d", pass);
    const bool solid = params->material == SPH_SOLID_J2;
    if (solid && pass == SPH_PASS_FORCE && params->eos != SPH_EOS_LINEAR)
        return fail(SPH_ERR_UNSUPPORTED, "the solid adjoint is provided for the linear EOS");
    if (!targets || !sources) return fail(SPH_ERR_ARG, "targets/sources is NULL");
    if (targets->prec != params->prec || sources->prec != params->prec)
        return fail(SPH_ERR_ARG, "particle precision does not match params.prec");
    const bool solid_force = solid && pass == SPH_PASS_FORCE;
    if (!check_particles(targets, "targets", true, solid_force) ||
        !check_particles(sources, "sources", true, solid_force))
        return SPH_ERR_ARG;
    if (target_idx && !n_targets_dev) return fail(SPH_ERR_ARG, "target_idx given without n_targets_dev");
    if (!source_cells.start || source_cells.ncells != g.ncells)
        return fail(SPH_ERR_ARG, "source bucket table missing or not on this grid");
    if (!rates_bar_targets && !rates_bar_sources) return fail(SPH_ERR_ARG, "no rate cotangents given");
    const sph_rates *rb[2] = {rates_bar_targets, rates_bar_sources};
    for (int q = 0; q < 2; ++q) {
        if (!rb[q]) continue;
        const char *side = q ? "sources" : "targets";
        if (pass == SPH_PASS_FORCE) {
            for (int k = 0; k < 6; ++k)
                if (!rb[q]->hi[k]) return fail(SPH_ERR_ARG, "rates_bar_%s.hi[%d] is NULL", side, k);
        } else {
            for (int k = 0; k < 9; ++k)
                if (!rb[q]->Lhi[k]) return fail(SPH_ERR_ARG, "rates_bar_%s.Lhi[%d] is NULL", side, k);
        }
    }
    if (!bar) return fail(SPH_ERR_ARG, "bar is NULL");
    for (int d = 0; d < 3; ++d)
        if (!bar->x[d] || !bar->v[d]) return fail(SPH_ERR_ARG, "bar.x / bar.v is NULL");
    if (!bar->omega) return fail(SPH_ERR_ARG, "bar.omega is NULL");
    if (pass == SPH_PASS_FORCE && (!bar->rho || !bar->p || !bar->c || !bar->e))
        return fail(SPH_ERR_ARG, "bar.rho/p/c/e is NULL");
    if (solid_force)
        for (int k = 0; k < 6; ++k)
            if (!bar->S[k]) return fail(SPH_ERR_ARG, "bar.S[%d] is NULL for a solid", k);
    if (targets->n == 0) return SPH_OK;
    const uint32_t src_max = 1u << 27;   // as in sph_interact
    if (sources->n >= src_max) return fail(SPH_ERR_ARG, "sources.n = %u must be below %u", sources->n, src_max);
    Workspace w;
    if (!check_ws(ws, ws_bytes, sources->n, w, stage_bytes(params->prec, SPH_SOLID_J2))) return SPH_ERR_WORKSPACE;
    bool self = targets->hash == sources->hash;
    if (self && targets->n != sources->n)
        return fail(SPH_ERR_ARG, "targets and sources share their hash array but not their size");
    const sph_rates none{};
    return hip_status(launch_interact_adjoint(P, g, params->prec, pass, *targets, target_idx, n_targets_dev, *sources,
                                              source_cells.start, self, rates_bar_targets ? *rates_bar_targets : none,
                                              rates_bar_sources ? *rates_bar_sources : none, *bar, w,
                                              (hipStream_t)stream),
                      "sph_interact_adjoint");
}

int sph_integrate_adjoint(const sph_params *params, int stage, const sph_particles *p, const sph_rates *rates,
                          const double *dt_dev, const sph_adjoint *bar, const sph_rates *rates_bar,
                          double *param_bar_dev, void *ws, size_t ws_bytes, void *stream)
{
    Params P;
    if (!make_params(params, nullptr, P)) return SPH_ERR_ARG;
    const bool solid = params->material == SPH_SOLID_J2;
    if (solid && params->eos != SPH_EOS_LINEAR)
        return fail(SPH_ERR_UNSUPPORTED, "the solid adjoint is provided for the linear EOS");
    if (params->wall_mask != 0 || params->gravity[0] != 0.0 || params->gravity[1] != 0.0 ||
        params->gravity[2] != 0.0)
        return fail(SPH_ERR_UNSUPPORTED, "adjoint is provided without walls and gravity");
    if (stage != SPH_STAGE_MOTION && stage != SPH_STAGE_EOS && stage != SPH_STAGE_STRESS &&
        stage != SPH_STAGE_INPUT_VELOCITY)
        return fail(SPH_ERR_ARG, "unknown adjoint stage %d", stage);
    if (stage == SPH_STAGE_STRESS && !solid) return fail(SPH_ERR_ARG, "the stress stage needs a solid");
    if (!p || p->prec != params->prec) return fail(SPH_ERR_ARG, "particles missing or precision mismatch");
    if (!check_particles(p, "particles", false, stage == SPH_STAGE_STRESS)) return SPH_ERR_ARG;
    if (!bar) return fail(SPH_ERR_ARG, "bar is NULL");
    Workspace w{};
    if (stage == SPH_STAGE_STRESS) {
        if (!dt_dev) return fail(SPH_ERR_ARG, "dt_dev is NULL");
        if (!check_rates(rates, SPH_PASS_GRADIENT, params->prec)) return SPH_ERR_ARG;
        if (!rates_bar) return fail(SPH_ERR_ARG, "rates_bar is NULL");
        for (int k = 0; k < 9; ++k)
            if (!rates_bar->Lhi[k]) return fail(SPH_ERR_ARG, "rates_bar.Lhi[%d] is NULL", k);
        for (int k = 0; k < 6; ++k)
            if (!bar->S[k]) return fail(SPH_ERR_ARG, "bar.S[%d] is NULL", k);
        if (!bar->eps_p) return fail(SPH_ERR_ARG, "bar.eps_p is NULL");
    } else {
        for (int d = 0; d < 3; ++d)
            if (!bar->x[d] || !bar->v[d]) return fail(SPH_ERR_ARG, "bar.x / bar.v is NULL");
        if (!bar->m || !bar->omega || !bar->E) return fail(SPH_ERR_ARG, "bar.m/omega/E is NULL");
    }
    if (stage == SPH_STAGE_MOTION) {
        if (!dt_dev) return fail(SPH_ERR_ARG, "dt_dev is NULL");
        if (!check_rates(rates, SPH_PASS_FORCE, params->prec)) return SPH_ERR_ARG;
        if (!rates_bar) return fail(SPH_ERR_ARG, "rates_bar is NULL");
        for (int k = 0; k < 6; ++k)
            if (!rates_bar->hi[k]) return fail(SPH_ERR_ARG, "rates_bar.hi[%d] is NULL", k);
    } else if (stage == SPH_STAGE_EOS) {
        if (!bar->rho || !bar->p || !bar->c || !bar->e) return fail(SPH_ERR_ARG, "bar.rho/p/c/e is NULL");
        if (!param_bar_dev) return fail(SPH_ERR_ARG, "param_bar_dev is NULL");
        if (!check_ws(ws, ws_bytes, p->n, w)) return SPH_ERR_WORKSPACE;
    }
    sph_rates none{};
    return hip_status(launch_integrate_adjoint(P, params->prec, stage, *p, rates ? *rates : none, dt_dev, *bar,
                                               rates_bar ? *rates_bar : none, param_bar_dev, w,
                                               (hipStream_t)stream),
                      "sph_integrate_adjoint");
}

int sph_objective_adjoint(int objective, const sph_particles *p, const uint8_t *tag, uint32_t tag_len,
                          uint32_t ntag, double scale, const sph_adjoint *bar, void *stream)
{
    if (objective != SPH_OBJ_KINETIC_ENERGY && objective != SPH_OBJ_TAGGED_MEAN_Z)
        return fail(SPH_ERR_ARG, "unknown objective %d", objective);
    if (!p) return fail(SPH_ERR_ARG, "p is NULL");
    if (p->prec != SPH_FP64 && p->prec != SPH_FP32_SPLIT) return fail(SPH_ERR_ARG, "unknown precision %d", p->prec);
    if (!bar) return fail(SPH_ERR_ARG, "bar is NULL");
    if (!std::isfinite(scale)) return fail(SPH_ERR_ARG, "scale is not finite");
    if (objective == SPH_OBJ_KINETIC_ENERGY) {
        if (p->n > 0 && (!p->v[0] || !p->v[1] || !p->v[2] || !p->m)) return fail(SPH_ERR_ARG, "p.v or p.m is NULL");
        if (!bar->v[0] || !bar->v[1] || !bar->v[2] || !bar->m) return fail(SPH_ERR_ARG, "bar.v or bar.m is NULL");
    } else {
        if (ntag == 0) return fail(SPH_ERR_ARG, "no tagged particle (ntag = 0)");
        if (p->n > 0 && !p->id) return fail(SPH_ERR_ARG, "p.id is NULL");
        if (tag_len > 0 && !tag) return fail(SPH_ERR_ARG, "tag is NULL");
        if (!bar->x[2]) return fail(SPH_ERR_ARG, "bar.x[2] is NULL");
    }
    if (p->n == 0) return SPH_OK;
    return hip_status(launch_objective_adjoint(p->prec, objective, *p, tag, tag_len, ntag, scale, *bar,
                                               (hipStream_t)stream),
                      "sph_objective_adjoint");
}

int sph_permute_adjoint(int prec, uint32_t n, const uint32_t *perm, const sph_adjoint *in, const sph_adjoint *out,
                        void *stream)
{
    if (prec != SPH_FP64 && prec != SPH_FP32_SPLIT) return fail(SPH_ERR_ARG, "unknown precision %d", prec);
    if (n == 0) return SPH_OK;
    if (!perm || !in || !out) return fail(SPH_ERR_ARG, "perm/in/out is NULL");
    const void *a[] = {in->x[0], in->x[1], in->x[2], in->v[0], in->v[1], in->v[2], in->m, in->omega, in->E,
                       in->S[0], in->S[1], in->S[2], in->S[3], in->S[4], in->S[5], in->eps_p};
    const void *b[] = {out->x[0], out->x[1], out->x[2], out->v[0], out->v[1], out->v[2], out->m, out->omega, out->E,
                       out->S[0], out->S[1], out->S[2], out->S[3], out->S[4], out->S[5], out->eps_p};
    for (int k = 0; k < 16; ++k) {
        if ((a[k] == nullptr) != (b[k] == nullptr)) return fail(SPH_ERR_ARG, "in/out field %d mismatch", k);
        if (a[k] && a[k] == b[k]) return fail(SPH_ERR_ARG, "in and out field %d overlap", k);
    }
    return hip_status(launch_permute_adjoint(prec, n, perm, *in, *out, (hipStream_t)stream), "sph_permute_adjoint");
}

// ------------------------------------------------------------- balancing

int sph_centroid(const sph_particles *p, double *cg_dev, void *ws, size_t ws_bytes, void *stream)
{
    if (!p) return fail(SPH_ERR_ARG, "p is NULL");
    if (p->prec != SPH_FP64 && p->prec != SPH_FP32_SPLIT) return fail(SPH_ERR_ARG, "unknown precision %d", p->prec);
    if (!cg_dev) return fail(SPH_ERR_ARG, "cg_dev is NULL");
    if (p->n > 0 && (!p->x[0] || !p->x[1] || !p->x[2] || !p->m)) return fail(SPH_ERR_ARG, "x or m is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, p->n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_centroid(p->prec, *p, cg_dev, w, (hipStream_t)stream), "sph_centroid");
}

int sph_balance_hash(const sph_particles *p, const double *cg_own_dev, const double *cg_other_dev, uint32_t hmax,
                     uint32_t *bhash_out, uint32_t *n_positive_dev, void *ws, size_t ws_bytes, void *stream)
{
    if (!p) return fail(SPH_ERR_ARG, "p is NULL");
    if (!cg_own_dev || !cg_other_dev || !n_positive_dev) return fail(SPH_ERR_ARG, "a centre or the count is NULL");
    if (hmax < 1 || hmax >= (1u << 20)) return fail(SPH_ERR_ARG, "hmax = %u must be in [1, 2^20)", hmax);
    if (p->n > 0 && (!p->x[0] || !p->x[1] || !p->x[2] || !bhash_out))
        return fail(SPH_ERR_ARG, "x or bhash_out is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, p->n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_balance_hash(*p, cg_own_dev, cg_other_dev, hmax, bhash_out, n_positive_dev, w,
                                          (hipStream_t)stream),
                      "sph_balance_hash");
}

int sph_balance_select(uint32_t n, const uint32_t *bhash, uint32_t hmax, const uint32_t *n_positive_own_dev,
                       const uint32_t *n_positive_other_dev, uint32_t *sel_out, uint32_t *k_dev, void *ws,
                       size_t ws_bytes, void *stream)
{
    if (!n_positive_own_dev || !n_positive_other_dev || !k_dev)
        return fail(SPH_ERR_ARG, "a count or k_dev is NULL");
    if (hmax < 1 || hmax >= (1u << 20)) return fail(SPH_ERR_ARG, "hmax = %u must be in [1, 2^20)", hmax);
    if (n > 0 && (!bhash || !sel_out)) return fail(SPH_ERR_ARG, "bhash or sel_out is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_balance_select(n, bhash, hmax, n_positive_own_dev, n_positive_other_dev, sel_out,
                                            k_dev, w, (hipStream_t)stream),
                      "sph_balance_select");
}

int sph_swap(sph_particles *a, const uint32_t *sel_a, sph_particles *b, const uint32_t *sel_b, const uint32_t *k_dev,
             uint32_t k_max, void *stream)
{
    if (!a || !b) return fail(SPH_ERR_ARG, "a/b is NULL");
    if (a->prec != b->prec) return fail(SPH_ERR_ARG, "a and b precisions differ");
    if (a->prec != SPH_FP64 && a->prec != SPH_FP32_SPLIT) return fail(SPH_ERR_ARG, "unknown precision %d", a->prec);
    if (k_max == 0) return SPH_OK;
    if (!sel_a || !sel_b || !k_dev) return fail(SPH_ERR_ARG, "sel_a/sel_b/k_dev is NULL");
    return hip_status(launch_swap(a->prec, *a, sel_a, *b, sel_b, k_dev, k_max, (hipStream_t)stream), "sph_swap");
}

int sph_centroid_types(const sph_particles *p, const uint8_t *type_dev, uint32_t ntypes, double alpha, double *cg_dev,
                       void *ws, size_t ws_bytes, void *stream)
{
    if (!p) return fail(SPH_ERR_ARG, "p is NULL");
    if (p->prec != SPH_FP64 && p->prec != SPH_FP32_SPLIT) return fail(SPH_ERR_ARG, "unknown precision %d", p->prec);
    if (ntypes < 1 || ntypes > SPH_MAX_TYPES) return fail(SPH_ERR_ARG, "ntypes = %u must be in [1, %d]", ntypes, SPH_MAX_TYPES);
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(SPH_ERR_ARG, "alpha = %g must be in [0, 1]", alpha);
    if (!cg_dev) return fail(SPH_ERR_ARG, "cg_dev is NULL");
    if (p->n > 0 && (!p->x[0] || !p->x[1] || !p->x[2] || !p->m || !type_dev))
        return fail(SPH_ERR_ARG, "x, m or type_dev is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, p->n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_centroid_types(p->prec, *p, type_dev, ntypes, alpha, cg_dev, w, (hipStream_t)stream),
                      "sph_centroid_types");
}

int sph_balance_hash_types(const sph_particles *p, const uint8_t *type_dev, uint32_t ntypes, const double *cg_own_dev,
                           const double *cg_other_dev, uint32_t hmax, uint32_t *bhash_out, uint32_t *n_positive_dev,
                           void *ws, size_t ws_bytes, void *stream)
{
    if (!p) return fail(SPH_ERR_ARG, "p is NULL");
    if (ntypes < 1 || ntypes > SPH_MAX_TYPES) return fail(SPH_ERR_ARG, "ntypes = %u must be in [1, %d]", ntypes, SPH_MAX_TYPES);
    if (!cg_own_dev || !cg_other_dev || !n_positive_dev) return fail(SPH_ERR_ARG, "a centre or the counts are NULL");
    if (hmax < 1 || hmax >= (1u << 20)) return fail(SPH_ERR_ARG, "hmax = %u must be in [1, 2^20)", hmax);
    if (p->n > 0 && (!p->x[0] || !p->x[1] || !p->x[2] || !bhash_out || !type_dev))
        return fail(SPH_ERR_ARG, "x, type_dev or bhash_out is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, p->n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_balance_hash_types(*p, type_dev, ntypes, cg_own_dev, cg_other_dev, hmax, bhash_out,
                                                n_positive_dev, w, (hipStream_t)stream),
                      "sph_balance_hash_types");
}

int sph_balance_select_types(uint32_t n, const uint8_t *type_dev, uint32_t ntypes, const uint32_t *bhash, uint32_t hmax,
                             const uint32_t *n_positive_own_dev, const uint32_t *n_positive_other_dev,
                             uint32_t *sel_out, uint32_t *k_dev, uint32_t *sel_offset_dev, void *ws, size_t ws_bytes,
                             void *stream)
{
    if (ntypes < 1 || ntypes > SPH_MAX_TYPES) return fail(SPH_ERR_ARG, "ntypes = %u must be in [1, %d]", ntypes, SPH_MAX_TYPES);
    if (!n_positive_own_dev || !n_positive_other_dev || !k_dev || !sel_offset_dev)
        return fail(SPH_ERR_ARG, "a count, k_dev or sel_offset_dev is NULL");
    if (hmax < 1 || hmax >= (1u << 20)) return fail(SPH_ERR_ARG, "hmax = %u must be in [1, 2^20)", hmax);
    if (n > 0 && (!bhash || !sel_out || !type_dev)) return fail(SPH_ERR_ARG, "bhash, type_dev or sel_out is NULL");
    Workspace w;
    if (!check_ws(ws, ws_bytes, n, w)) return SPH_ERR_WORKSPACE;
    return hip_status(launch_balance_select_types(n, type_dev, ntypes, bhash, hmax, n_positive_own_dev,
                                                  n_positive_other_dev, sel_out, k_dev, sel_offset_dev, w,
                                                  (hipStream_t)stream),
                      "sph_balance_select_types");
}

}  // extern "C"
