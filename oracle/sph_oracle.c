/*
 * FP64 CPU oracle for the particle-decomposition SPH hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library and must never serve as a
 * fallback for it.
 *
 * What it computes, step by step (paper: Section I for bucket hashing and
 * radix sort, Section II steps a-g for the particle decomposition; the SPH
 * physics itself is only named there, so the pair terms below follow the
 * documented reading of an SPH-ALE scheme with an acoustic Riemann solver):
 *
 *   hash        bucket of side L = 2h: c_d = clamp(floor((x_d - o_d) / L), 0, n_d - 1),
 *               hash = c_x + n_x (c_y + n_y c_z)                      (Section I)
 *   sort        stable counting sort of the current order by hash    (Section I)
 *   cell start  start[c] = number of particles with hash < c         (Section I)
 *   mark        flag_i = some remote particle lies in the bucket of i or in one
 *               of the surrounding buckets; comm_i = flag ? hash_i : G, G = ncells;
 *               B = flagged particles in sorted order                 (Section II, step c)
 *   interact    per target i, sum over j with 0 < |x_i - x_j|^2 < (2h)^2 of the
 *               pair terms (Section II, steps e and f); a coincident pair has
 *               no direction and every term carries F(0) = 0, so it adds 0
 *   integrate   symplectic Euler, reflective walls, EOS              (Section II, step g)
 *   balance     centres of gravity, balancing hash towards the other GPU's
 *               centre, selection of the k = min(n+_A, n+_B) largest, and
 *               the pairwise swap                                    (Section III.A)
 *
 * Every floating-point operation is IEEE binary64, built without FMA
 * contraction.  Sums run over j in ascending sorted index, visiting the 27
 * buckets in ascending hash order.  OpenMP parallelises over targets only.
 *
 * Parity status: hash, sort, cell start, mark and the neighbour set are pinned
 * by brute force; pair terms by closed forms, antisymmetry and invariants;
 * integrate by closed forms.  Fidelity of the pair terms to the cited
 * Gamma-SPH-ALE formulation is parity unpinned (the paper gives no equations).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Sets the threads of the following OpenMP loops (no effect without OpenMP). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* Threads the OpenMP loops use (1 without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

typedef struct {
    double o[3];
    double L;
    int32_t n[3];
} og_t;

typedef struct {
    double h, rho0, c0, gamma, K, G, Y0, H, beta, cfl;
    double g[3], wlo[3], whi[3];
    int32_t wall_mask, material; /* material 0 = Tait fluid, 1 = J2 solid */
    int32_t eos, pad;            /* solids: 0 = linear, 1 = Mie-Gruneisen */
    double mg_s, mg_gamma0, p_cut;
} op_t;

typedef struct {
    int64_t n;
    double *x, *v;              /* n*3, row-major */
    double *m, *w, *rho, *p, *c, *E;
    double *S;                  /* n*6 (xx yy zz xy xz yz) or NULL */
    double *ep;                 /* n or NULL */
    uint32_t *id;
    uint32_t *hash;
} os_t;

/* ------------------------------------------------------------------ grid */

static int64_t cell_of(double x, double o, double L, int32_t n)
{
    double t = floor((x - o) / L);
    if (!(t >= 0.0)) return 0;          /* negative (or NaN) -> first bucket */
    if (t > (double)(n - 1)) return n - 1;
    return (int64_t)t;
}

void or_hash(const og_t *g, int64_t n, const double *x, uint32_t *hash)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_of(x[3 * i + 0], g->o[0], g->L, g->n[0]);
        int64_t cy = cell_of(x[3 * i + 1], g->o[1], g->L, g->n[1]);
        int64_t cz = cell_of(x[3 * i + 2], g->o[2], g->L, g->n[2]);
        hash[i] = (uint32_t)(cx + (int64_t)g->n[0] * (cy + (int64_t)g->n[1] * cz));
    }
}

/* Stable counting sort: perm[k] = index (in the current order) of the k-th
 * particle in ascending key order, ties in current order. */
int or_sort_perm(int64_t n, const uint32_t *key, uint32_t nkeys, uint32_t *perm)
{
    int64_t *pos = (int64_t *)calloc((size_t)nkeys + 1, sizeof(int64_t));
    if (!pos) return -1;
    for (int64_t i = 0; i < n; ++i) pos[key[i] + 1]++;
    for (uint32_t k = 0; k < nkeys; ++k) pos[k + 1] += pos[k];
    for (int64_t i = 0; i < n; ++i) perm[pos[key[i]]++] = (uint32_t)i;
    free(pos);
    return 0;
}

/* start[c] for c in [0, ncells]: number of sorted keys below c. */
int or_cell_start(int64_t n, const uint32_t *sorted_key, uint32_t ncells, uint32_t *start)
{
    int64_t *cnt = (int64_t *)calloc((size_t)ncells + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int64_t k = 0; k < n; ++k) cnt[sorted_key[k]]++;
    int64_t run = 0;
    for (uint32_t c = 0; c <= ncells; ++c) {
        start[c] = (uint32_t)run;
        if (c < ncells) run += cnt[c];
    }
    free(cnt);
    return 0;
}

static void gather3(double *dst, const double *src, const uint32_t *perm, int64_t n, int k)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < k; ++a) dst[(int64_t)k * i + a] = src[(int64_t)k * perm[i] + a];
}

/* dst[k] = src[perm[k]] for every field present in src (dst must match). */
void or_gather(os_t *dst, const os_t *src, const uint32_t *perm)
{
    int64_t n = src->n;
    gather3(dst->x, src->x, perm, n, 3);
    gather3(dst->v, src->v, perm, n, 3);
    gather3(dst->m, src->m, perm, n, 1);
    gather3(dst->w, src->w, perm, n, 1);
    gather3(dst->rho, src->rho, perm, n, 1);
    gather3(dst->p, src->p, perm, n, 1);
    gather3(dst->c, src->c, perm, n, 1);
    gather3(dst->E, src->E, perm, n, 1);
    if (src->S) gather3(dst->S, src->S, perm, n, 6);
    if (src->ep) gather3(dst->ep, src->ep, perm, n, 1);
    for (int64_t i = 0; i < n; ++i) dst->id[i] = src->id[perm[i]];
    if (src->hash && dst->hash)
        for (int64_t i = 0; i < n; ++i) dst->hash[i] = src->hash[perm[i]];
}

static void decode(const og_t *g, uint32_t h, int64_t c[3])
{
    c[0] = h % (uint32_t)g->n[0];
    c[1] = (h / (uint32_t)g->n[0]) % (uint32_t)g->n[1];
    c[2] = h / ((uint32_t)g->n[0] * (uint32_t)g->n[1]);
}

/* ----------------------------------------------- communication hash (step c) */

void or_mark(const og_t *g, int64_t n, const uint32_t *hash, const uint32_t *rstart,
             uint32_t *comm, uint32_t *bidx, uint32_t *nb)
{
    uint32_t G = (uint32_t)((int64_t)g->n[0] * g->n[1] * g->n[2]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        decode(g, hash[i], c);
        int flag = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t a = c[0] + dx, b = c[1] + dy, e = c[2] + dz;
                    if (a < 0 || b < 0 || e < 0 || a >= g->n[0] || b >= g->n[1] || e >= g->n[2])
                        continue;
                    uint32_t q = (uint32_t)(a + (int64_t)g->n[0] * (b + (int64_t)g->n[1] * e));
                    if (rstart[q + 1] > rstart[q]) flag = 1;
                }
        comm[i] = flag ? hash[i] : G;
    }
    uint32_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (comm[i] != G) bidx[k++] = (uint32_t)i;
    *nb = k;
}

/* --------------------------------------------------------------- kernel */

/* Cubic spline (M4) in 3D, sigma = 1 / (pi h^3), support 2h. */
double or_kernel_W(double r, double h)
{
    double q = r / h, s = 1.0 / (M_PI * h * h * h);
    if (q < 1.0) return s * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
    if (q < 2.0) {
        double t = 2.0 - q;
        return s * 0.25 * t * t * t;
    }
    return 0.0;
}

/* F = -dW/dr >= 0, so that grad_i W_ij = F n with n = (x_j - x_i) / r. */
double or_kernel_F(double r, double h)
{
    double q = r / h, s = 1.0 / (M_PI * h * h * h);
    if (q < 1.0) return s * (3.0 * q - 2.25 * q * q) / h;
    if (q < 2.0) {
        double t = 2.0 - q;
        return s * 0.75 * t * t / h;
    }
    return 0.0;
}

/* --------------------------------------------------------------- EOS */

/* Mie-Gruneisen (Section IV.A names it, with a cut-off pressure for
 * spalling; the paper gives no formula).  Reference curve: the shock
 * Hugoniot of a linear shock-velocity law Us = c0 + s up, which in
 * mu = rho / rho0 - 1 reads pH = rho0 c0^2 mu (1 + mu) / (1 - (s - 1) mu)^2
 * with specific energy eH = pH mu / (2 rho0 (1 + mu)); off the Hugoniot
 * p = pH + Gamma0 rho0 (e - eH) (Gamma rho held at Gamma0 rho0), which
 * simplifies to the form below.  In tension the linear branch rho0 c0^2 mu.
 * The pole of the Hugoniot is kept away by D >= 1/16.  Sound speed:
 * cb^2 = dp/drho at fixed e + (p / rho^2) dp/de, with dp/de = Gamma0 rho0,
 * the thermal part taken on max(p, 0); the longitudinal speed adds 4G/(3 rho). */
static void eos_mie_gruneisen(const op_t *P, double rho, double e, double *p, double *c)
{
    double mu = rho / P->rho0 - 1.0;
    double dpde = P->mg_gamma0 * P->rho0;
    double pu, dpdrho;
    if (mu > 0.0) {
        double b = P->mg_s - 1.0;
        double D = 1.0 - b * mu;
        if (D < 0.0625) D = 0.0625;
        double a = 1.0 - 0.5 * P->mg_gamma0;
        /* f(mu) = mu (1 + a mu) / D^2, f'(mu) = (1 + (2a + b) mu) / D^3 */
        pu = P->rho0 * P->c0 * P->c0 * (mu * (1.0 + a * mu) / (D * D)) + dpde * e;
        dpdrho = P->c0 * P->c0 * ((1.0 + (2.0 * a + b) * mu) / (D * D * D));
    } else {
        pu = P->rho0 * P->c0 * P->c0 * mu + dpde * e;
        dpdrho = P->c0 * P->c0;
    }
    double cb2 = dpdrho + (pu > 0.0 ? pu : 0.0) * dpde / (rho * rho);
    *p = pu > P->p_cut ? pu : P->p_cut;
    *c = sqrt(cb2 + 4.0 * P->G / (3.0 * rho));
}

static void eos(const op_t *P, double rho, double e, double *p, double *c)
{
    if (P->material == 0) {
        double B = P->rho0 * P->c0 * P->c0 / P->gamma;
        double s = rho / P->rho0;
        *p = B * (pow(s, P->gamma) - 1.0);
        *c = P->c0 * pow(s, 0.5 * (P->gamma - 1.0));
    } else if (P->eos == 1) {
        eos_mie_gruneisen(P, rho, e, p, c);
    } else {
        *p = P->K * (rho / P->rho0 - 1.0);
        *c = sqrt((P->K + 4.0 * P->G / 3.0) / P->rho0);
    }
}

void or_eos(const op_t *P, double rho, double e, double *p, double *c) { eos(P, rho, e, p, c); }

/* ---------------------------------------------------------- pair terms */

/* Symmetric 3x3 from (xx yy zz xy xz yz). */
static void sym_full(const double *s, double M[3][3])
{
    M[0][0] = s[0]; M[1][1] = s[1]; M[2][2] = s[2];
    M[0][1] = M[1][0] = s[3];
    M[0][2] = M[2][0] = s[4];
    M[1][2] = M[2][1] = s[5];
}

/*
 * FORCE terms of target i from source j.  d = x_j - x_i, r = |d| > 0.
 * Linearised (acoustic) Riemann problem along n between left state i and
 * right state j with equal impedance Z = mean(rho) * mean(c):
 *   u* - ubar = beta (P_i - P_j) / (2 Z),  p* = mean(p) + beta Z (u_i - u_j) / 2,
 * v* = mean(v) + (u* - ubar) n, E* = mean(e) + |v*|^2 / 2, A = 2 w_i w_j,
 * Phi = mean(rho) (u* - ubar) F.  Then
 *   mdot  = -A Phi
 *   mvdot = -A (Phi v* + Pi g),          Pi g = p* g - mean(S) g
 *   mEdot = -A (Phi E* + (Pi g) . v*)
 *   wdot  = w_i w_j (v_j - v_i) . g
 * Solids use P = p - n.S.n for the normal stress in u*.
 * out: mdot, mvdot[3], mEdot, wdot.
 */
void or_pair(const op_t *P, const double d[3], const double vi[3], const double vj[3],
             double wi, double wj, double rhoi, double rhoj, double pi_, double pj,
             double ci, double cj, double ei, double ej, const double *Si, const double *Sj,
             double out[6])
{
    double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    double F = or_kernel_F(r, P->h);
    double n[3] = {d[0] / r, d[1] / r, d[2] / r};
    double g[3] = {F * n[0], F * n[1], F * n[2]};
    double ui = (vi[0] * n[0] + vi[1] * n[1]) + vi[2] * n[2];
    double uj = (vj[0] * n[0] + vj[1] * n[1]) + vj[2] * n[2];
    double rb = 0.5 * (rhoi + rhoj), cb = 0.5 * (ci + cj), pb = 0.5 * (pi_ + pj);
    double Z = rb * cb;
    double Pi = pi_, Pj = pj;
    double Snbar[3] = {0.0, 0.0, 0.0};
    if (Si && Sj) {
        double A[3][3], B[3][3];
        sym_full(Si, A);
        sym_full(Sj, B);
        double ai[3], bj[3];
        for (int a = 0; a < 3; ++a) {
            ai[a] = (A[a][0] * n[0] + A[a][1] * n[1]) + A[a][2] * n[2];
            bj[a] = (B[a][0] * n[0] + B[a][1] * n[1]) + B[a][2] * n[2];
        }
        Pi = pi_ - ((n[0] * ai[0] + n[1] * ai[1]) + n[2] * ai[2]);
        Pj = pj - ((n[0] * bj[0] + n[1] * bj[1]) + n[2] * bj[2]);
        for (int a = 0; a < 3; ++a) Snbar[a] = 0.5 * (ai[a] + bj[a]);
    }
    double du = P->beta * (Pi - Pj) / (2.0 * Z);
    double ps = pb + P->beta * Z * (ui - uj) * 0.5;
    double vs[3];
    for (int a = 0; a < 3; ++a) vs[a] = 0.5 * (vi[a] + vj[a]) + du * n[a];
    double Es = 0.5 * (ei + ej) + 0.5 * ((vs[0] * vs[0] + vs[1] * vs[1]) + vs[2] * vs[2]);
    double A = 2.0 * wi * wj;
    double Phi = rb * du * F;
    double t[3];
    for (int a = 0; a < 3; ++a) t[a] = ps * g[a] - F * Snbar[a];
    out[0] = -A * Phi;
    for (int a = 0; a < 3; ++a) out[1 + a] = -A * (Phi * vs[a] + t[a]);
    out[4] = -A * (Phi * Es + ((t[0] * vs[0] + t[1] * vs[1]) + t[2] * vs[2]));
    double dv[3] = {vj[0] - vi[0], vj[1] - vi[1], vj[2] - vi[2]};
    out[5] = wi * wj * ((dv[0] * g[0] + dv[1] * g[1]) + dv[2] * g[2]);
}

/* GRADIENT term: L_ab += w_j (v_j - v_i)_a g_b. */
void or_pair_grad(const op_t *P, const double d[3], const double vi[3], const double vj[3],
                  double wj, double out[9])
{
    double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    double F = or_kernel_F(r, P->h);
    double g[3] = {F * (d[0] / r), F * (d[1] / r), F * (d[2] / r)};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) out[3 * a + b] = wj * (vj[a] - vi[a]) * g[b];
}

/* ------------------------------------------------- round-off magnitude bounds */

/* Sum of |entries| of a symmetric stress (off-diagonals twice): bounds |S n|_k. */
static double sym_abs(const double *s)
{
    return (fabs(s[0]) + fabs(s[1]) + fabs(s[2])) + 2.0 * (fabs(s[3]) + fabs(s[4]) + fabs(s[5]));
}

/* The FORCE terms evaluated on magnitudes: every input replaced by its
 * absolute value, every difference by a sum, and every component of n by 1.
 * Standard forward-error analysis bounds the rounding error of an evaluation
 * of or_pair by (operation count) * (unit round-off) * this value, and a
 * perturbation of the direction n or of the velocities by the same relative
 * amount; it cannot vanish through cancellation the way the terms can. */
static void pair_bound(const op_t *P, double r, const double vi[3], const double vj[3], double wi,
                       double wj, double rhoi, double rhoj, double pi_, double pj, double ci,
                       double cj, double ei, double ej, const double *Si, const double *Sj,
                       double out[6])
{
    double F = or_kernel_F(r, P->h);
    double ui = fabs(vi[0]) + fabs(vi[1]) + fabs(vi[2]);
    double uj = fabs(vj[0]) + fabs(vj[1]) + fabs(vj[2]);
    double rb = 0.5 * (rhoi + rhoj), cb = 0.5 * (ci + cj);
    double Z = rb * cb;
    double si = Si ? sym_abs(Si) : 0.0, sj = Sj ? sym_abs(Sj) : 0.0;
    double du = fabs(P->beta) * ((fabs(pi_) + si) + (fabs(pj) + sj)) / (2.0 * Z);
    double ps = 0.5 * (fabs(pi_) + fabs(pj)) + fabs(P->beta) * Z * (ui + uj) * 0.5;
    double vs[3];
    for (int a = 0; a < 3; ++a) vs[a] = 0.5 * (fabs(vi[a]) + fabs(vj[a])) + du;
    double Es = 0.5 * (fabs(ei) + fabs(ej)) + 0.5 * ((vs[0] * vs[0] + vs[1] * vs[1]) + vs[2] * vs[2]);
    double A = 2.0 * fabs(wi) * fabs(wj);
    double Phi = rb * du * F;
    double t = ps * F + F * 0.5 * (si + sj);
    out[0] = A * Phi;
    for (int a = 0; a < 3; ++a) out[1 + a] = A * (Phi * vs[a] + t);
    out[4] = A * (Phi * Es + t * ((vs[0] + vs[1]) + vs[2]));
    out[5] = fabs(wi) * fabs(wj) * F * ((fabs(vj[0]) + fabs(vi[0])) + (fabs(vj[1]) + fabs(vi[1])) +
                                        (fabs(vj[2]) + fabs(vi[2])));
}

static void pair_grad_bound(const op_t *P, double r, const double vi[3], const double vj[3], double wj,
                            double out[9])
{
    double F = or_kernel_F(r, P->h);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) out[3 * a + b] = fabs(wj) * (fabs(vj[a]) + fabs(vi[a])) * F;
}

/* F_max / F(r): rescales a pair term to the kernel's peak strength
 * (F peaks at q = 2/3 with F_max = 1 / (pi h^4)). */
static double peak_factor(double h, double r2)
{
    double Fmax = 1.0 / (M_PI * h * h * h) / h;
    return Fmax / or_kernel_F(sqrt(r2), h);
}

/* -------------------------------------------------------- interaction pass */

/*
 * Accumulate into rates (n_tgt_all*6) or L (n_tgt_all*9) for targets
 * tidx[t] (all targets when tidx == NULL) from sources sorted by hash with
 * cell table sstart.  self != 0: sources are the targets, j == i is skipped.
 * pass 0 = FORCE, 1 = GRADIENT.
 */
static void interact_impl(const op_t *P, const og_t *g, int pass, const os_t *tg,
                          const uint32_t *tidx, int64_t nt, const os_t *sr, const uint32_t *sstart,
                          int self, double *rates, double *L, int absval)
{
    double R = 2.0 * P->h;
    double R2 = R * R;
    int solid = (P->material == 1);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tidx ? (int64_t)tidx[t] : t;
        int64_t c[3];
        decode(g, tg->hash[i], c);
        const double *xi = tg->x + 3 * i, *vi = tg->v + 3 * i;
        double ei = tg->E[i] - 0.5 * ((vi[0] * vi[0] + vi[1] * vi[1]) + vi[2] * vi[2]);
        double acc[9] = {0.0};
        if (pass == 0)
            for (int a = 0; a < 6; ++a) acc[a] = rates[6 * i + a];
        else
            for (int a = 0; a < 9; ++a) acc[a] = L[9 * i + a];
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t a = c[0] + dx, b = c[1] + dy, e = c[2] + dz;
                    if (a < 0 || b < 0 || e < 0 || a >= g->n[0] || b >= g->n[1] || e >= g->n[2])
                        continue;
                    uint32_t q = (uint32_t)(a + (int64_t)g->n[0] * (b + (int64_t)g->n[1] * e));
                    for (uint32_t j = sstart[q]; j < sstart[q + 1]; ++j) {
                        if (self && (int64_t)j == i) continue;
                        const double *xj = sr->x + 3 * (int64_t)j;
                        double d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
                        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                        if (!(r2 < R2) || r2 == 0.0) continue;   /* coincident: no direction, F(0) = 0 */
                        const double *vj = sr->v + 3 * (int64_t)j;
                        if (pass == 0) {
                            double ej = sr->E[j] - 0.5 * ((vj[0] * vj[0] + vj[1] * vj[1]) + vj[2] * vj[2]);
                            double o[6];
                            const double *Si = solid ? tg->S + 6 * i : NULL;
                            const double *Sj = solid ? sr->S + 6 * (int64_t)j : NULL;
                            if (absval)
                                pair_bound(P, sqrt(r2), vi, vj, tg->w[i], sr->w[j], tg->rho[i], sr->rho[j],
                                           tg->p[i], sr->p[j], tg->c[i], sr->c[j], ei, ej, Si, Sj, o);
                            else
                                or_pair(P, d, vi, vj, tg->w[i], sr->w[j], tg->rho[i], sr->rho[j], tg->p[i],
                                        sr->p[j], tg->c[i], sr->c[j], ei, ej, Si, Sj, o);
                            double f = absval == 2 ? peak_factor(P->h, r2) : 1.0;
                            for (int k = 0; k < 6; ++k) acc[k] += o[k] * f;
                        } else {
                            double o[9];
                            if (absval)
                                pair_grad_bound(P, sqrt(r2), vi, vj, sr->w[j], o);
                            else
                                or_pair_grad(P, d, vi, vj, sr->w[j], o);
                            double f = absval == 2 ? peak_factor(P->h, r2) : 1.0;
                            for (int k = 0; k < 9; ++k) acc[k] += o[k] * f;
                        }
                    }
                }
        if (pass == 0)
            for (int a = 0; a < 6; ++a) rates[6 * i + a] = acc[a];
        else
            for (int a = 0; a < 9; ++a) L[9 * i + a] = acc[a];
    }
}

void or_interact(const op_t *P, const og_t *g, int pass, const os_t *tg, const uint32_t *tidx,
                 int64_t nt, const os_t *sr, const uint32_t *sstart, int self, double *rates,
                 double *L)
{
    interact_impl(P, g, pass, tg, tidx, nt, sr, sstart, self, rates, L, 0);
}

/* Per-target sums of the magnitude bounds (pair_bound): the scale against
 * which round-off in a pair sum is measured. */
void or_interact_abs(const op_t *P, const og_t *g, int pass, const os_t *tg, const uint32_t *tidx,
                     int64_t nt, const os_t *sr, const uint32_t *sstart, int self, double *rates,
                     double *L)
{
    interact_impl(P, g, pass, tg, tidx, nt, sr, sstart, self, rates, L, 1);
}

/* The same bounds with every pair at the kernel's peak strength (F_max / F).
 * Near the support edge F ~ (2 - q)^2 amplifies any rounding of q or r
 * relative to the (vanishing) term itself; this scale bounds that. */
void or_interact_peak(const op_t *P, const og_t *g, int pass, const os_t *tg, const uint32_t *tidx,
                      int64_t nt, const os_t *sr, const uint32_t *sstart, int self, double *rates,
                      double *L)
{
    interact_impl(P, g, pass, tg, tidx, nt, sr, sstart, self, rates, L, 2);
}

/* Every ordered pair (i, j) the FORCE pass visits with r < 2h; returns the
 * count, writing at most cap pairs. */
int64_t or_neighbors(const op_t *P, const og_t *g, const os_t *tg, const os_t *sr,
                     const uint32_t *sstart, int self, uint32_t *pi_out, uint32_t *pj_out,
                     int64_t cap)
{
    double R = 2.0 * P->h;
    double R2 = R * R;
    int64_t k = 0;
    for (int64_t i = 0; i < tg->n; ++i) {
        int64_t c[3];
        decode(g, tg->hash[i], c);
        const double *xi = tg->x + 3 * i;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t a = c[0] + dx, b = c[1] + dy, e = c[2] + dz;
                    if (a < 0 || b < 0 || e < 0 || a >= g->n[0] || b >= g->n[1] || e >= g->n[2])
                        continue;
                    uint32_t q = (uint32_t)(a + (int64_t)g->n[0] * (b + (int64_t)g->n[1] * e));
                    for (uint32_t j = sstart[q]; j < sstart[q + 1]; ++j) {
                        if (self && (int64_t)j == i) continue;
                        const double *xj = sr->x + 3 * (int64_t)j;
                        double d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
                        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                        if (!(r2 < R2) || r2 == 0.0) continue;   /* coincident: no direction, F(0) = 0 */
                        if (k < cap) {
                            pi_out[k] = (uint32_t)i;
                            pj_out[k] = j;
                        }
                        ++k;
                    }
                }
    }
    return k;
}

/* ------------------------------------------------------------- integrate */

enum { OR_MOTION = 0, OR_STRESS = 1, OR_EOS = 2 };

static void finish_particle(const op_t *P, const os_t *s, int64_t i)
{
    const double *v = s->v + 3 * i;
    s->rho[i] = s->m[i] / s->w[i];
    eos(P, s->rho[i], s->E[i] - 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]), &s->p[i], &s->c[i]);
}

/* diag: [0] dt_next = cfl h / max(c + |v|), [1] sum m, [2..4] sum m v,
 * [5] sum m E, [6] sum m |v|^2 / 2.  Sums run in index order. */
static void diagnostics(const op_t *P, const os_t *s, double *diag)
{
    double vmax = 0.0, M = 0.0, px = 0.0, py = 0.0, pz = 0.0, Et = 0.0, KE = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
        const double *v = s->v + 3 * i;
        double v2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
        double sp = s->c[i] + sqrt(v2);
        if (sp > vmax) vmax = sp;
        M += s->m[i];
        px += s->m[i] * v[0];
        py += s->m[i] * v[1];
        pz += s->m[i] * v[2];
        Et += s->m[i] * s->E[i];
        KE += 0.5 * s->m[i] * v2;
    }
    diag[0] = vmax > 0.0 ? P->cfl * P->h / vmax : INFINITY;
    diag[1] = M;
    diag[2] = px;
    diag[3] = py;
    diag[4] = pz;
    diag[5] = Et;
    diag[6] = KE;
}

void or_integrate(const op_t *P, int stage, os_t *s, const double *rates, const double *L,
                  double dt, double *diag)
{
    int64_t n = s->n;
    if (stage == OR_MOTION) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double *r = rates + 6 * i;
            double *v = s->v + 3 * i, *x = s->x + 3 * i;
            double m = s->m[i];
            double mn = m + dt * r[0];
            double vn[3];
            double gv = (P->g[0] * v[0] + P->g[1] * v[1]) + P->g[2] * v[2];
            for (int a = 0; a < 3; ++a) vn[a] = (m * v[a] + dt * (r[1 + a] + m * P->g[a])) / mn;
            double En = (m * s->E[i] + dt * (r[4] + m * gv)) / mn;
            s->w[i] = s->w[i] + dt * r[5];
            s->m[i] = mn;
            s->E[i] = En;
            for (int a = 0; a < 3; ++a) {
                double xn = x[a] + dt * vn[a];
                if ((P->wall_mask >> (2 * a)) & 1)
                    if (xn < P->wlo[a]) {
                        xn = 2.0 * P->wlo[a] - xn;
                        vn[a] = -vn[a];
                    }
                if ((P->wall_mask >> (2 * a + 1)) & 1)
                    if (xn > P->whi[a]) {
                        xn = 2.0 * P->whi[a] - xn;
                        vn[a] = -vn[a];
                    }
                x[a] = xn;
                v[a] = vn[a];
            }
            finish_particle(P, s, i);
        }
    } else if (stage == OR_STRESS) {
        double G = P->G;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double *l = L + 9 * i;
            double D[3][3], W[3][3], S[3][3], Sd[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    D[a][b] = 0.5 * (l[3 * a + b] + l[3 * b + a]);
                    W[a][b] = 0.5 * (l[3 * a + b] - l[3 * b + a]);
                }
            sym_full(s->S + 6 * i, S);
            double tr = (D[0][0] + D[1][1]) + D[2][2];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double ws = 0.0, sw = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        ws += W[a][k] * S[k][b];
                        sw += S[a][k] * W[k][b];
                    }
                    Sd[a][b] = 2.0 * G * (D[a][b] - (a == b ? tr / 3.0 : 0.0)) + ws - sw;
                }
            double St[6] = {S[0][0] + dt * Sd[0][0], S[1][1] + dt * Sd[1][1], S[2][2] + dt * Sd[2][2],
                            S[0][1] + dt * Sd[0][1], S[0][2] + dt * Sd[0][2], S[1][2] + dt * Sd[1][2]};
            double J = (St[0] * St[0] + St[1] * St[1]) + St[2] * St[2];
            J += 2.0 * ((St[3] * St[3] + St[4] * St[4]) + St[5] * St[5]);
            double q = sqrt(1.5 * J);
            double sy = P->Y0 + P->H * s->ep[i];
            if (q > sy) {
                double dep = (q - sy) / (3.0 * G + P->H);
                double f = 1.0 - 3.0 * G * dep / q;
                for (int k = 0; k < 6; ++k) St[k] *= f;
                s->ep[i] += dep;
            }
            for (int k = 0; k < 6; ++k) s->S[6 * i + k] = St[k];
        }
        diag[0] = dt;
        return;
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) finish_particle(P, s, i);
    }
    diagnostics(P, s, diag);
}

/* ----------------------------------------------------------- whole steps */

typedef struct {
    uint32_t *hash, *perm, *start;
    os_t tmp;
    double *rates, *L;
} owork_t;

static int alloc_state(os_t *s, int64_t n, int solid)
{
    memset(s, 0, sizeof(*s));
    s->n = n;
    s->x = malloc(sizeof(double) * 3 * n);
    s->v = malloc(sizeof(double) * 3 * n);
    s->m = malloc(sizeof(double) * n);
    s->w = malloc(sizeof(double) * n);
    s->rho = malloc(sizeof(double) * n);
    s->p = malloc(sizeof(double) * n);
    s->c = malloc(sizeof(double) * n);
    s->E = malloc(sizeof(double) * n);
    s->id = malloc(sizeof(uint32_t) * n);
    s->hash = malloc(sizeof(uint32_t) * n);
    if (solid) {
        s->S = malloc(sizeof(double) * 6 * n);
        s->ep = malloc(sizeof(double) * n);
    }
    return (s->x && s->v && s->m && s->w && s->rho && s->p && s->c && s->E && s->id && s->hash) ? 0 : -1;
}

static void free_state(os_t *s)
{
    free(s->x); free(s->v); free(s->m); free(s->w); free(s->rho); free(s->p); free(s->c);
    free(s->E); free(s->id); free(s->hash); free(s->S); free(s->ep);
}

static void copy_state(os_t *dst, const os_t *src)
{
    int64_t n = src->n;
    memcpy(dst->x, src->x, sizeof(double) * 3 * n);
    memcpy(dst->v, src->v, sizeof(double) * 3 * n);
    memcpy(dst->m, src->m, sizeof(double) * n);
    memcpy(dst->w, src->w, sizeof(double) * n);
    memcpy(dst->rho, src->rho, sizeof(double) * n);
    memcpy(dst->p, src->p, sizeof(double) * n);
    memcpy(dst->c, src->c, sizeof(double) * n);
    memcpy(dst->E, src->E, sizeof(double) * n);
    memcpy(dst->id, src->id, sizeof(uint32_t) * n);
    if (src->S) memcpy(dst->S, src->S, sizeof(double) * 6 * n);
    if (src->ep) memcpy(dst->ep, src->ep, sizeof(double) * n);
}

/*
 * Run nsteps whole steps on s (reordered in place into the last step's
 * sorted order).  dts: if fixed_dt > 0 every step uses it; otherwise the
 * first step uses the EOS-stage dt and each later one the previous step's
 * dt_next.  If dts_in != NULL, step k uses dts_in[k] (replayed schedule).
 * dts_out[k] receives the dt used by step k.  diag_out (7 doubles) gets the
 * last step's diagnostics.
 */
int or_run(const op_t *P, const og_t *g, os_t *s, int nsteps, double fixed_dt,
           const double *dts_in, double *dts_out, double *diag_out)
{
    int64_t n = s->n;
    int solid = (P->material == 1);
    uint32_t ncells = (uint32_t)((int64_t)g->n[0] * g->n[1] * g->n[2]);
    owork_t w;
    if (alloc_state(&w.tmp, n, solid)) return -1;
    w.perm = malloc(sizeof(uint32_t) * n);
    w.start = malloc(sizeof(uint32_t) * ((size_t)ncells + 1));
    w.rates = malloc(sizeof(double) * 6 * n);
    w.L = malloc(sizeof(double) * 9 * n);
    double diag[7];
    or_integrate(P, OR_EOS, s, NULL, NULL, 0.0, diag);
    double dt = diag[0];
    for (int k = 0; k < nsteps; ++k) {
        if (fixed_dt > 0.0) dt = fixed_dt;
        if (dts_in) dt = dts_in[k];
        if (dts_out) dts_out[k] = dt;
        or_hash(g, n, s->x, s->hash);
        or_sort_perm(n, s->hash, ncells, w.perm);
        or_gather(&w.tmp, s, w.perm);
        copy_state(s, &w.tmp);
        memcpy(s->hash, w.tmp.hash, sizeof(uint32_t) * n);
        or_cell_start(n, s->hash, ncells, w.start);
        if (solid) {
            memset(w.L, 0, sizeof(double) * 9 * n);
            or_interact(P, g, 1, s, NULL, n, s, w.start, 1, NULL, w.L);
            or_integrate(P, OR_STRESS, s, NULL, w.L, dt, diag);
        }
        memset(w.rates, 0, sizeof(double) * 6 * n);
        or_interact(P, g, 0, s, NULL, n, s, w.start, 1, w.rates, NULL);
        or_integrate(P, OR_MOTION, s, w.rates, NULL, dt, diag);
        dt = diag[0];
    }
    if (diag_out) memcpy(diag_out, diag, sizeof(diag));
    free_state(&w.tmp);
    free(w.perm); free(w.start); free(w.rates); free(w.L);
    return 0;
}

/* ------------------------------------------------------------- balancing
 * Periodic swap heuristic between two GPUs A and B (Section III.A), the part
 * one GPU computes.  Readings (the paper states them in words only):
 *   centre of gravity  Cg = sum m_i x_i / sum m_i (mass-weighted), summed in
 *                      index order;
 *   balancing hash     with e = Cg_B - Cg_A and M = (Cg_A + Cg_B) / 2, the
 *                      projection past the midpoint towards B is
 *                      s = (x - M).e / |e|; hash 0 when s <= 0 (own side),
 *                      hmax when s >= |e| / 2 (at or beyond the other Cg),
 *                      else ceil(hmax s / (|e| / 2)).  Evaluated without a
 *                      square root as v = hmax (2 t / |e|^2), t = (x - M).e,
 *                      in this operation order:
 *                        t = ((x0 - M0) e0 + (x1 - M1) e1) + (x2 - M2) e2
 *                        ee = (e0 e0 + e1 e1) + e2 e2
 *                        v = hmax * ((t + t) / ee)
 *                        hash = t > 0 ? (v >= hmax ? hmax : ceil(v)) : 0
 *                      and 0 for every particle when ee = 0;
 *   swap count         k = min(number with positive hash on A, on B);
 *   selection          the k particles of largest hash, ties in ascending
 *                      index (a stable sort by descending hash);
 *   swap               the selected particles of A and of B exchange places,
 *                      pairwise in selection order (every field), so both
 *                      GPUs keep their particle counts.
 */
void or_centroid(const os_t *s, double cg[4])
{
    double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
        const double m = s->m[i];
        sx += m * s->x[3 * i + 0];
        sy += m * s->x[3 * i + 1];
        sz += m * s->x[3 * i + 2];
        sm += m;
    }
    cg[0] = sm > 0.0 ? sx / sm : 0.0;
    cg[1] = sm > 0.0 ? sy / sm : 0.0;
    cg[2] = sm > 0.0 ? sz / sm : 0.0;
    cg[3] = sm;
}

int64_t or_balance_hash(const os_t *s, const double cg_own[3], const double cg_other[3], uint32_t hmax,
                        uint32_t *bhash)
{
    double e[3], M[3];
    for (int d = 0; d < 3; ++d) {
        e[d] = cg_other[d] - cg_own[d];
        M[d] = 0.5 * (cg_own[d] + cg_other[d]);
    }
    const double ee = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
    int64_t npos = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        uint32_t h = 0;
        if (ee > 0.0) {
            const double *x = s->x + 3 * i;
            const double t = ((x[0] - M[0]) * e[0] + (x[1] - M[1]) * e[1]) + (x[2] - M[2]) * e[2];
            if (t > 0.0) {
                const double v = (double)hmax * ((t + t) / ee);
                h = v >= (double)hmax ? hmax : (uint32_t)ceil(v);
            }
        }
        bhash[i] = h;
        npos += h > 0;
    }
    return npos;
}

/* Indices of the k particles of largest balancing hash, ties in ascending
 * index: a stable counting sort by hmax - hash, first k entries. */
int or_balance_select(int64_t n, const uint32_t *bhash, uint32_t hmax, int64_t k, uint32_t *sel)
{
    uint32_t *key = calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    uint32_t *perm = calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    if (!key || !perm) {
        free(key);
        free(perm);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) key[i] = hmax - (bhash[i] < hmax ? bhash[i] : hmax);
    or_sort_perm(n, key, hmax + 1, perm);
    for (int64_t t = 0; t < k && t < n; ++t) sel[t] = perm[t];
    free(key);
    free(perm);
    return 0;
}

static void swap_d(double *a, double *b, int k)
{
    for (int q = 0; q < k; ++q) {
        const double t = a[q];
        a[q] = b[q];
        b[q] = t;
    }
}

void or_swap(os_t *a, const uint32_t *sel_a, os_t *b, const uint32_t *sel_b, int64_t k)
{
    for (int64_t t = 0; t < k; ++t) {
        const int64_t i = sel_a[t], j = sel_b[t];
        swap_d(a->x + 3 * i, b->x + 3 * j, 3);
        swap_d(a->v + 3 * i, b->v + 3 * j, 3);
        swap_d(a->m + i, b->m + j, 1);
        swap_d(a->w + i, b->w + j, 1);
        swap_d(a->rho + i, b->rho + j, 1);
        swap_d(a->p + i, b->p + j, 1);
        swap_d(a->c + i, b->c + j, 1);
        swap_d(a->E + i, b->E + j, 1);
        if (a->S && b->S) swap_d(a->S + 6 * i, b->S + 6 * j, 6);
        if (a->ep && b->ep) swap_d(a->ep + i, b->ep + j, 1);
        const uint32_t id = a->id[i];
        a->id[i] = b->id[j];
        b->id[j] = id;
        const uint32_t hh = a->hash[i];
        a->hash[i] = b->hash[j];
        b->hash[j] = hh;
    }
}
