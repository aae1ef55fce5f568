/*
 * Plain CPU oracle for the volumetric-ray-casting (VRC) fluence estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline timing of the benchmark may load it; the
 * library itself never calls it, and the two share no code.
 *
 * It follows the method's definition step by step, in double precision:
 *
 *  1. Total cross section of every material at the ray energy (Sec. 3: the
 *     cross sections of all materials are found first, by table lookup and
 *     linear interpolation between table points).  Here: binary search for
 *     the bracketing interval, lin-lin interpolation, end values held
 *     outside the table.  Optionally a material is a mixture of tabulated
 *     components, Sigma_m(E) = sum_j f_j Sigma_j(E), each component looked
 *     up on its own table and the terms added in component order; and
 *     optionally every voxel carries a density factor, the cell's
 *     Sigma_t,i(E) of Eqs. 1-4 then being rho_i * Sigma_m(E).
 *  2. Trace the ray through the mesh (Sec. 3; trav.inc for a Cartesian
 *     mesh, trav_rz.inc for an R-Z one, Sec. 6.3): the cells crossed, in
 *     order, with the length in each.
 *  3. Score every crossed voxel i by the VRC estimator (Eq. 4, i.e. the
 *     expected-value estimator of Eq. 1 with the entering weight of Eq. 2):
 *        W_i = w * exp(-tau_in)                       (Eq. 2)
 *        F_i = W_i * (1 - exp(-Sigma_i * l_i)) / Sigma_i   (Eq. 1 / Eq. 3)
 *     with 1 - exp(-x) evaluated as -expm1(-x), F_i = W_i * l_i when
 *     Sigma_i = 0 (the limit), and tau_in advanced by Sigma_i * l_i after
 *     the voxel (a compensated sum: a plain one drifts by about n ulp of
 *     tau over n segments, more than 1e-12 on rays of 10^5 segments).  The
 *     ray weight w already carries the 1/N of Eq. 4.
 *  4. Accumulate F_i into the tally of the ray's energy bin with a
 *     compensated (Neumaier) sum, and keep, per voxel, the sum of squares and
 *     the number of rays that scored (for the relative standard error that
 *     decides which voxels a tolerance applies to; Sec. 5 compares only cells
 *     below 5% uncertainty).
 *
 * Pins (tests/test_oracle_pins.py): the lookup against numpy.interp; the
 * traversal against exact rational arithmetic and hand cases; the scores
 * against the homogeneous telescoping sum, the void limit, the collision
 * form, an axis-aligned closed form and fine-step path integration; the
 * tally against exactly rounded sums; the estimator's mean against cubature
 * of a point source and against the track-length estimator of an analog
 * walk.  Density factors and mixtures (tests/test_oracle_density.py): unit
 * factors and one-component mixtures against the plain tallies, density
 * levels against scaled tables, closed forms on homogeneous and two-region
 * meshes, zero density against a void material, mixtures against summed
 * tables and against numpy's interpolation.  No function here is left
 * unpinned.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define REAL double
#define TRAV_NAME(x) x##_f64
#include "trav.inc"
#undef REAL
#undef TRAV_NAME

#define REAL float
#define TRAV_NAME(x) x##_f32
#include "trav.inc"
#undef REAL
#undef TRAV_NAME

#define REAL double
#define TRZ_NAME(x) x##_rz64
#include "trav_rz.inc"
#undef REAL
#undef TRZ_NAME

#define REAL float
#define TRZ_NAME(x) x##_rz32
#include "trav_rz.inc"
#undef REAL
#undef TRZ_NAME

/* ------------------------------------------------------------------------ */
/* step 1: Sigma_t(E) by table lookup (Sec. 3)                               */
/* ------------------------------------------------------------------------ */

/* first index k in [0, K] with e[k] > E */
static int64_t upper_bound(const double *e, int64_t K, double E)
{
    int64_t lo = 0, hi = K;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (e[mid] > E) hi = mid; else lo = mid + 1;
    }
    return lo;
}

double oracle_sigma(const double *e, const double *s, int64_t K, double E)
{
    int64_t ub = upper_bound(e, K, E);
    if (ub == 0) return s[0];
    if (ub == K) return s[K - 1];
    int64_t k = ub - 1;
    double slope = (s[k + 1] - s[k]) / (e[k + 1] - e[k]);
    return s[k] + slope * (E - e[k]);
}

/* 1 if E lies outside the table (the end value was used) */
static int outside_table(const double *e, int64_t K, double E)
{
    return E < e[0] || E > e[K - 1];
}

/* Sigma of every material at each of n energies: out[i*n_mat + m] */
void oracle_sigma_all(int n_mat, const int64_t *offs, const double *energy, const double *sigma,
                      int64_t n, const double *E, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        for (int m = 0; m < n_mat; ++m)
            out[i * n_mat + m] = oracle_sigma(energy + offs[m], sigma + offs[m],
                                              offs[m + 1] - offs[m], E[i]);
}

/* energy bin: edges[b] <= E < edges[b+1]; E == edges[n_bins] goes to the last bin;
 * -1 outside.  edges == NULL means one bin that takes every energy. */
int oracle_ebin(int n_bins, const double *edges, double E)
{
    if (edges == NULL) return 0;
    if (!(E >= edges[0] && E <= edges[n_bins])) return -1;
    if (E == edges[n_bins]) return n_bins - 1;
    for (int b = 0; b < n_bins; ++b)
        if (edges[b] <= E && E < edges[b + 1]) return b;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* step 2: tracing (public wrappers around trav.inc)                         */
/* ------------------------------------------------------------------------ */

int64_t oracle_trace_f64(const double *lo, const double *h, const int32_t *n,
                         const double *o, const double *u, int64_t cap,
                         int64_t *vox, double *len, double *span)
{
    event_f64 *ws = (event_f64 *)malloc(sizeof(event_f64) * (size_t)(n[0] + n[1] + n[2] + 3));
    if (!ws) return -1;
    int64_t r = trace_ws_f64(lo, h, n, o, u, cap, vox, len, span, ws);
    free(ws);
    return r;
}

int64_t oracle_trace_f32(const float *lo, const float *h, const int32_t *n,
                         const float *o, const float *u, int64_t cap,
                         int64_t *vox, float *len, float *span)
{
    event_f32 *ws = (event_f32 *)malloc(sizeof(event_f32) * (size_t)(n[0] + n[1] + n[2] + 3));
    if (!ws) return -1;
    int64_t r = trace_ws_f32(lo, h, n, o, u, cap, vox, len, span, ws);
    free(ws);
    return r;
}

/* many FP32 rays at once, CSR output (offs has n_rays+1 entries); returns the
 * total segment count, or -1 (inconsistency) / -2 (cap too small) */
int64_t oracle_trace_many_f32(const float *lo, const float *h, const int32_t *n, int64_t n_rays,
                              const float *ox, const float *oy, const float *oz,
                              const float *ux, const float *uy, const float *uz,
                              int64_t cap, int64_t *offs, int64_t *vox, float *len)
{
    event_f32 *ws = (event_f32 *)malloc(sizeof(event_f32) * (size_t)(n[0] + n[1] + n[2] + 3));
    if (!ws) return -1;
    int64_t total = 0;
    offs[0] = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        float o[3] = {ox[r], oy[r], oz[r]};
        float u[3] = {ux[r], uy[r], uz[r]};
        int64_t room = cap - total;
        if (room < 0) room = 0;
        int64_t k = trace_ws_f32(lo, h, n, o, u, room, vox + total, len + total, NULL, ws);
        if (k < 0) { free(ws); return -1; }
        if (k > room) { free(ws); return -2; }
        total += k;
        offs[r + 1] = total;
    }
    free(ws);
    return total;
}

int64_t oracle_trace_many_f64(const double *lo, const double *h, const int32_t *n, int64_t n_rays,
                              const double *ox, const double *oy, const double *oz,
                              const double *ux, const double *uy, const double *uz,
                              int64_t cap, int64_t *offs, int64_t *vox, double *len)
{
    event_f64 *ws = (event_f64 *)malloc(sizeof(event_f64) * (size_t)(n[0] + n[1] + n[2] + 3));
    if (!ws) return -1;
    int64_t total = 0;
    offs[0] = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        double o[3] = {ox[r], oy[r], oz[r]};
        double u[3] = {ux[r], uy[r], uz[r]};
        int64_t room = cap - total;
        if (room < 0) room = 0;
        int64_t k = trace_ws_f64(lo, h, n, o, u, room, vox + total, len + total, NULL, ws);
        if (k < 0) { free(ws); return -1; }
        if (k > room) { free(ws); return -2; }
        total += k;
        offs[r + 1] = total;
    }
    free(ws);
    return total;
}

/* R-Z meshes (trav_rz.inc): one ray, and many rays as CSR (offs has
 * n_rays+1 entries; returns the total, -1 inconsistency, -2 cap too small) */
int64_t oracle_trace_rz_f64(double cx, double cy, int32_t nr, const double *radii, int32_t nz, const double *zpl,
                            const double *o, const double *u, int64_t cap, int64_t *cell, double *len, double *span)
{
    rz_event_rz64 *ws = (rz_event_rz64 *)malloc(sizeof(rz_event_rz64) * (size_t)(2 * nr + nz + 2));
    if (!ws) return -1;
    int64_t r = trace_rz_ws_rz64(cx, cy, nr, radii, nz, zpl, o, u, cap, cell, len, span, ws);
    free(ws);
    return r;
}

int64_t oracle_trace_rz_f32(float cx, float cy, int32_t nr, const float *radii, int32_t nz, const float *zpl,
                            const float *o, const float *u, int64_t cap, int64_t *cell, float *len, float *span)
{
    rz_event_rz32 *ws = (rz_event_rz32 *)malloc(sizeof(rz_event_rz32) * (size_t)(2 * nr + nz + 2));
    if (!ws) return -1;
    int64_t r = trace_rz_ws_rz32(cx, cy, nr, radii, nz, zpl, o, u, cap, cell, len, span, ws);
    free(ws);
    return r;
}

int64_t oracle_trace_rz_many_f64(double cx, double cy, int32_t nr, const double *radii, int32_t nz,
                                 const double *zpl, int64_t n_rays, const double *ox, const double *oy,
                                 const double *oz, const double *ux, const double *uy, const double *uz,
                                 int64_t cap, int64_t *offs, int64_t *cell, double *len)
{
    rz_event_rz64 *ws = (rz_event_rz64 *)malloc(sizeof(rz_event_rz64) * (size_t)(2 * nr + nz + 2));
    if (!ws) return -1;
    int64_t total = 0;
    offs[0] = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        double o[3] = {ox[r], oy[r], oz[r]};
        double u[3] = {ux[r], uy[r], uz[r]};
        int64_t room = cap - total;
        if (room < 0) room = 0;
        int64_t k = trace_rz_ws_rz64(cx, cy, nr, radii, nz, zpl, o, u, room, cell + total, len + total, NULL, ws);
        if (k < 0) { free(ws); return -1; }
        if (k > room) { free(ws); return -2; }
        total += k;
        offs[r + 1] = total;
    }
    free(ws);
    return total;
}

int64_t oracle_trace_rz_many_f32(float cx, float cy, int32_t nr, const float *radii, int32_t nz,
                                 const float *zpl, int64_t n_rays, const float *ox, const float *oy,
                                 const float *oz, const float *ux, const float *uy, const float *uz,
                                 int64_t cap, int64_t *offs, int64_t *cell, float *len)
{
    rz_event_rz32 *ws = (rz_event_rz32 *)malloc(sizeof(rz_event_rz32) * (size_t)(2 * nr + nz + 2));
    if (!ws) return -1;
    int64_t total = 0;
    offs[0] = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        float o[3] = {ox[r], oy[r], oz[r]};
        float u[3] = {ux[r], uy[r], uz[r]};
        int64_t room = cap - total;
        if (room < 0) room = 0;
        int64_t k = trace_rz_ws_rz32(cx, cy, nr, radii, nz, zpl, o, u, room, cell + total, len + total, NULL, ws);
        if (k < 0) { free(ws); return -1; }
        if (k > room) { free(ws); return -2; }
        total += k;
        offs[r + 1] = total;
    }
    free(ws);
    return total;
}

/* per-ray segment counts of a batch in FP32 (fp64 = 0; float inputs) or FP64
 * (fp64 = 1; double inputs) traversal, on n_threads threads; returns the
 * total, or -1 on an internal inconsistency */
typedef struct {
    int fp64;
    const void *lo, *h;
    const int32_t *n;
    const void *o[3], *u[3];
    int64_t r0, r1;
    int64_t *counts;
    int64_t total;
    int err;
} count_job;

static void *run_count(void *arg)
{
    count_job *j = (count_job *)arg;
    size_t nev = (size_t)(j->n[0] + j->n[1] + j->n[2] + 3);
    void *ws = malloc((j->fp64 ? sizeof(event_f64) : sizeof(event_f32)) * nev);
    if (!ws) { j->err = 1; return NULL; }
    for (int64_t r = j->r0; r < j->r1; ++r) {
        int64_t k;
        if (j->fp64) {
            double o[3], u[3];
            for (int a = 0; a < 3; ++a) { o[a] = ((const double *)j->o[a])[r]; u[a] = ((const double *)j->u[a])[r]; }
            k = trace_ws_f64((const double *)j->lo, (const double *)j->h, j->n, o, u, 0, NULL, NULL, NULL,
                             (event_f64 *)ws);
        } else {
            float o[3], u[3];
            for (int a = 0; a < 3; ++a) { o[a] = ((const float *)j->o[a])[r]; u[a] = ((const float *)j->u[a])[r]; }
            k = trace_ws_f32((const float *)j->lo, (const float *)j->h, j->n, o, u, 0, NULL, NULL, NULL,
                             (event_f32 *)ws);
        }
        if (k < 0) { j->err = 1; k = 0; }
        j->counts[r] = k;
        j->total += k;
    }
    free(ws);
    return NULL;
}

int64_t oracle_count_many(int fp64, const void *lo, const void *h, const int32_t *n, int64_t n_rays,
                          const void *ox, const void *oy, const void *oz,
                          const void *ux, const void *uy, const void *uz,
                          int n_threads, int64_t *counts)
{
    if (n_threads < 1) n_threads = 1;
    count_job *jobs = (count_job *)calloc((size_t)n_threads, sizeof(count_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -1; }
    for (int t = 0; t < n_threads; ++t) {
        count_job *j = &jobs[t];
        j->fp64 = fp64; j->lo = lo; j->h = h; j->n = n;
        j->o[0] = ox; j->o[1] = oy; j->o[2] = oz; j->u[0] = ux; j->u[1] = uy; j->u[2] = uz;
        j->r0 = n_rays * t / n_threads;
        j->r1 = n_rays * (t + 1) / n_threads;
        j->counts = counts;
        pthread_create(&th[t], NULL, run_count, j);
    }
    int64_t total = 0;
    int err = 0;
    for (int t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        total += jobs[t].total;
        err |= jobs[t].err;
    }
    free(jobs); free(th);
    return err ? -1 : total;
}

/* ------------------------------------------------------------------------ */
/* steps 3-4: scoring and tallying                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *lo, *h;
    const int32_t *n;
    const uint8_t *mat;
    int n_mat;
    const int64_t *offs;
    const double *energy, *sigma;
    int n_bins;
    const double *edges;
    const double *rho;       /* per-voxel density factor, or NULL (1 everywhere) */
    int n_mix;               /* > 0: the mesh's ids name mixtures of the n_mat tables */
    const int64_t *mix_offs; /* mixture k: components mix_comp[mix_offs[k] .. mix_offs[k+1]) */
    const int32_t *mix_comp;
    const double *mix_frac;
    /* R-Z mesh instead of the Cartesian one (rz = 1): axis through (cx, cy),
     * radii[nr + 1] from 0, z planes zpl[nzz + 1]; cell i + nr k */
    int rz;
    double cx, cy;
    int32_t nr, nzz;
    const double *radii, *zpl;
} problem;

static int64_t problem_cells(const problem *p)
{
    return p->rz ? (int64_t)p->nr * p->nzz : (int64_t)p->n[0] * p->n[1] * p->n[2];
}

static int64_t problem_cap(const problem *p)
{
    return p->rz ? 2 * (int64_t)p->nr + p->nzz + 2 : (int64_t)p->n[0] + p->n[1] + p->n[2] + 3;
}

/* the ray's cells and lengths, by the problem's geometry (ws: problem_cap events of either kind) */
static int64_t problem_trace(const problem *p, const double *o, const double *u, int64_t cap, int64_t *vox,
                             double *len, void *ws)
{
    if (p->rz)
        return trace_rz_ws_rz64(p->cx, p->cy, p->nr, p->radii, p->nzz, p->zpl, o, u, cap, vox, len, NULL,
                                (rz_event_rz64 *)ws);
    return trace_ws_f64(p->lo, p->h, p->n, o, u, cap, vox, len, NULL, (event_f64 *)ws);
}

/* Sigma of every material id at energy E into sig (n_mat tables, or n_mix
 * mixtures of them); the number of table lookups outside a table is added to
 * *clamped when clamped is not NULL.  Returns the number of ids, -1 on a bad
 * argument. */
static int material_sigmas(const problem *p, double E, double *sig, int64_t *clamped)
{
    double tab[256];
    if (p->n_mat > 256 || p->n_mix > 256) return -1;
    for (int m = 0; m < p->n_mat; ++m) {
        const double *ee = p->energy + p->offs[m];
        int64_t K = p->offs[m + 1] - p->offs[m];
        tab[m] = oracle_sigma(ee, p->sigma + p->offs[m], K, E);
        if (clamped && outside_table(ee, K, E)) ++*clamped;
    }
    if (p->n_mix <= 0) {
        memcpy(sig, tab, sizeof(double) * (size_t)p->n_mat);
        return p->n_mat;
    }
    for (int k = 0; k < p->n_mix; ++k) {
        double v = 0.0;
        for (int64_t j = p->mix_offs[k]; j < p->mix_offs[k + 1]; ++j) {
            int c = p->mix_comp[j];
            if (c < 0 || c >= p->n_mat) return -1;
            v += p->mix_frac[j] * tab[c];
        }
        sig[k] = v;
    }
    return p->n_mix;
}

/* Sigma of voxel v: its material's Sigma times its density factor */
static double voxel_sigma(const problem *p, const double *sig, int64_t v)
{
    double s = sig[p->mat[v]];
    return p->rho ? p->rho[v] * s : s;
}

/* optical depth tau = tau_hi + tau_lo, accumulated with Neumaier's compensated sum */
typedef struct {
    double hi, lo;
} depth;

static void depth_add(depth *d, double x)
{
    double t = d->hi + x;
    if (fabs(d->hi) >= fabs(x)) d->lo += (d->hi - t) + x;
    else d->lo += (x - t) + d->hi;
    d->hi = t;
}

/* VRC score of one voxel (Eqs. 1-4): weight entering times (1-exp(-x))/Sigma */
static double vrc_score(double w, depth tau_in, double sig, double l)
{
    double w_in = w * exp(-tau_in.hi) * exp(-tau_in.lo);   /* Eq. 2 */
    if (sig > 0) {
        double x = sig * l;
        return w_in * (-expm1(-x)) / sig;      /* Eq. 1 with W -> W_i (Eq. 3) */
    }
    return w_in * l;                           /* limit Sigma -> 0 */
}

/*
 * Per-ray record: voxels, lengths and scores of one FP64 ray.  Returns the
 * segment count (only the first cap are written), -1 on an internal error.
 * *bin_out receives the energy bin (-1: not scored).
 */
int64_t oracle_ray_scores(const double *lo, const double *h, const int32_t *n, const uint8_t *mat,
                          int n_mat, const int64_t *offs, const double *energy, const double *sigma,
                          int n_bins, const double *edges, const double *rho,
                          int n_mix, const int64_t *mix_offs, const int32_t *mix_comp, const double *mix_frac,
                          const double *o, const double *u, double E, double w,
                          int64_t cap, int64_t *vox, double *len, double *score, int *bin_out)
{
    problem p = {lo, h, n, mat, n_mat, offs, energy, sigma, n_bins, edges, rho, n_mix, mix_offs, mix_comp, mix_frac,
                 0, 0.0, 0.0, 0, 0, NULL, NULL};
    double sig[256];
    if (material_sigmas(&p, E, sig, NULL) < 0) return -1;
    *bin_out = oracle_ebin(n_bins, edges, E);
    int64_t k = oracle_trace_f64(lo, h, n, o, u, cap, vox, len, NULL);
    if (k < 0) return k;
    int64_t m_seg = k < cap ? k : cap;
    depth tau = {0.0, 0.0};
    for (int64_t s = 0; s < m_seg; ++s) {
        double sg = voxel_sigma(&p, sig, vox[s]);
        score[s] = (*bin_out >= 0) ? vrc_score(w, tau, sg, len[s]) : 0.0;
        depth_add(&tau, sg * len[s]);
    }
    return k;
}

typedef struct {
    const problem *p;
    int64_t r0, r1;
    const double *ox, *oy, *oz, *ux, *uy, *uz, *e, *w;
    double *sum, *comp, *sq;
    int64_t *cnt;
    int64_t n_seg, n_scored, n_out_of_range, n_clamped, n_err;
} job;

static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

static void *run_job(void *arg)
{
    job *j = (job *)arg;
    const problem *p = j->p;
    const int64_t nvox = problem_cells(p);
    int64_t cap = problem_cap(p);
    int64_t *vox = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    double *len = (double *)malloc(sizeof(double) * (size_t)cap);
    void *ws = malloc((sizeof(event_f64) > sizeof(rz_event_rz64) ? sizeof(event_f64) : sizeof(rz_event_rz64)) *
                      (size_t)cap);
    double sig[256];
    if (!vox || !len || !ws) { j->n_err = 1; free(vox); free(len); free(ws); return NULL; }
    for (int64_t r = j->r0; r < j->r1; ++r) {
        double E = j->e[r];
        int b = oracle_ebin(p->n_bins, p->edges, E);
        double o[3] = {j->ox[r], j->oy[r], j->oz[r]};
        double u[3] = {j->ux[r], j->uy[r], j->uz[r]};
        int64_t k = problem_trace(p, o, u, cap, vox, len, ws);
        if (k < 0 || k > cap) { j->n_err++; continue; }
        j->n_seg += k;
        if (b < 0) { j->n_out_of_range++; continue; }
        j->n_scored++;
        if (material_sigmas(p, E, sig, &j->n_clamped) < 0) { j->n_err++; continue; }
        depth tau = {0.0, 0.0};
        for (int64_t s = 0; s < k; ++s) {
            double sg = voxel_sigma(p, sig, vox[s]);
            double f = vrc_score(j->w[r], tau, sg, len[s]);
            depth_add(&tau, sg * len[s]);
            int64_t t = (int64_t)b * nvox + vox[s];
            neumaier_add(&j->sum[t], &j->comp[t], f);
            if (j->sq) j->sq[t] += f * f;
            if (j->cnt && f != 0.0) j->cnt[t] += 1;
        }
    }
    free(vox); free(len); free(ws);
    return NULL;
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/*
 * Whole-tally run.  tally[b*nvox + v] receives the compensated sum; tally_sq
 * and tally_cnt (optional) the sum of squares and the number of non-zero
 * contributions.  Outputs are overwritten.  stats: [0] segments traced,
 * [1] rays scored, [2] rays outside the energy bins, [3] material lookups
 * outside a table, [4] internal errors.  *seconds: wall time of the
 * tracing-and-scoring part (set-up and the final reduction excluded, as the
 * paper times the transport part only, Sec. 4).  Rays are split into
 * n_threads static chunks with private tallies.
 */
static int cast_problem(const problem *pp, int64_t n_rays,
                        const double *ox, const double *oy, const double *oz,
                        const double *ux, const double *uy, const double *uz,
                        const double *e, const double *w, int n_threads,
                        double *tally, double *tally_sq, int64_t *tally_cnt,
                        int64_t *stats, double *seconds)
{
    problem p = *pp;
    const int n_bins = p.n_bins;
    const int64_t nvox = problem_cells(&p);
    const int64_t nt = (int64_t)n_bins * nvox;
    if (n_threads < 1) n_threads = 1;
    job *jobs = (job *)calloc((size_t)n_threads, sizeof(job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) return -3;
    int rc = 0;
    for (int t = 0; t < n_threads; ++t) {
        job *j = &jobs[t];
        j->p = &p;
        j->r0 = n_rays * t / n_threads;
        j->r1 = n_rays * (t + 1) / n_threads;
        j->ox = ox; j->oy = oy; j->oz = oz; j->ux = ux; j->uy = uy; j->uz = uz; j->e = e; j->w = w;
        j->sum = (double *)calloc((size_t)nt, sizeof(double));
        j->comp = (double *)calloc((size_t)nt, sizeof(double));
        j->sq = tally_sq ? (double *)calloc((size_t)nt, sizeof(double)) : NULL;
        j->cnt = tally_cnt ? (int64_t *)calloc((size_t)nt, sizeof(int64_t)) : NULL;
        if (!j->sum || !j->comp || (tally_sq && !j->sq) || (tally_cnt && !j->cnt)) rc = -3;
    }
    if (rc == 0) {
        double t0 = now_s();
        for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
        for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
        if (seconds) *seconds = now_s() - t0;
        for (int64_t i = 0; i < nt; ++i) {
            double s = 0.0, c = 0.0, q = 0.0;
            int64_t k = 0;
            for (int t = 0; t < n_threads; ++t) {
                neumaier_add(&s, &c, jobs[t].sum[i]);
                neumaier_add(&s, &c, jobs[t].comp[i]);
                if (tally_sq) q += jobs[t].sq[i];
                if (tally_cnt) k += jobs[t].cnt[i];
            }
            tally[i] = s + c;
            if (tally_sq) tally_sq[i] = q;
            if (tally_cnt) tally_cnt[i] = k;
        }
        if (stats) {
            memset(stats, 0, 5 * sizeof(int64_t));
            for (int t = 0; t < n_threads; ++t) {
                stats[0] += jobs[t].n_seg;
                stats[1] += jobs[t].n_scored;
                stats[2] += jobs[t].n_out_of_range;
                stats[3] += jobs[t].n_clamped;
                stats[4] += jobs[t].n_err;
            }
            if (stats[4]) rc = -1;
        }
    }
    for (int t = 0; t < n_threads; ++t) {
        free(jobs[t].sum); free(jobs[t].comp); free(jobs[t].sq); free(jobs[t].cnt);
    }
    free(jobs); free(th);
    return rc;
}

int oracle_cast(const double *lo, const double *h, const int32_t *n, const uint8_t *mat,
                int n_mat, const int64_t *offs, const double *energy, const double *sigma,
                int n_bins, const double *edges, const double *rho,
                int n_mix, const int64_t *mix_offs, const int32_t *mix_comp, const double *mix_frac,
                int64_t n_rays,
                const double *ox, const double *oy, const double *oz,
                const double *ux, const double *uy, const double *uz,
                const double *e, const double *w, int n_threads,
                double *tally, double *tally_sq, int64_t *tally_cnt,
                int64_t *stats, double *seconds)
{
    problem p = {lo, h, n, mat, n_mat, offs, energy, sigma, n_bins, edges, rho, n_mix, mix_offs, mix_comp, mix_frac,
                 0, 0.0, 0.0, 0, 0, NULL, NULL};
    return cast_problem(&p, n_rays, ox, oy, oz, ux, uy, uz, e, w, n_threads, tally, tally_sq, tally_cnt, stats,
                        seconds);
}

/* The whole-tally run of oracle_cast on an R-Z mesh (cells i + nr k; the
 * material of cell c is mat[c], its density factor rho[c] if rho is not
 * NULL). */
int oracle_cast_rz(double cx, double cy, int32_t nr, const double *radii, int32_t nz, const double *zpl,
                   const uint8_t *mat, int n_mat, const int64_t *offs, const double *energy, const double *sigma,
                   int n_bins, const double *edges, const double *rho, int64_t n_rays,
                   const double *ox, const double *oy, const double *oz,
                   const double *ux, const double *uy, const double *uz,
                   const double *e, const double *w, int n_threads,
                   double *tally, double *tally_sq, int64_t *tally_cnt,
                   int64_t *stats, double *seconds)
{
    problem p = {NULL, NULL, NULL, mat, n_mat, offs, energy, sigma, n_bins, edges, rho, 0, NULL, NULL, NULL,
                 1, cx, cy, nr, nz, radii, zpl};
    return cast_problem(&p, n_rays, ox, oy, oz, ux, uy, uz, e, w, n_threads, tally, tally_sq, tally_cnt, stats,
                        seconds);
}

/* Per-ray record of oracle_ray_scores on an R-Z mesh. */
int64_t oracle_ray_scores_rz(double cx, double cy, int32_t nr, const double *radii, int32_t nz, const double *zpl,
                             const uint8_t *mat, int n_mat, const int64_t *offs, const double *energy,
                             const double *sigma, int n_bins, const double *edges, const double *rho,
                             const double *o, const double *u, double E, double w,
                             int64_t cap, int64_t *vox, double *len, double *score, int *bin_out)
{
    problem p = {NULL, NULL, NULL, mat, n_mat, offs, energy, sigma, n_bins, edges, rho, 0, NULL, NULL, NULL,
                 1, cx, cy, nr, nz, radii, zpl};
    double sig[256];
    if (material_sigmas(&p, E, sig, NULL) < 0) return -1;
    *bin_out = oracle_ebin(n_bins, edges, E);
    int64_t k = oracle_trace_rz_f64(cx, cy, nr, radii, nz, zpl, o, u, cap, vox, len, NULL);
    if (k < 0) return k;
    int64_t m_seg = k < cap ? k : cap;
    depth tau = {0.0, 0.0};
    for (int64_t s = 0; s < m_seg; ++s) {
        double sg = voxel_sigma(&p, sig, vox[s]);
        score[s] = (*bin_out >= 0) ? vrc_score(w, tau, sg, len[s]) : 0.0;
        depth_add(&tau, sg * len[s]);
    }
    return k;
}
