/*
 * Plain FP64 CPU oracle of the hybrid force-free / PIC step
 * (Soudais, Cerutti & Contopoulos 2024, Sect. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  Single-threaded, unblocked, written for
 * reading against the paper.  Built with -ffp-contract=off so every
 * product and sum is rounded as written.
 *
 * Step n -> n+1 (state E^n, B^n, x^n, u^{n-1/2}); the order is our reading
 * of the time cycle of Sect. 3 (the cycle diagram itself is not available):
 *   1. flux function Psi from B_r^n (eq. psi), blending function f(Psi)
 *      at nodes (eq. transition, four thresholds), kill flag per cell;
 *   2. particles in cells whose four corners have f = 1 are removed
 *      (particles are absent from the pure force-free domain);
 *   3. every sort_interval steps: stable counting sort by cell;
 *   3a. sources: surface pair injection (Sect. 4), Goldreich-Julian
 *      extraction of electrons and ions (Sect. 5);
 *   4. push (eq. motion with the radiation-reaction force g of Sect. 3 and
 *      the effective field of eq. bperp; the force's strength ramped in
 *      time and the momentum across B removed near the star, Sect. 5),
 *      move, charge-conserving deposit;
 *   4a. threshold pair creation by the pushed leptons (Sect. 5);
 *   5. field step: Faraday half step (eq. faraday), force-free current at
 *      nodes (drift part of eq. JFFE), blend (eq. blending), Ampere
 *      (eq. ampere), force-free E correction at nodes (E.B projection and
 *      |E| <= |B| cap of Sect. 3) averaged back to the staggered mesh,
 *      Faraday half step, absorbing layer (Sect. 4).
 * Geometry: r_i = rmin exp(i dlog), theta_j = j pi/nth, Stokes (finite
 * volume) form of the curls on primal and dual faces, 2 pi dropped.
 */
#include "ffpic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

#define ORA_MAXTHREADS 256

struct species {
    int64_t n, cap;
    double *r, *th, *ur, *uth, *uph;
};

struct ora_sim {
    ora_params p;
    int nr, nth, ld;
    size_t nn;
    double dlog, dth, dt, omega;
    double *rn, *rh;          /* r_i (nr+1), r_{i+1/2} (nr) */
    double *thn, *sn, *cn;    /* theta_j, sin, cos at nodes (nth+1) */
    double *sh, *ch;          /* sin, cos at theta_{j+1/2} (nth) */
    double *F[ORA_NCOMP];
    uint8_t *kill;            /* nr*nth */
    struct species sp[ORA_MAXSPEC];
    int64_t removed[ORA_MAXSPEC][4];
    double *tbuf[ORA_MAXTHREADS];   /* OpenMP build: per-thread deposit rows */
    size_t tcap[ORA_MAXTHREADS];
    int64_t step;
    int32_t *offsets[ORA_MAXSPEC];
};

#define AT(s, a, i, j) ((s)->F[a][(size_t)(i) * (s)->ld + (j)])

/* ------------------------------------------------------------------ */
/* geometry (Sect. 4 grid: log-spaced r, uniform theta on [0, pi])     */

static double sq(double x) { return x * x; }

/* primal faces, 2 pi dropped */
static double area_r(const ora_sim *s, int i, int j)
{
    return s->rn[i] * s->rn[i] * (s->cn[j] - s->cn[j + 1]);
}
static double area_th(const ora_sim *s, int i, int j)
{
    return s->sn[j] * (s->rn[i + 1] * s->rn[i + 1] - s->rn[i] * s->rn[i]) * 0.5;
}
static double area_ph(const ora_sim *s, int i)
{
    return s->dth * (s->rn[i + 1] * s->rn[i + 1] - s->rn[i] * s->rn[i]) * 0.5;
}
/* dual cells around node (i, j): theta in [theta_{j-1/2}, theta_{j+1/2}],
   clipped to [0, pi] on the axis (cap cells) */
static double cos_lo(const ora_sim *s, int j) { return j == 0 ? 1.0 : s->ch[j - 1]; }
static double cos_hi(const ora_sim *s, int j) { return j == s->nth ? -1.0 : s->ch[j]; }
static double dual_dth(const ora_sim *s, int j)
{
    return (j == 0 || j == s->nth) ? 0.5 * s->dth : s->dth;
}
static double r_lo(const ora_sim *s, int i) { return i == 0 ? s->rn[0] : s->rh[i - 1]; }
static double r_hi(const ora_sim *s, int i) { return i == s->nr ? s->rn[s->nr] : s->rh[i]; }
static double darea_r(const ora_sim *s, int i, int j)   /* at (i+1/2, j) */
{
    return s->rh[i] * s->rh[i] * (cos_lo(s, j) - cos_hi(s, j));
}
static double darea_th(const ora_sim *s, int i, int j)  /* at (i, j+1/2) */
{
    return s->sh[j] * (sq(r_hi(s, i)) - sq(r_lo(s, i))) * 0.5;
}
static double darea_ph(const ora_sim *s, int i, int j)  /* at (i, j) */
{
    return dual_dth(s, j) * (sq(r_hi(s, i)) - sq(r_lo(s, i))) * 0.5;
}
static double dvol(const ora_sim *s, int i, int j)
{
    double a = r_lo(s, i), b = r_hi(s, i);
    return (b * b * b - a * a * a) / 3.0 * (cos_lo(s, j) - cos_hi(s, j));
}

/* ------------------------------------------------------------------ */
/* flux function and blending function                                 */

/* Piecewise blending of eq. transition generalised to the two force-free
   domains of Table 1: f = 1 below psi_0 (FF-I) and from psi_3 up (FF-II),
   linear on (psi_0, psi_1) and (psi_2, psi_3), 0 in between.  Equal
   thresholds give a sharp boundary (FF iff psi < psi_0, FF iff psi >= psi_3). */
double ora_blend(double psi, const double t[4])
{
    if (psi >= t[3]) return 1.0;
    if (psi < t[0]) return 1.0;
    if (psi < t[1]) return (t[1] - psi) / (t[1] - t[0]);
    if (psi > t[2]) return (psi - t[2]) / (t[3] - t[2]);
    return 0.0;
}

/* eq. psi: Psi(r, theta) = int_0^theta B_r r^2 sin theta' dtheta', summed
   cell by cell along theta in increasing j. */
static void compute_psi_mask(ora_sim *s)
{
    int nr = s->nr, nth = s->nth;
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= nr; i++) {
        double psi = 0.0;
        AT(s, ORA_PSI, i, 0) = 0.0;
        for (int j = 0; j < nth; j++) {
            psi = psi + AT(s, ORA_BR, i, j) * area_r(s, i, j);
            AT(s, ORA_PSI, i, j + 1) = psi;
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j <= nth; j++)
            AT(s, ORA_F, i, j) = s->p.ff_enable
                ? ora_blend(AT(s, ORA_PSI, i, j), s->p.psi_thr) : 0.0;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < nth; j++)
            s->kill[(size_t)i * nth + j] =
                AT(s, ORA_F, i, j) == 1.0 && AT(s, ORA_F, i + 1, j) == 1.0 &&
                AT(s, ORA_F, i, j + 1) == 1.0 && AT(s, ORA_F, i + 1, j + 1) == 1.0;
}

/* ------------------------------------------------------------------ */
/* initial fields                                                      */

static double psi_init(const ora_sim *s, int i, int j)
{
    double r = s->rn[i], st = s->sn[j], ct = s->cn[j], mu = s->p.mu;
    switch (s->p.init) {
    case 1: /* aligned dipole, eq. flux_dipole */
        return mu * st * st / r;
    case 2: case 3: /* monopole, Psi_M = Psi_star (1 - cos theta) */
        return mu * (1.0 - ct);
    case 4: { /* dipole with the lines beyond the light cylinder opened */
        double cs = r < s->p.r_lc ? sqrt(1.0 - r / s->p.r_lc) : 0.0;
        if (fabs(ct) < cs) return mu * st * st / r;
        return mu / s->p.r_lc * (1.0 - fabs(ct)) / (1.0 - cs);
    }
    default:
        return 0.0;
    }
}

static void init_fields(ora_sim *s)
{
    int nr = s->nr, nth = s->nth;
    for (int c = 0; c < ORA_NCOMP; c++) memset(s->F[c], 0, s->nn * sizeof(double));
    if (s->p.init == 0) return;
    double *psi = malloc(s->nn * sizeof(double));
#define PS(i, j) psi[(size_t)(i) * s->ld + (j)]
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j <= nth; j++) PS(i, j) = psi_init(s, i, j);
    double om = s->omega;
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j < nth; j++) {
            AT(s, ORA_BR, i, j) = (PS(i, j + 1) - PS(i, j)) / area_r(s, i, j);
            /* corotation E = -Omega grad Psi, edge form (E = -(Omega x r) x B) */
            AT(s, ORA_ETH, i, j) = i == nr ? 0.0
                : -om * (PS(i, j + 1) - PS(i, j)) / (s->rn[i] * s->dth);
        }
    for (int i = 0; i < nr; i++)
        for (int j = 0; j <= nth; j++) {
            if (j > 0 && j < nth)
                AT(s, ORA_BTH, i, j) = -(PS(i + 1, j) - PS(i, j)) / area_th(s, i, j);
            AT(s, ORA_ER, i, j) = -om * (PS(i + 1, j) - PS(i, j)) / (s->rn[i + 1] - s->rn[i]);
        }
    if (s->p.init == 3) /* Michel: B_phi = -(Psi_star / R_LC) sin(theta) / r */
        for (int i = 0; i < nr; i++)
            for (int j = 0; j < nth; j++)
                AT(s, ORA_BPH, i, j) = -om * (PS(i, j + 1) - PS(i, j)) / (s->rh[i] * s->dth);
#undef PS
    free(psi);
    memcpy(s->F[ORA_B0R], s->F[ORA_BR], s->nn * sizeof(double));
    memcpy(s->F[ORA_B0TH], s->F[ORA_BTH], s->nn * sizeof(double));
    memcpy(s->F[ORA_B0PH], s->F[ORA_BPH], s->nn * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* creation                                                            */

static int valid(const ora_params *p)
{
    if (p->nr < 2 || p->nth < 2 || p->nr > 65535 || p->nth > 65535) return 0;
    if (!(p->rmin > 0) || !(p->rmax > p->rmin)) return 0;
    if (!(p->r_abs > p->rmin) || !(p->r_abs <= p->rmax)) return 0;
    if (!(p->cfl > 0 && p->cfl <= 1)) return 0;
    if (!(p->r_lc > 0)) return 0;
    for (int k = 0; k < 3; k++)
        if (!(p->psi_thr[k] <= p->psi_thr[k + 1])) return 0;
    if (p->nspec < 0 || p->nspec > ORA_MAXSPEC) return 0;
    if (p->sort_interval < 1) return 0;
    if (p->rr_ramp_n < 0 || p->rr_ramp_n > 4) return 0;
    for (int k = 0; k < p->rr_ramp_n; k++) {
        if (!(p->rr_ramp_f[k] >= 0.0) || !isfinite(p->rr_ramp_t[k])) return 0;
        if (k > 0 && !(p->rr_ramp_t[k] >= p->rr_ramp_t[k - 1])) return 0;
    }
    if (!(p->shell_r >= 0.0)) return 0;
    if (!(p->gj_extract >= 0.0)) return 0;
    if (p->gj_extract > 0.0)
        for (int k = 0; k < 2; k++)
            if (p->gj_species[k] < 0 || p->gj_species[k] >= p->nspec) return 0;
    if (p->gj_extract > 0.0 && p->gj_species[0] == p->gj_species[1]) return 0;
    if (!(p->gamma_th >= 0.0)) return 0;
    if (p->gamma_th > 0.0) {
        if (!(p->gamma_s >= 1.0) || !(p->gamma_s < p->gamma_th)) return 0;
        for (int k = 0; k < 2; k++)
            if (p->pair_species[k] < 0 || p->pair_species[k] >= p->nspec) return 0;
        if (p->pair_species[0] == p->pair_species[1]) return 0;
    }
    return 1;
}

/* time step: CFL number times the 2-D Courant limit of the smallest
   (innermost) cell, r_1 - r_0 by r_0 dtheta (checked against Table 1) */
double ora_timestep(const ora_params *p)
{
    double dlog = log(p->rmax / p->rmin) / p->nr, dth = PI / p->nth;
    double r0 = p->rmin, r1 = p->rmin * exp(dlog);
    double drr = r1 - r0, drt = r0 * dth;
    return p->cfl / sqrt(1.0 / (drr * drr) + 1.0 / (drt * drt));
}

ora_sim *ora_create(const ora_params *p)
{
    if (!valid(p)) return NULL;
    ora_sim *s = calloc(1, sizeof(*s));
    s->p = *p;
    s->nr = p->nr;
    s->nth = p->nth;
    s->ld = p->nth + 1;
    s->nn = (size_t)(p->nr + 1) * (p->nth + 1);
    s->dlog = log(p->rmax / p->rmin) / p->nr;
    s->dth = PI / p->nth;
    s->dt = ora_timestep(p);
    s->omega = 1.0 / p->r_lc;
    s->rn = malloc((p->nr + 1) * sizeof(double));
    s->rh = malloc(p->nr * sizeof(double));
    for (int i = 0; i <= p->nr; i++) s->rn[i] = p->rmin * exp(i * s->dlog);
    for (int i = 0; i < p->nr; i++) s->rh[i] = p->rmin * exp((i + 0.5) * s->dlog);
    s->thn = malloc((p->nth + 1) * sizeof(double));
    s->sn = malloc((p->nth + 1) * sizeof(double));
    s->cn = malloc((p->nth + 1) * sizeof(double));
    s->sh = malloc(p->nth * sizeof(double));
    s->ch = malloc(p->nth * sizeof(double));
    for (int j = 0; j <= p->nth; j++) {
        s->thn[j] = j * s->dth;
        s->sn[j] = sin(s->thn[j]);
        s->cn[j] = cos(s->thn[j]);
    }
    s->sn[0] = 0.0; s->cn[0] = 1.0;
    s->sn[p->nth] = 0.0; s->cn[p->nth] = -1.0;
    for (int j = 0; j < p->nth; j++) {
        s->sh[j] = sin((j + 0.5) * s->dth);
        s->ch[j] = cos((j + 0.5) * s->dth);
    }
    for (int c = 0; c < ORA_NCOMP; c++) s->F[c] = calloc(s->nn, sizeof(double));
    s->kill = calloc((size_t)p->nr * p->nth, 1);
    init_fields(s);
    compute_psi_mask(s);
    return s;
}

void ora_destroy(ora_sim *s)
{
    if (!s) return;
    free(s->rn); free(s->rh); free(s->thn); free(s->sn); free(s->cn);
    free(s->sh); free(s->ch);
    for (int c = 0; c < ORA_NCOMP; c++) free(s->F[c]);
    for (int t = 0; t < ORA_MAXTHREADS; t++) free(s->tbuf[t]);
    free(s->kill);
    for (int k = 0; k < ORA_MAXSPEC; k++) {
        struct species *q = &s->sp[k];
        free(q->r); free(q->th); free(q->ur); free(q->uth); free(q->uph);
        free(s->offsets[k]);
    }
    free(s);
}

void ora_info(const ora_sim *s, double out[4])
{
    out[0] = s->dt; out[1] = s->dlog; out[2] = s->dth; out[3] = s->omega;
}

/* geometry tables: 0 r_i (nr+1), 1 r_{i+1/2} (nr), 2 theta_j (nth+1),
   3 sin theta_j (nth+1), 4 cos theta_j (nth+1), 5 sin theta_{j+1/2} (nth),
   6 cos theta_{j+1/2} (nth) */
void ora_geometry(const ora_sim *s, int which, double *dst)
{
    const double *src[7] = {s->rn, s->rh, s->thn, s->sn, s->cn, s->sh, s->ch};
    size_t len[7] = {(size_t)s->nr + 1, (size_t)s->nr, (size_t)s->nth + 1, (size_t)s->nth + 1,
                     (size_t)s->nth + 1, (size_t)s->nth, (size_t)s->nth};
    if (which >= 0 && which < 7) memcpy(dst, src[which], len[which] * sizeof(double));
}

/* threads of the OpenMP build (no effect in the single-thread build) */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_get_field(const ora_sim *s, int c, double *dst)
{
    memcpy(dst, s->F[c], s->nn * sizeof(double));
}

void ora_set_field(ora_sim *s, int c, const double *src)
{
    memcpy(s->F[c], src, s->nn * sizeof(double));
    if (c >= ORA_BR && c <= ORA_BPH)
        memcpy(s->F[c + ORA_B0R - ORA_BR], src, s->nn * sizeof(double));
    if (c == ORA_BR) compute_psi_mask(s);
}

int64_t ora_step_count(const ora_sim *s) { return s->step; }
void ora_set_step(ora_sim *s, int64_t step) { s->step = step; }

void ora_removed(const ora_sim *s, int sp, int64_t out[4])
{
    for (int k = 0; k < 4; k++) out[k] = s->removed[sp][k];
}

/* ------------------------------------------------------------------ */
/* particle location: cell by comparison against the node tables,
   offsets in logical (log r, theta) units                              */

static void locate(const ora_sim *s, double r, double th, int *ci, int *cj,
                   double *a, double *b)
{
    int nr = s->nr, nth = s->nth;
    int i = (int)floor(log(r / s->p.rmin) / s->dlog);
    if (i < 0) i = 0;
    if (i > nr - 1) i = nr - 1;
    while (i > 0 && r < s->rn[i]) i--;
    while (i < nr - 1 && r >= s->rn[i + 1]) i++;
    double aa = log(r / s->rn[i]) / s->dlog;
    if (aa < 0.0) aa = 0.0;
    if (aa > 1.0) aa = 1.0;
    int j = (int)floor(th / s->dth);
    if (j < 0) j = 0;
    if (j > nth - 1) j = nth - 1;
    while (j > 0 && th < s->thn[j]) j--;
    while (j < nth - 1 && th >= s->thn[j + 1]) j++;
    double bb = (th - s->thn[j]) / s->dth;
    if (bb < 0.0) bb = 0.0;
    if (bb > 1.0) bb = 1.0;
    *ci = i; *cj = j; *a = aa; *b = bb;
}

/* ------------------------------------------------------------------ */
/* sort: stable counting sort by cell key i*nth + j, dead slots last and
   dropped                                                              */

static void sort_species(ora_sim *s, int k)
{
    struct species *q = &s->sp[k];
    int64_t nkeys = (int64_t)s->nr * s->nth;
    int64_t *cnt = calloc(nkeys + 2, sizeof(int64_t));
    int64_t *key = malloc((q->n + 1) * sizeof(int64_t));
    for (int64_t p = 0; p < q->n; p++) {
        if (q->r[p] > 0.0) {
            int i, j; double a, b;
            locate(s, q->r[p], q->th[p], &i, &j, &a, &b);
            key[p] = (int64_t)i * s->nth + j;
        } else {
            key[p] = nkeys;
        }
        cnt[key[p] + 1]++;
    }
    for (int64_t c = 0; c <= nkeys; c++) cnt[c + 1] += cnt[c];
    int64_t alive = cnt[nkeys];
    free(s->offsets[k]);
    s->offsets[k] = malloc((nkeys + 1) * sizeof(int32_t));
    for (int64_t c = 0; c <= nkeys; c++) s->offsets[k][c] = (int32_t)cnt[c];
    double *arr[5] = {q->r, q->th, q->ur, q->uth, q->uph};
    double *tmp = malloc((q->n + 1) * sizeof(double));
    int64_t *dst = malloc((q->n + 1) * sizeof(int64_t));
    for (int64_t p = 0; p < q->n; p++) dst[p] = cnt[key[p]]++;
    for (int a = 0; a < 5; a++) {
        for (int64_t p = 0; p < q->n; p++) tmp[dst[p]] = arr[a][p];
        memcpy(arr[a], tmp, q->n * sizeof(double));
    }
    q->n = alive;
    free(tmp); free(dst); free(key); free(cnt);
}

void ora_sort_offsets(const ora_sim *s, int k, int32_t *off)
{
    int64_t nkeys = (int64_t)s->nr * s->nth;
    if (s->offsets[k]) memcpy(off, s->offsets[k], (nkeys + 1) * sizeof(int32_t));
    else memset(off, 0, (nkeys + 1) * sizeof(int32_t));
}

/* particles in cells entirely inside the force-free domain are removed */
static void kill_masked(ora_sim *s)
{
    for (int k = 0; k < s->p.nspec; k++) {
        struct species *q = &s->sp[k];
        int64_t nk = 0;
#pragma omp parallel for reduction(+ : nk) schedule(static)
        for (int64_t p = 0; p < q->n; p++) {
            if (!(q->r[p] > 0.0)) continue;
            int i, j; double a, b;
            locate(s, q->r[p], q->th[p], &i, &j, &a, &b);
            if (s->kill[(size_t)i * s->nth + j]) {
                q->r[p] = -1.0;
                nk++;
            }
        }
        s->removed[k][1] += nk;
    }
}

int64_t ora_load_particles(ora_sim *s, int k, int64_t n, const double *r,
                           const double *th, const double *ur,
                           const double *uth, const double *uph)
{
    struct species *q = &s->sp[k];
    if (q->n + n > q->cap) {
        int64_t cap = q->n + n;
        q->r = realloc(q->r, cap * sizeof(double));
        q->th = realloc(q->th, cap * sizeof(double));
        q->ur = realloc(q->ur, cap * sizeof(double));
        q->uth = realloc(q->uth, cap * sizeof(double));
        q->uph = realloc(q->uph, cap * sizeof(double));
        q->cap = cap;
    }
    for (int64_t p = 0; p < n; p++) {
        int64_t d = q->n + p;
        int ok = isfinite(r[p]) && isfinite(th[p]) && isfinite(ur[p]) &&
                 isfinite(uth[p]) && isfinite(uph[p]) && r[p] >= s->p.rmin &&
                 r[p] < s->p.r_abs && th[p] >= 0.0 && th[p] <= PI;
        q->r[d] = ok ? r[p] : -1.0;
        q->th[d] = th[p]; q->ur[d] = ur[p]; q->uth[d] = uth[p]; q->uph[d] = uph[p];
        if (!ok) s->removed[k][0]++;
    }
    q->n += n;
    kill_masked(s);
    sort_species(s, k);
    return q->n;
}

int64_t ora_num_particles(const ora_sim *s, int k) { return s->sp[k].n; }

int64_t ora_get_particles(const ora_sim *s, int k, double *r, double *th,
                          double *ur, double *uth, double *uph, int32_t *cell)
{
    const struct species *q = &s->sp[k];
    for (int64_t p = 0; p < q->n; p++) {
        if (r) r[p] = q->r[p];
        if (th) th[p] = q->th[p];
        if (ur) ur[p] = q->ur[p];
        if (uth) uth[p] = q->uth[p];
        if (uph) uph[p] = q->uph[p];
        if (cell) {
            if (q->r[p] > 0.0) {
                int i, j; double a, b;
                locate(s, q->r[p], q->th[p], &i, &j, &a, &b);
                cell[p] = i * s->nth + j;
            } else {
                cell[p] = -1;
            }
        }
    }
    return q->n;
}

/* ------------------------------------------------------------------ */
/* field gather: each component bilinear in logical coordinates from its
   own staggered position; parity ghosts across the axis (r components
   even, theta and phi components odd); constant beyond the radial ends  */

typedef struct { int lo; double w; } lin;

static lin at_node(int c, double o) { lin l = {c, o}; return l; }
static lin at_half_r(int i, double a, int nr)
{
    lin l;
    if (a >= 0.5) { l.lo = i; l.w = a - 0.5; } else { l.lo = i - 1; l.w = a + 0.5; }
    if (l.lo < 0) { l.lo = 0; l.w = 0.0; }
    if (l.lo > nr - 2) { l.lo = nr - 2; l.w = 1.0; }
    return l;
}
static lin at_half_t(int j, double b)
{
    lin l;
    if (b >= 0.5) { l.lo = j; l.w = b - 0.5; } else { l.lo = j - 1; l.w = b + 0.5; }
    return l;
}

/* theta-half-indexed value with axis ghosts */
static double hval(const ora_sim *s, int c, int i, int k, double parity)
{
    if (k < 0) return parity * AT(s, c, i, 0);
    if (k >= s->nth) return parity * AT(s, c, i, s->nth - 1);
    return AT(s, c, i, k);
}

static double bilin(const ora_sim *s, int c, lin lr, lin lt, int thalf, double parity)
{
    double v00, v10, v01, v11;
    if (thalf) {
        v00 = hval(s, c, lr.lo, lt.lo, parity);
        v10 = hval(s, c, lr.lo + 1, lt.lo, parity);
        v01 = hval(s, c, lr.lo, lt.lo + 1, parity);
        v11 = hval(s, c, lr.lo + 1, lt.lo + 1, parity);
    } else {
        v00 = AT(s, c, lr.lo, lt.lo);
        v10 = AT(s, c, lr.lo + 1, lt.lo);
        v01 = AT(s, c, lr.lo, lt.lo + 1);
        v11 = AT(s, c, lr.lo + 1, lt.lo + 1);
    }
    return (1.0 - lr.w) * (1.0 - lt.w) * v00 + lr.w * (1.0 - lt.w) * v10 +
           (1.0 - lr.w) * lt.w * v01 + lr.w * lt.w * v11;
}

static void gather(const ora_sim *s, int i, int j, double a, double b,
                   double E[3], double B[3])
{
    lin rn = at_node(i, a), rh = at_half_r(i, a, s->nr);
    lin tn = at_node(j, b), th = at_half_t(j, b);
    E[0] = bilin(s, ORA_ER, rh, tn, 0, 1.0);
    E[1] = bilin(s, ORA_ETH, rn, th, 1, -1.0);
    E[2] = bilin(s, ORA_EPH, rn, tn, 0, 1.0);
    B[0] = bilin(s, ORA_BR, rn, th, 1, 1.0);
    B[1] = bilin(s, ORA_BTH, rh, tn, 0, 1.0);
    B[2] = bilin(s, ORA_BPH, rh, th, 1, -1.0);
}

void ora_gather(const ora_sim *s, double r, double th, double E[3], double B[3])
{
    int i, j; double a, b;
    locate(s, r, th, &i, &j, &a, &b);
    gather(s, i, j, a, b, E, B);
}

/* ------------------------------------------------------------------ */
/* pusher: Boris rotation for the Lorentz force of eq. motion, then the
   Landau-Lifshitz radiation-reaction force g (Sect. 3) added explicitly
   with the time-centred velocity; B_perp from eq. bperp.               */

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

void ora_boris_rr(double u[3], const double E[3], const double B[3],
                  double dt, double wq, double rr)
{
    double h = 0.5 * dt * wq;
    double um[3], t[3], sv[3], up[3], c[3], uL[3];
    for (int k = 0; k < 3; k++) um[k] = u[k] + h * E[k];
    double gm = sqrt(1.0 + dot3(um, um));
    for (int k = 0; k < 3; k++) t[k] = h * B[k] / gm;
    double t2 = dot3(t, t);
    for (int k = 0; k < 3; k++) sv[k] = 2.0 * t[k] / (1.0 + t2);
    cross3(um, t, c);
    for (int k = 0; k < 3; k++) up[k] = um[k] + c[k];
    cross3(up, sv, c);
    for (int k = 0; k < 3; k++) uL[k] = um[k] + c[k] + h * E[k];
    if (rr != 0.0) {
        double ub[3], beta[3], bxB[3], Fv[3], FxB[3];
        for (int k = 0; k < 3; k++) ub[k] = 0.5 * (u[k] + uL[k]);
        double gb = sqrt(1.0 + dot3(ub, ub));
        for (int k = 0; k < 3; k++) beta[k] = ub[k] / gb;
        cross3(beta, B, bxB);
        for (int k = 0; k < 3; k++) Fv[k] = E[k] + bxB[k];
        double be = dot3(beta, E);
        double bp2 = dot3(Fv, Fv) - be * be;
        if (bp2 < 0.0) bp2 = 0.0;
        cross3(Fv, B, FxB);
        for (int k = 0; k < 3; k++)
            uL[k] = uL[k] + dt * rr * (FxB[k] + be * E[k] - gb * gb * bp2 * beta[k]);
    }
    for (int k = 0; k < 3; k++) u[k] = uL[k];
}

/* ------------------------------------------------------------------ */
/* charge-conserving deposit: zigzag split of the move in logical
   coordinates; radial and polar charge fluxes through the dual faces,
   azimuthal current from v_phi at the mid-point                        */

/* deposit target: the three accumulators of the rows from i0 on, ld
   entries a row (the grid's own, or in the parallel build one thread's
   private rows, added to the grid's afterwards in thread order) */
typedef struct { double *acc[3]; int i0, ld, rows; } jtarget;
#define JT(t, k, i, j) ((t)->acc[k][(size_t)((i) - (t)->i0) * (t)->ld + (j)])

static void deposit(const ora_sim *s, const jtarget *t, double Q, int i1, int j1, double a1,
                    double b1, int i2, int j2, double a2, double b2, double vph)
{
    int di = i2 - i1, dj = j2 - j1;
    double x1 = a1, y1 = b1, x2 = di + a2, y2 = dj + b2;
    double xr = fmin((di < 0 ? di : 0) + 1.0, fmax((di > 0 ? di : 0), 0.5 * (x1 + x2)));
    double yr = fmin((dj < 0 ? dj : 0) + 1.0, fmax((dj > 0 ? dj : 0), 0.5 * (y1 + y2)));
    double fx1 = Q * (xr - x1), fy1 = Q * (yr - y1);
    double fx2 = Q * (x2 - xr), fy2 = Q * (y2 - yr);
    double wx1 = 0.5 * (x1 + xr), wy1 = 0.5 * (y1 + yr);
    double wx2 = 0.5 * (xr + x2) - di, wy2 = 0.5 * (yr + y2) - dj;
    JT(t, 0, i1, j1) += fx1 * (1.0 - wy1);
    JT(t, 0, i1, j1 + 1) += fx1 * wy1;
    JT(t, 1, i1, j1) += fy1 * (1.0 - wx1);
    JT(t, 1, i1 + 1, j1) += fy1 * wx1;
    JT(t, 0, i2, j2) += fx2 * (1.0 - wy2);
    JT(t, 0, i2, j2 + 1) += fx2 * wy2;
    JT(t, 1, i2, j2) += fy2 * (1.0 - wx2);
    JT(t, 1, i2 + 1, j2) += fy2 * wx2;
    double xm = 0.5 * (x1 + x2), ym = 0.5 * (y1 + y2);
    int im = (int)floor(xm), jm = (int)floor(ym);
    if (i1 + im > s->nr - 1) im = s->nr - 1 - i1;
    if (j1 + jm > s->nth - 1) jm = s->nth - 1 - j1;
    double wx = xm - im, wy = ym - jm;
    double qv = Q * vph;
    JT(t, 2, i1 + im, j1 + jm) += qv * (1.0 - wx) * (1.0 - wy);
    JT(t, 2, i1 + im + 1, j1 + jm) += qv * wx * (1.0 - wy);
    JT(t, 2, i1 + im, j1 + jm + 1) += qv * (1.0 - wx) * wy;
    JT(t, 2, i1 + im + 1, j1 + jm + 1) += qv * wx * wy;
}

/* Radiation-reaction ramp of Sect. 5 (reduced strength while the
   magnetosphere fills, raised to the nominal value later): piecewise
   linear through the knots (t_k, f_k), constant before the first and
   after the last; no knots = 1. */
double ora_rr_factor(const ora_params *p, double t)
{
    int n = p->rr_ramp_n;
    if (n <= 0) return 1.0;
    if (t <= p->rr_ramp_t[0]) return p->rr_ramp_f[0];
    for (int k = 1; k < n; k++) {
        if (t < p->rr_ramp_t[k]) {
            double t0 = p->rr_ramp_t[k - 1], t1 = p->rr_ramp_t[k];
            double x = (t - t0) / (t1 - t0);
            return p->rr_ramp_f[k - 1] + x * (p->rr_ramp_f[k] - p->rr_ramp_f[k - 1]);
        }
    }
    return p->rr_ramp_f[n - 1];
}

/* one particle of species k: Boris rotation and radiation reaction in the
   local Cartesian frame at azimuth 0 (x along the cylindrical radius, y
   along phi, z along the rotation axis), move, rotation back into the
   meridional plane, deposit; removed[0], removed[1] count the particles
   that reach the star and the absorber */
typedef struct { double Q, wq, rr; } push_consts;

static void push_one(ora_sim *s, int k, int64_t p, const push_consts *pc, const jtarget *t,
                     int64_t removed[2])
{
    struct species *q = &s->sp[k];
    double dt = s->dt;
    if (!(q->r[p] > 0.0)) return;
    double r = q->r[p], th = q->th[p];
    int i, j; double a, b;
    locate(s, r, th, &i, &j, &a, &b);
    double Es[3], Bs[3];
    gather(s, i, j, a, b, Es, Bs);
    double st = sin(th), ct = cos(th);
    double E[3] = {Es[0] * st + Es[1] * ct, Es[2], Es[0] * ct - Es[1] * st};
    double B[3] = {Bs[0] * st + Bs[1] * ct, Bs[2], Bs[0] * ct - Bs[1] * st};
    double u[3] = {q->ur[p] * st + q->uth[p] * ct, q->uph[p],
                   q->ur[p] * ct - q->uth[p] * st};
    ora_boris_rr(u, E, B, dt, pc->wq, pc->rr);
    if (r < s->p.shell_r) {
        /* shell around the star (Sect. 5): only the momentum along the
           local magnetic field is kept */
        double b2 = dot3(B, B);
        if (b2 > 0.0) {
            double ub = dot3(u, B) / b2;
            for (int c = 0; c < 3; c++) u[c] = ub * B[c];
        }
    }
    double g = sqrt(1.0 + dot3(u, u));
    double v[3] = {u[0] / g, u[1] / g, u[2] / g};
    double x = r * st + dt * v[0], y = dt * v[1], z = r * ct + dt * v[2];
    double w = sqrt(x * x + y * y);
    double cp = w > 0.0 ? x / w : 1.0, sp = w > 0.0 ? y / w : 0.0;
    double ux = cp * u[0] + sp * u[1], uy = -sp * u[0] + cp * u[1], uz = u[2];
    double r2 = sqrt(w * w + z * z);
    double th2 = atan2(w, z);
    if (!(r2 >= s->p.rmin)) { q->r[p] = -1.0; removed[0]++; return; }
    if (r2 >= s->p.r_abs) { q->r[p] = -1.0; removed[1]++; return; }
    double st2 = w / r2, ct2 = z / r2;
    int i2, j2; double a2, b2;
    locate(s, r2, th2, &i2, &j2, &a2, &b2);
    deposit(s, t, pc->Q, i, j, a, b, i2, j2, a2, b2, v[1]);
    q->r[p] = r2;
    q->th[p] = th2;
    q->ur[p] = ux * st2 + uz * ct2;
    q->uth[p] = ux * ct2 - uz * st2;
    q->uph[p] = uy;
}

#ifdef _OPENMP
/* The same push on T threads, each over an equal range of slots.  After a
   sort the slots of a range hold a compact band of cells, so each thread
   deposits into private rows covering its particles' cells and the reach
   of a move; the private rows are then added to the grid's in thread
   order, so the result does not depend on the threads' timing. */
static void push_species_threads(ora_sim *s, int k, const push_consts *pc, int T)
{
    struct species *q = &s->sp[k];
    const int64_t n = q->n;
    jtarget tg[ORA_MAXTHREADS];
    int64_t rem[ORA_MAXTHREADS][2];
    if (T > ORA_MAXTHREADS) T = ORA_MAXTHREADS;
#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num();
        const int64_t a = n * t / T, b = n * (t + 1) / T;
        int imin = s->nr, imax = -1;
        for (int64_t p = a; p < b; p++) {
            if (!(q->r[p] > 0.0)) continue;
            int i, j; double aa, bb;
            locate(s, q->r[p], q->th[p], &i, &j, &aa, &bb);
            if (i < imin) imin = i;
            if (i > imax) imax = i;
        }
        rem[t][0] = rem[t][1] = 0;
        tg[t].rows = 0;
        if (imax >= 0) {
            int r0 = imin - 1 < 0 ? 0 : imin - 1;
            int r1 = imax + 2 > s->nr ? s->nr : imax + 2;
            size_t len = (size_t)(r1 - r0 + 1) * s->ld;
            if (s->tcap[t] < 3 * len) {
                free(s->tbuf[t]);
                s->tbuf[t] = malloc(3 * len * sizeof(double));
                s->tcap[t] = 3 * len;
            }
            memset(s->tbuf[t], 0, 3 * len * sizeof(double));
            tg[t].i0 = r0;
            tg[t].ld = s->ld;
            tg[t].rows = r1 - r0 + 1;
            for (int c = 0; c < 3; c++) tg[t].acc[c] = s->tbuf[t] + c * len;
            for (int64_t p = a; p < b; p++) push_one(s, k, p, pc, &tg[t], rem[t]);
        }
    }
    /* each grid row adds the threads' rows in thread order */
#pragma omp parallel for schedule(static) num_threads(T)
    for (int i = 0; i <= s->nr; i++) {
        for (int t = 0; t < T; t++) {
            if (tg[t].rows == 0 || i < tg[t].i0 || i >= tg[t].i0 + tg[t].rows) continue;
            for (int c = 0; c < 3; c++) {
                double *dst = s->F[ORA_JR + c] + (size_t)i * s->ld;
                const double *src = tg[t].acc[c] + (size_t)(i - tg[t].i0) * s->ld;
                for (int j = 0; j < s->ld; j++) dst[j] += src[j];
            }
        }
    }
    for (int t = 0; t < T; t++) {
        s->removed[k][2] += rem[t][0];
        s->removed[k][3] += rem[t][1];
    }
}
#endif

static void push_species(ora_sim *s, int k)
{
    struct species *q = &s->sp[k];
    double qm = s->p.qm[k];
    push_consts pc;
    pc.Q = (qm > 0 ? 1.0 : -1.0) * s->p.weight[k];
    pc.wq = s->p.omega_b * qm;
    pc.rr = s->p.rr_coef * ora_rr_factor(&s->p, (double)s->step * s->dt) *
            fabs(qm) * fabs(qm) * fabs(qm);
#ifdef _OPENMP
    const int T = omp_get_max_threads();
    if (T > 1 && q->n >= 4096) {
        push_species_threads(s, k, &pc, T);
        return;
    }
#endif
    jtarget grid = {{s->F[ORA_JR], s->F[ORA_JTH], s->F[ORA_JPH]}, 0, s->ld, s->nr + 1};
    int64_t rem[2] = {0, 0};
    for (int64_t p = 0; p < q->n; p++) push_one(s, k, p, &pc, &grid, rem);
    s->removed[k][2] += rem[0];
    s->removed[k][3] += rem[1];
}

/* ------------------------------------------------------------------ */
/* field step                                                          */

/* eq. faraday in Stokes form on the primal faces */
static void faraday(ora_sim *s, double h)
{
    int nr = s->nr, nth = s->nth;
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j < nth; j++) {
            double circ = s->rn[i] * (s->sn[j + 1] * AT(s, ORA_EPH, i, j + 1) -
                                      s->sn[j] * AT(s, ORA_EPH, i, j));
            AT(s, ORA_BR, i, j) -= h * circ / area_r(s, i, j);
        }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        for (int j = 1; j < nth; j++) {
            double circ = s->sn[j] * (s->rn[i + 1] * AT(s, ORA_EPH, i + 1, j) -
                                      s->rn[i] * AT(s, ORA_EPH, i, j));
            AT(s, ORA_BTH, i, j) += h * circ / area_th(s, i, j);
        }
        AT(s, ORA_BTH, i, 0) = 0.0;
        AT(s, ORA_BTH, i, nth) = 0.0;
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < nth; j++) {
            double circ = s->dth * (s->rn[i + 1] * AT(s, ORA_ETH, i + 1, j) -
                                    s->rn[i] * AT(s, ORA_ETH, i, j)) -
                          (s->rn[i + 1] - s->rn[i]) *
                              (AT(s, ORA_ER, i, j + 1) - AT(s, ORA_ER, i, j));
            AT(s, ORA_BPH, i, j) -= h * circ / area_ph(s, i);
        }
}

/* node collocation by arithmetic averages of the neighbouring staggered
   values (Sect. 3); one-sided at the radial ends, parity at the axis */
static void node_E(const ora_sim *s, int i, int j, double e[3])
{
    int nr = s->nr, nth = s->nth;
    e[0] = i == 0 ? AT(s, ORA_ER, 0, j) : i == nr ? AT(s, ORA_ER, nr - 1, j)
         : 0.5 * (AT(s, ORA_ER, i - 1, j) + AT(s, ORA_ER, i, j));
    e[1] = (j == 0 || j == nth) ? 0.0
         : 0.5 * (AT(s, ORA_ETH, i, j - 1) + AT(s, ORA_ETH, i, j));
    e[2] = AT(s, ORA_EPH, i, j);
}
static void node_B(const ora_sim *s, int i, int j, double b[3])
{
    int nr = s->nr, nth = s->nth;
    b[0] = j == 0 ? AT(s, ORA_BR, i, 0) : j == nth ? AT(s, ORA_BR, i, nth - 1)
         : 0.5 * (AT(s, ORA_BR, i, j - 1) + AT(s, ORA_BR, i, j));
    b[1] = i == 0 ? AT(s, ORA_BTH, 0, j) : i == nr ? AT(s, ORA_BTH, nr - 1, j)
         : 0.5 * (AT(s, ORA_BTH, i - 1, j) + AT(s, ORA_BTH, i, j));
    if (j == 0 || j == nth) {
        b[2] = 0.0;
    } else if (i == 0) {
        b[2] = 0.5 * (AT(s, ORA_BPH, 0, j - 1) + AT(s, ORA_BPH, 0, j));
    } else if (i == nr) {
        b[2] = 0.5 * (AT(s, ORA_BPH, nr - 1, j - 1) + AT(s, ORA_BPH, nr - 1, j));
    } else {
        b[2] = 0.25 * (AT(s, ORA_BPH, i - 1, j - 1) + AT(s, ORA_BPH, i - 1, j) +
                       AT(s, ORA_BPH, i, j - 1) + AT(s, ORA_BPH, i, j));
    }
}

static double div_E(const ora_sim *s, int i, int j)
{
    double flux = darea_r(s, i, j) * AT(s, ORA_ER, i, j) -
                  darea_r(s, i - 1, j) * AT(s, ORA_ER, i - 1, j);
    if (j < s->nth) flux += darea_th(s, i, j) * AT(s, ORA_ETH, i, j);
    if (j > 0) flux -= darea_th(s, i, j - 1) * AT(s, ORA_ETH, i, j - 1);
    return flux / dvol(s, i, j);
}

/* E.B projection, then |E| <= |B| cap (Sect. 3); B = 0 gives E = 0 */
void ora_ff_node(const double E[3], const double B[3], double o[3])
{
    double b2 = dot3(B, B);
    if (!(b2 > 0.0)) { o[0] = o[1] = o[2] = 0.0; return; }
    double eb = dot3(E, B);
    for (int k = 0; k < 3; k++) o[k] = E[k] - eb * B[k] / b2;
    double e2 = dot3(o, o);
    if (e2 >= b2 && e2 > 0.0) {
        double c = sqrt(b2 / e2);
        for (int k = 0; k < 3; k++) o[k] = c * o[k];
    }
}

static double absorb(const ora_sim *s, double r)
{
    if (!(r > s->p.r_abs)) return 1.0;
    double L = s->p.rmax - s->p.r_abs;
    double x = (r - s->p.r_abs) / L;
    return exp(-(40.0 / L) * s->dt * x * x * x);
}

static void field_step(ora_sim *s)
{
    int nr = s->nr, nth = s->nth;
    size_t nn = s->nn;
    double dt = s->dt, fourpi = 4.0 * PI;
    double *jn = calloc(3 * nn, sizeof(double));   /* node J_FFE */
    double *del = calloc(3 * nn, sizeof(double));  /* node E corrections */
#define JN(c, i, j) jn[(c) * nn + (size_t)(i) * s->ld + (j)]
#define DL(c, i, j) del[(c) * nn + (size_t)(i) * s->ld + (j)]
    faraday(s, 0.5 * dt);                               /* B^{n+1/2} */

    /* force-free current at nodes: drift part of eq. JFFE,
       J = rho (E x B) / B^2 with rho = div E / 4 pi (E^n, B^{n+1/2}) */
    if (s->p.ff_enable) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i <= nr; i++)
            for (int j = 0; j <= nth; j++) {
                int ii = i == 0 ? 1 : i;
                double rho = i == nr ? 0.0 : div_E(s, ii, j) / fourpi;
                double e[3], b[3], x[3];
                node_E(s, i, j, e);
                node_B(s, i, j, b);
                double b2 = dot3(b, b);
                cross3(e, b, x);
                for (int c = 0; c < 3; c++)
                    JN(c, i, j) = b2 > 0.0 ? rho * x[c] / b2 : 0.0;
            }
    }

    /* eq. ampere with the blended current of eq. blending */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j <= nth; j++) {
            double A = darea_r(s, i, j);
            double circ = (j < nth ? s->rh[i] * s->sh[j] * AT(s, ORA_BPH, i, j) : 0.0) -
                          (j > 0 ? s->rh[i] * s->sh[j - 1] * AT(s, ORA_BPH, i, j - 1) : 0.0);
            double f = 0.5 * (AT(s, ORA_F, i, j) + AT(s, ORA_F, i + 1, j));
            double J = (1.0 - f) * AT(s, ORA_JR, i, j) / (dt * A) +
                       f * 0.5 * (JN(0, i, j) + JN(0, i + 1, j));
            AT(s, ORA_ER, i, j) += dt * circ / A - fourpi * dt * J;
        }
#pragma omp parallel for schedule(static)
    for (int i = 1; i < nr; i++)
        for (int j = 0; j < nth; j++) {
            double A = darea_th(s, i, j);
            double circ = -(s->rh[i] * s->sh[j] * AT(s, ORA_BPH, i, j) -
                            s->rh[i - 1] * s->sh[j] * AT(s, ORA_BPH, i - 1, j));
            double f = 0.5 * (AT(s, ORA_F, i, j) + AT(s, ORA_F, i, j + 1));
            double J = (1.0 - f) * AT(s, ORA_JTH, i, j) / (dt * A) +
                       f * 0.5 * (JN(1, i, j) + JN(1, i, j + 1));
            AT(s, ORA_ETH, i, j) += dt * circ / A - fourpi * dt * J;
        }
#pragma omp parallel for schedule(static)
    for (int i = 1; i < nr; i++)
        for (int j = 1; j < nth; j++) {
            double A = darea_ph(s, i, j);
            double circ = s->dth * (s->rh[i] * AT(s, ORA_BTH, i, j) -
                                    s->rh[i - 1] * AT(s, ORA_BTH, i - 1, j)) -
                          (s->rh[i] - s->rh[i - 1]) *
                              (AT(s, ORA_BR, i, j) - AT(s, ORA_BR, i, j - 1));
            double f = AT(s, ORA_F, i, j);
            double J = (1.0 - f) * AT(s, ORA_JPH, i, j) / dvol(s, i, j) + f * JN(2, i, j);
            AT(s, ORA_EPH, i, j) += dt * circ / A - fourpi * dt * J;
        }

    /* force-free E correction at nodes, weighted by f, averaged back */
    if (s->p.ff_enable) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i <= nr; i++)
            for (int j = 0; j <= nth; j++) {
                double f = AT(s, ORA_F, i, j);
                if (!(f > 0.0)) continue;
                double e[3], b[3], o[3];
                node_E(s, i, j, e);
                node_B(s, i, j, b);
                ora_ff_node(e, b, o);
                for (int c = 0; c < 3; c++) DL(c, i, j) = f * (o[c] - e[c]);
            }
#pragma omp parallel for schedule(static)
        for (int i = 0; i < nr; i++)
            for (int j = 0; j <= nth; j++)
                AT(s, ORA_ER, i, j) += 0.5 * (DL(0, i, j) + DL(0, i + 1, j));
#pragma omp parallel for schedule(static)
        for (int i = 1; i < nr; i++)
            for (int j = 0; j < nth; j++)
                AT(s, ORA_ETH, i, j) += 0.5 * (DL(1, i, j) + DL(1, i, j + 1));
#pragma omp parallel for schedule(static)
        for (int i = 1; i < nr; i++)
            for (int j = 1; j < nth; j++)
                AT(s, ORA_EPH, i, j) += DL(2, i, j);
    }

    faraday(s, 0.5 * dt);                               /* B^{n+1} */

    /* absorbing layer beyond r_abs: damp E, relax B to its initial value */
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= nr; i++) {
        double ln = absorb(s, s->rn[i]);
        double lh = i < nr ? absorb(s, s->rh[i]) : 1.0;
        if (ln == 1.0 && lh == 1.0) continue;
        for (int j = 0; j <= nth; j++) {
            if (i < nr) {
                AT(s, ORA_ER, i, j) *= lh;
                AT(s, ORA_BTH, i, j) = AT(s, ORA_B0TH, i, j) +
                    lh * (AT(s, ORA_BTH, i, j) - AT(s, ORA_B0TH, i, j));
                if (j < nth)
                    AT(s, ORA_BPH, i, j) = AT(s, ORA_B0PH, i, j) +
                        lh * (AT(s, ORA_BPH, i, j) - AT(s, ORA_B0PH, i, j));
            }
            AT(s, ORA_EPH, i, j) *= ln;
            if (j < nth) {
                AT(s, ORA_ETH, i, j) *= ln;
                AT(s, ORA_BR, i, j) = AT(s, ORA_B0R, i, j) +
                    ln * (AT(s, ORA_BR, i, j) - AT(s, ORA_B0R, i, j));
            }
        }
    }
    memset(s->F[ORA_JR], 0, nn * sizeof(double));
    memset(s->F[ORA_JTH], 0, nn * sizeof(double));
    memset(s->F[ORA_JPH], 0, nn * sizeof(double));
#undef JN
#undef DL
    free(jn);
    free(del);
}

/* ------------------------------------------------------------------ */

/* ------------------------------------------------------------------ */
/* surface pair injection (Sect. 4, monopole test: pairs injected with
   multiplicity kappa_inj in the first cell layer above the star, PIC
   domain only)                                                        */

/* Philox4x32 with 10 rounds, as defined by Salmon, Moraes, Dror & Shaw
   (2011): each round multiplies words 0 and 2 by two constants, mixes the
   high halves with words 1 and 3 and the key, and the key is bumped by
   two Weyl constants between rounds. */
void ora_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Expected pairs per step in surface cell (0, j): kappa_inj times the
   Goldreich-Julian number density |rho_GJ| / q = Omega |B_r| / (2 pi q)
   (B_r at the cell's lower face, the stellar surface) in the cell volume,
   renewed once per crossing time of the cell at c. */
double ora_inject_rate(const ora_sim *s, int j)
{
    double br = fabs(AT(s, ORA_BR, 0, j));
    double q = s->p.weight[0];
    double vol = (s->rn[1] * s->rn[1] * s->rn[1] - s->rn[0] * s->rn[0] * s->rn[0]) / 3.0 *
                 (s->cn[j] - s->cn[j + 1]);
    return s->p.inject_kappa * (s->omega * br / (2.0 * PI)) / q * vol *
           (s->dt / (s->rn[1] - s->rn[0]));
}

#define INJ_TAG 0x696E6A63u   /* counter word 3 of the injection draws */

static double u01(uint32_t x) { return (double)x * (1.0 / 4294967296.0); }

static void append(struct species *q, double r, double th, double ur, double uth,
                   double uph)
{
    if (q->n + 1 > q->cap) {
        int64_t cap = 2 * q->cap + 16;
        q->r = realloc(q->r, cap * sizeof(double));
        q->th = realloc(q->th, cap * sizeof(double));
        q->ur = realloc(q->ur, cap * sizeof(double));
        q->uth = realloc(q->uth, cap * sizeof(double));
        q->uph = realloc(q->uph, cap * sizeof(double));
        q->cap = cap;
    }
    int64_t d = q->n++;
    q->r[d] = r; q->th[d] = th;
    q->ur[d] = ur; q->uth[d] = uth; q->uph[d] = uph;
}

/* In every surface cell outside the pure force-free domain: floor(N) pairs
   plus one more with probability frac(N), at uniform logical offsets in
   the cell, in corotation (u_phi = gamma Omega r sin theta); the same
   positions for every species (pairs carry no net charge). */
static void inject_pairs(ora_sim *s)
{
    if (!(s->p.inject_kappa > 0.0) || s->p.nspec == 0) return;
    uint32_t key[2] = {(uint32_t)s->p.rng_seed, (uint32_t)(s->p.rng_seed >> 32)};
    uint32_t stp = (uint32_t)s->step;
    for (int j = 0; j < s->nth; j++) {
        if (s->kill[j]) continue;
        double N = ora_inject_rate(s, j);
        double fl = floor(N);
        uint32_t ctr[4] = {stp, (uint32_t)j, 0u, INJ_TAG}, o[4];
        ora_philox4x32(ctr, key, o);
        int n = (int)fl + (u01(o[0]) < N - fl ? 1 : 0);
        for (int p = 0; p < n; p++) {
            uint32_t c2[4] = {stp, (uint32_t)j, (uint32_t)(p + 1), INJ_TAG};
            ora_philox4x32(c2, key, o);
            double a = u01(o[0]), b = u01(o[1]);
            double r = s->rn[0] * exp(a * s->dlog);
            double th = s->thn[j] + b * s->dth;
            double v = s->omega * r * sin(th);
            double uph = v / sqrt(1.0 - v * v);
            for (int k = 0; k < s->p.nspec; k++) append(&s->sp[k], r, th, 0.0, 0.0, uph);
        }
    }
}

/* Goldreich-Julian charge of surface cell (0, j), |rho_GJ| V with
   |rho_GJ| = Omega |B_r| / (2 pi) at the stellar surface, times the
   extraction multiplicity (V per radian of azimuth, as every volume here) */
double ora_gj_target(const ora_sim *s, int j)
{
    double br = fabs(AT(s, ORA_BR, 0, j));
    double vol = (s->rn[1] * s->rn[1] * s->rn[1] - s->rn[0] * s->rn[0] * s->rn[0]) / 3.0 *
                 (s->cn[j] - s->cn[j + 1]);
    return s->p.gj_extract * (s->omega * br / (2.0 * PI)) * vol;
}

#define EXT_TAG 0x676A6578u   /* counter word 3 of the extraction draws */

/* Goldreich-Julian extraction (Sect. 5, dipole): every step, each surface
   cell outside the pure force-free domain whose particles (all species,
   counted by charge magnitude, species in order) hold less than the
   target charge receives ceil(deficit / (w_e + w_i)) electron-ion pairs
   at uniform logical offsets, in corotation, with no poloidal momentum;
   the electron of each pair is appended first. */
static void extract_gj(ora_sim *s)
{
    if (!(s->p.gj_extract > 0.0)) return;
    int nth = s->nth;
    double *have = calloc(nth, sizeof(double));
    for (int k = 0; k < s->p.nspec; k++) {
        struct species *q = &s->sp[k];
        int64_t *cnt = calloc(nth, sizeof(int64_t));
        for (int64_t p = 0; p < q->n; p++) {
            if (!(q->r[p] > 0.0) || !(q->r[p] < s->rn[1])) continue;
            int i, j; double a, b;
            locate(s, q->r[p], q->th[p], &i, &j, &a, &b);
            if (i == 0) cnt[j]++;
        }
        for (int j = 0; j < nth; j++) have[j] += s->p.weight[k] * (double)cnt[j];
        free(cnt);
    }
    int se = s->p.gj_species[0], si = s->p.gj_species[1];
    double wpair = s->p.weight[se] + s->p.weight[si];
    uint32_t key[2] = {(uint32_t)s->p.rng_seed, (uint32_t)(s->p.rng_seed >> 32)};
    uint32_t stp = (uint32_t)s->step;
    for (int j = 0; j < nth; j++) {
        if (s->kill[j]) continue;
        double deficit = ora_gj_target(s, j) - have[j];
        if (!(deficit > 0.0)) continue;
        int n = (int)ceil(deficit / wpair);
        for (int p = 0; p < n; p++) {
            uint32_t ctr[4] = {stp, (uint32_t)j, (uint32_t)(p + 1), EXT_TAG}, o[4];
            ora_philox4x32(ctr, key, o);
            double a = u01(o[0]), b = u01(o[1]);
            double r = s->rn[0] * exp(a * s->dlog);
            double th = s->thn[j] + b * s->dth;
            double v = s->omega * r * sin(th);
            double uph = v / sqrt(1.0 - v * v);
            append(&s->sp[se], r, th, 0.0, 0.0, uph);
            append(&s->sp[si], r, th, 0.0, 0.0, uph);
        }
    }
    free(have);
}

/* Threshold pair creation (Sect. 5): after the push, every electron or
   positron with gamma > gamma_th creates one pair (an electron and a
   positron) at its position, moving along its direction of motion with
   Lorentz factor gamma_s.  The parent keeps its momentum.  Parents are
   taken species by species, in slot order; the pairs are appended in that
   order (the new particles are not parents in the same step). */
static void create_pairs(ora_sim *s)
{
    if (!(s->p.gamma_th > 0.0)) return;
    int se = s->p.pair_species[0], sz = s->p.pair_species[1];
    double gth2 = s->p.gamma_th * s->p.gamma_th;
    double us = sqrt(s->p.gamma_s * s->p.gamma_s - 1.0);
    int64_t n0[2] = {s->sp[se].n, s->sp[sz].n};
    for (int h = 0; h < 2; h++) {
        struct species *q = &s->sp[h == 0 ? se : sz];
        for (int64_t p = 0; p < n0[h]; p++) {
            if (!(q->r[p] > 0.0)) continue;
            double u2 = q->ur[p] * q->ur[p] + q->uth[p] * q->uth[p] + q->uph[p] * q->uph[p];
            if (!(1.0 + u2 > gth2)) continue;
            double f = us / sqrt(u2);
            double r = q->r[p], th = q->th[p];
            double ur = q->ur[p] * f, uth = q->uth[p] * f, uph = q->uph[p] * f;
            append(&s->sp[se], r, th, ur, uth, uph);
            append(&s->sp[sz], r, th, ur, uth, uph);
        }
    }
}

void ora_run_phases(ora_sim *s, int ph)
{
    if (ph & ORA_PHASE_MASK) compute_psi_mask(s);
    if (ph & ORA_PHASE_KILL) kill_masked(s);
    if (ph & ORA_PHASE_SORT)
        for (int k = 0; k < s->p.nspec; k++) sort_species(s, k);
    if (ph & ORA_PHASE_INJECT) inject_pairs(s);
    if (ph & ORA_PHASE_EXTRACT) extract_gj(s);
    if (ph & ORA_PHASE_PUSH)
        for (int k = 0; k < s->p.nspec; k++) push_species(s, k);
    if (ph & ORA_PHASE_PAIRS) create_pairs(s);
    if (ph & ORA_PHASE_FIELDS) field_step(s);
}

void ora_step(ora_sim *s, int nsteps)
{
    for (int n = 0; n < nsteps; n++) {
        int ph = ORA_PHASE_MASK | ORA_PHASE_KILL | ORA_PHASE_INJECT | ORA_PHASE_EXTRACT |
                 ORA_PHASE_PUSH | ORA_PHASE_PAIRS | ORA_PHASE_FIELDS;
        if (s->step % s->p.sort_interval == 0) ph |= ORA_PHASE_SORT;
        ora_run_phases(s, ph);
        s->step++;
    }
}

/* ------------------------------------------------------------------ */
/* diagnostics                                                         */

void ora_moments(const ora_sim *s, int k, double out[5])
{
    const struct species *q = &s->sp[k];
    double n = 0, g = 0, ur = 0, ut = 0, up = 0;
    for (int64_t p = 0; p < q->n; p++) {
        if (!(q->r[p] > 0.0)) continue;
        n += 1.0;
        g += sqrt(1.0 + q->ur[p] * q->ur[p] + q->uth[p] * q->uth[p] + q->uph[p] * q->uph[p]);
        ur += q->ur[p]; ut += q->uth[p]; up += q->uph[p];
    }
    out[0] = n; out[1] = g; out[2] = ur; out[3] = ut; out[4] = up;
}

/* sum over particles of Q S(xi - i) S(eta - j), the node charge whose
   change the deposit's fluxes balance */
/* Synchrotron function F(x) = x * int_x^inf K_{5/3}(s) ds.  With the
   integral representation K_nu(s) = int_0^inf exp(-s cosh t) cosh(nu t) dt
   the s-integral can be done first:
       F(x) = x int_0^inf exp(-x cosh t) cosh(5t/3) / cosh t dt,
   evaluated here with the trapezoidal rule (step 1/40), which converges
   geometrically for this even function, analytic in a strip about the
   real axis, until exp(-x cosh t) underflows. */
double ora_synchrotron_F(double x)
{
    if (!(x > 0.0)) return 0.0;
    const double h = 0.025;
    double sum = 0.0;
    for (int k = 0;; k++) {
        double t = k * h;
        double ch = cosh(t);
        double e = x * ch;
        if (e > 745.0) break;
        double v = exp(-e) * cosh(5.0 * t / 3.0) / ch;
        sum += (k == 0 ? 0.5 : 1.0) * v;
    }
    return x * h * sum;
}

/* Spectra of one species over a region (Sect. 5 observables):
   - dN[m]: summed weight of live particles with rmin <= r < rmax,
     thmin <= theta < thmax and gamma in [g_m, g_m+1), g_m = gmin
     exp(m log(gmax/gmin) / ngamma), gamma = sqrt(1 + u.u);
   - prad: summed w P with P = K gamma^2 Bperp^2, the leading radiated power
     of the radiation-reaction force g (K the coefficient the push applies
     this step, Bperp of eq. bperp from the fields gathered at the particle);
   - sed[k]: summed w nu dP/dnu at nu_k = numin (numax/numin)^(k/(nnu-1)),
     the synchrotron spectrum of each particle normalised to P:
     nu dP/dnu = P x F(x) 9 sqrt(3) / (8 pi), x = nu / nu_c,
     nu_c = 3/(4 pi) gamma^2 omega_b |qm| Bperp (gyro-frequency omega_b |qm| B
     in code units). */
void ora_spectra(const ora_sim *s, int k, const ora_spec_req *rq, double *dN, double *sed,
                 double *prad)
{
    const struct species *q = &s->sp[k];
    double qm = s->p.qm[k], w = s->p.weight[k];
    double K = s->p.rr_coef * ora_rr_factor(&s->p, (double)s->step * s->dt) *
               fabs(qm) * fabs(qm) * fabs(qm);
    double dlg = log(rq->gmax / rq->gmin) / rq->ngamma;
    double *edge = malloc((rq->ngamma + 1) * sizeof(double));
    for (int m = 0; m <= rq->ngamma; m++) edge[m] = rq->gmin * exp(m * dlg);
    double *nu = malloc(rq->nnu * sizeof(double));
    for (int m = 0; m < rq->nnu; m++)
        nu[m] = rq->nnu > 1 ? rq->numin * exp(m * log(rq->numax / rq->numin) / (rq->nnu - 1))
                            : rq->numin;
    for (int m = 0; m < rq->ngamma; m++) dN[m] = 0.0;
    for (int m = 0; m < rq->nnu; m++) sed[m] = 0.0;
    double ptot = 0.0;
    for (int64_t p = 0; p < q->n; p++) {
        double r = q->r[p], th = q->th[p];
        if (!(r > 0.0)) continue;
        if (!(r >= rq->rmin && r < rq->rmax && th >= rq->thmin && th < rq->thmax)) continue;
        double u[3] = {q->ur[p], q->uth[p], q->uph[p]};
        double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int m = 0; m < rq->ngamma; m++)
            if (g >= edge[m] && g < edge[m + 1]) dN[m] += w;
        double E[3], B[3];
        ora_gather(s, r, th, E, B);
        double beta[3] = {u[0] / g, u[1] / g, u[2] / g}, bxB[3], F[3];
        cross3(beta, B, bxB);
        for (int c = 0; c < 3; c++) F[c] = E[c] + bxB[c];
        double be = dot3(beta, E);
        double bp2 = dot3(F, F) - be * be;
        if (bp2 < 0.0) bp2 = 0.0;
        double P = K * g * g * bp2;
        ptot += w * P;
        double nuc = 3.0 / (4.0 * PI) * g * g * s->p.omega_b * fabs(qm) * sqrt(bp2);
        if (!(nuc > 0.0) || !(P > 0.0)) continue;
        for (int m = 0; m < rq->nnu; m++) {
            double x = nu[m] / nuc;
            sed[m] += w * P * x * ora_synchrotron_F(x) * 9.0 * sqrt(3.0) / (8.0 * PI);
        }
    }
    *prad = ptot;
    free(edge);
    free(nu);
}

void ora_node_charge(const ora_sim *s, double *qn)
{
    memset(qn, 0, s->nn * sizeof(double));
    for (int k = 0; k < s->p.nspec; k++) {
        const struct species *q = &s->sp[k];
        double Q = (s->p.qm[k] > 0 ? 1.0 : -1.0) * s->p.weight[k];
        for (int64_t p = 0; p < q->n; p++) {
            if (!(q->r[p] > 0.0)) continue;
            int i, j; double a, b;
            locate(s, q->r[p], q->th[p], &i, &j, &a, &b);
            qn[(size_t)i * s->ld + j] += Q * (1.0 - a) * (1.0 - b);
            qn[(size_t)(i + 1) * s->ld + j] += Q * a * (1.0 - b);
            qn[(size_t)i * s->ld + j + 1] += Q * (1.0 - a) * b;
            qn[(size_t)(i + 1) * s->ld + j + 1] += Q * a * b;
        }
    }
}

/* Gauss-law residual div E - 4 pi rho at interior nodes */
void ora_gauss(const ora_sim *s, double *g)
{
    double *qn = malloc(s->nn * sizeof(double));
    ora_node_charge(s, qn);
    memset(g, 0, s->nn * sizeof(double));
    for (int i = 1; i < s->nr; i++)
        for (int j = 0; j <= s->nth; j++)
            g[(size_t)i * s->ld + j] = div_E(s, i, j) -
                4.0 * PI * qn[(size_t)i * s->ld + j] / dvol(s, i, j);
    free(qn);
}

/* div B over primal cells */
void ora_divb(const ora_sim *s, double *d)
{
    memset(d, 0, s->nn * sizeof(double));
    for (int i = 0; i < s->nr; i++)
        for (int j = 0; j < s->nth; j++) {
            double flux = area_r(s, i + 1, j) * AT(s, ORA_BR, i + 1, j) -
                          area_r(s, i, j) * AT(s, ORA_BR, i, j) +
                          area_th(s, i, j + 1) * AT(s, ORA_BTH, i, j + 1) -
                          area_th(s, i, j) * AT(s, ORA_BTH, i, j);
            double v = (s->rn[i + 1] * s->rn[i + 1] * s->rn[i + 1] -
                        s->rn[i] * s->rn[i] * s->rn[i]) / 3.0 *
                       (s->cn[j] - s->cn[j + 1]);
            d[(size_t)i * s->ld + j] = flux / v;
        }
}

/* Poynting flux through the sphere r_i: (c/4 pi) * 2 pi *
   int (E_th B_ph - E_ph B_th) r^2 sin(theta) dtheta */
void ora_poynting(const ora_sim *s, double *L)
{
    for (int i = 0; i <= s->nr; i++) {
        if (i == 0 || i == s->nr) { L[i] = 0.0; continue; }
        double acc = 0.0;
        for (int j = 0; j < s->nth; j++) {
            double bph = 0.5 * (AT(s, ORA_BPH, i - 1, j) + AT(s, ORA_BPH, i, j));
            acc += AT(s, ORA_ETH, i, j) * bph * (s->cn[j] - s->cn[j + 1]);
        }
        for (int j = 0; j <= s->nth; j++) {
            double bth = 0.5 * (AT(s, ORA_BTH, i - 1, j) + AT(s, ORA_BTH, i, j));
            acc -= AT(s, ORA_EPH, i, j) * bth * (cos_lo(s, j) - cos_hi(s, j));
        }
        L[i] = 0.5 * s->rn[i] * s->rn[i] * acc;
    }
}
