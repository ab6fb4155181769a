/*
 * Plain FP64 CPU oracle of one hybrid force-free / PIC time step on an
 * axisymmetric (r, theta) Yee grid (Soudais, Cerutti & Contopoulos 2024,
 * Sect. 3).  TEST INFRASTRUCTURE ONLY: it exists to check the GPU library;
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code with the GPU path.
 *
 * Storage: every field component lives in an (nr+1) x (nth+1) node-shaped
 * array, theta fastest, index i*(nth+1)+j.  Component positions (Yee):
 *   E_r (i+1/2, j)   E_th (i, j+1/2)   E_ph (i, j)
 *   B_r (i, j+1/2)   B_th (i+1/2, j)   B_ph (i+1/2, j+1/2)
 *   J like E; Psi and f at nodes.  Entry [i][j] holds the value at the
 *   position whose lower corner is node (i, j); unused entries stay zero.
 * Particles: per species, FP64 (r, theta, u_r, u_theta, u_phi); a dead slot
 * has r = -1 until the next sort compacts it away.
 *
 * What pins each part (tests/test_oracle_pins.py, tests/test_oracle_kinematics.py,
 * tests/golden/; tests/test_oracle_mutations.py checks that planted mistakes
 * in the push's frame changes, move and azimuthal deposit fail these pins):
 *   push frame changes and move: free streaming follows the 3-D straight
 *   line (also across the equator and past the poles), a uniform E along the
 *   axis accelerates u_z linearly, gyration in a uniform B0 z built from
 *   nodal Psi follows the discrete orbit to second order, the azimuthal
 *   E x B drift -E0/B0; azimuthal deposit: total Q v_phi centred on the
 *   move's midpoint, its density integrating to the ring current Q v_phi /
 *   varpi;
 *   time step and radial spacing: Table 1 values; Boris rotation: the exact
 *   discrete rotation angle and |u| conservation; E x B drift; radiation
 *   reaction: closed-form cooling, first-order convergence; flux function:
 *   telescoping of B built from nodal Psi (three inits), second-order
 *   dipole; blending function: equality cases and linear bands; force-free
 *   node correction: E.B = 0, |E| <= |B|, idempotence; gather: exact for
 *   linear fields, axis parity; deposit + Ampere: discrete Gauss law kept
 *   to roundoff; Faraday: div B kept to roundoff; corotation E curl-free;
 *   sort: stability; Michel monopole: stationary to second order, and a
 *   vacuum monopole spinning up to Michel's luminosity; Philox: published
 *   known answers; injection: closed-form rate, binomial counts, Gauss law;
 *   radiation-reaction ramp: its knots and linear pieces; shell: momentum
 *   left along B only (a particle gyrating across B stops, |u| kept
 *   outside); extraction: closed-form dipole charge per cell, top-up of a
 *   partly filled cell, Gauss law; pair creation: one pair per parent above
 *   threshold per step, at its position, along its motion, with gamma_s.
 * Parity unpinned (defined here and checked GPU against oracle only, no
 * closed form behind them): the blend of J at staggered points (mean of
 * the adjacent node f), averaging the correction back from nodes rather
 * than E itself, the absorbing-layer profile, the opened-dipole initial
 * field, and the placement of the radiation-reaction kick after the Boris
 * rotation (its first-order convergence is pinned, its ordering is not).
 * The paper leaves these choices of the plasma sources open; the pins check
 * that the code does what the choice says, not the choice itself: the
 * extraction's top-up rule (all species' charge counted, ceil of the
 * deficit over a pair's charge), the parent keeping its momentum when it
 * creates a pair, the shell projection placed after the radiation-reaction
 * kick, and the knots of the ramp.
 */
#ifndef FFPIC_ORACLE_H
#define FFPIC_ORACLE_H
#include <stdint.h>

#define ORA_MAXSPEC 4

typedef struct {
    int nr, nth;
    double rmin, rmax, r_lc, r_abs, mu, cfl, omega_b, rr_coef;
    double psi_thr[4];
    int ff_enable, init, sort_interval, nspec;
    double qm[ORA_MAXSPEC], weight[ORA_MAXSPEC];
    double inject_kappa;      /* surface pair injection multiplicity (0 = off) */
    uint64_t rng_seed;        /* key of the counter-based generator */
    /* plasma sources of the dipole (Sect. 5) */
    int rr_ramp_n;            /* knots of the radiation-reaction ramp (0 = off) */
    double rr_ramp_t[4];      /* knot times, non-decreasing */
    double rr_ramp_f[4];      /* factor on rr_coef at each knot */
    double shell_r;           /* r < shell_r: transverse momentum removed (0 = off) */
    double gj_extract;        /* Goldreich-Julian extraction multiplicity (0 = off) */
    int gj_species[2];        /* extracted electron and ion species */
    double gamma_th, gamma_s; /* threshold pair creation (gamma_th = 0: off) */
    int pair_species[2];      /* electron and positron species (parents and pairs) */
} ora_params;

enum { ORA_ER, ORA_ETH, ORA_EPH, ORA_BR, ORA_BTH, ORA_BPH,
       ORA_JR, ORA_JTH, ORA_JPH, ORA_PSI, ORA_F,
       ORA_B0R, ORA_B0TH, ORA_B0PH, ORA_NCOMP };

enum { ORA_PHASE_MASK = 1, ORA_PHASE_KILL = 2, ORA_PHASE_SORT = 4,
       ORA_PHASE_PUSH = 8, ORA_PHASE_FIELDS = 16, ORA_PHASE_INJECT = 32,
       ORA_PHASE_EXTRACT = 64, ORA_PHASE_PAIRS = 128 };

typedef struct ora_sim ora_sim;

ora_sim *ora_create(const ora_params *p);
double ora_timestep(const ora_params *p);
void ora_destroy(ora_sim *s);
/* out: dt, dlog, dth, omega */
void ora_info(const ora_sim *s, double out[4]);
void ora_get_field(const ora_sim *s, int comp, double *dst);
/* geometry tables: 0 r_i, 1 r_{i+1/2}, 2 theta_j, 3 sin theta_j,
   4 cos theta_j, 5 sin theta_{j+1/2}, 6 cos theta_{j+1/2} */
void ora_geometry(const ora_sim *s, int which, double *dst);
void ora_set_field(ora_sim *s, int comp, const double *src);
/* appends, then removes out-of-domain and masked particles and sorts;
   returns the number of particles of that species after loading */
int64_t ora_load_particles(ora_sim *s, int sp, int64_t n, const double *r,
                           const double *th, const double *ur,
                           const double *uth, const double *uph);
int64_t ora_num_particles(const ora_sim *s, int sp);
/* copies all slots; cell = i*nth + j, or -1 for a dead slot */
int64_t ora_get_particles(const ora_sim *s, int sp, double *r, double *th,
                          double *ur, double *uth, double *uph, int32_t *cell);
void ora_step(ora_sim *s, int nsteps);
/* threads of the OpenMP build (the single-thread build ignores it, and
   reports 1) */
void ora_set_threads(int n);
int ora_threads(void);
/* Philox4x32-10 counter-based generator (Salmon et al. 2011): out = the
   four 32-bit words for counter ctr and key */
void ora_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* expected number of injected pairs per step in surface cell (0, j) */
double ora_inject_rate(const ora_sim *s, int j);
/* Goldreich-Julian charge of surface cell (0, j) times the extraction
   multiplicity: the charge the extraction keeps the cell at */
double ora_gj_target(const ora_sim *s, int j);
/* factor on the radiation-reaction coefficient at time t */
double ora_rr_factor(const ora_params *p, double t);
void ora_run_phases(ora_sim *s, int phases);
int64_t ora_step_count(const ora_sim *s);
void ora_set_step(ora_sim *s, int64_t step);   /* test hook: the step counter */
/* removed[cause] for cause = 0 load, 1 force-free kill, 2 star, 3 absorber */
void ora_removed(const ora_sim *s, int sp, int64_t out[4]);

/* diagnostics */
void ora_moments(const ora_sim *s, int sp, double out[5]);
void ora_gauss(const ora_sim *s, double *g);      /* node map */
void ora_divb(const ora_sim *s, double *d);       /* primal-cell map */
void ora_node_charge(const ora_sim *s, double *q);/* sum Q S S per node */
void ora_poynting(const ora_sim *s, double *L);   /* nr+1 radii */
void ora_sort_offsets(const ora_sim *s, int sp, int32_t *off);
/* species spectra over a region: gamma histogram, radiated power and the
   synchrotron SED (see the definition in the source) */
typedef struct {
    double rmin, rmax, thmin, thmax;   /* region: rmin <= r < rmax, thmin <= theta < thmax */
    double gmin, gmax;                 /* ngamma log-spaced gamma bins */
    double numin, numax;               /* nnu log-spaced frequencies (code units) */
    int ngamma, nnu;
} ora_spec_req;
void ora_spectra(const ora_sim *s, int sp, const ora_spec_req *req, double *dN,
                 double *sed, double *prad);
/* synchrotron function x int_x^inf K_{5/3} */
double ora_synchrotron_F(double x);

/* pieces exported for the closed-form pins */
void ora_boris_rr(double u[3], const double E[3], const double B[3],
                  double dt, double omega_b_qm, double rr);
void ora_ff_node(const double E[3], const double B[3], double out[3]);
double ora_blend(double psi, const double thr[4]);
void ora_gather(const ora_sim *s, double r, double th, double E[3], double B[3]);

#endif
