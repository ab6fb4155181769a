/*
 * ffpic.h -- C ABI of the MI355X hybrid force-free / particle-in-cell step
 * for axisymmetric pulsar magnetospheres (Soudais, Cerutti & Contopoulos
 * 2024, "Scaling up global kinetic models of pulsar magnetospheres using a
 * hybrid force-free-PIC numerical approach", Sect. 3).
 *
 * One call of ffpic_step advances one magnetosphere by n time steps on the
 * GPU.  Each time step is (Sect. 3):
 *   - the flux function Psi of eq. (psi) and the blending function f(Psi)
 *     of eq. (transition), rebuilt from the current B_r every step;
 *   - removal of particles from cells inside the pure force-free domain;
 *   - every sort_interval steps, a stable sort of each species by cell;
 *   - optional plasma sources: surface pair injection (Sect. 4) and
 *     Goldreich-Julian extraction of electrons and ions (Sect. 5);
 *   - the particle push of eq. (motion) with the radiation-reaction force
 *     g and the effective field of eq. (bperp), a modified Boris scheme;
 *   - a charge-conserving current deposit;
 *   - optional threshold pair creation by the pushed leptons (Sect. 5);
 *   - the Yee/FDTD field update of eqs. (faraday) and (ampere) with the
 *     blended current of eq. (blending), whose force-free part is the
 *     drift current of eq. (JFFE), followed by the force-free E correction
 *     (E.B projection and the cap |E| <= |B|) on the force-free domain;
 *   - the corotation condition on the star and the absorbing layer of
 *     Sect. 4.
 *
 * Units: c = 1, lengths in stellar radii, Omega = 1 / r_lc.
 *
 * Grid: nr x nth cells, r log-spaced on [rmin, rmax], theta uniform on
 * [0, pi] (Sect. 4).  Every field component is exchanged as an
 * (nr+1) x (nth+1) node-shaped array of doubles, theta fastest
 * (index i*(nth+1) + j).  Entry [i][j] of a component holds its value at
 * the staggered position whose lower corner is node (i, j):
 *   E_r (i+1/2, j)   E_th (i, j+1/2)   E_ph (i, j)
 *   B_r (i, j+1/2)   B_th (i+1/2, j)   B_ph (i+1/2, j+1/2)
 * Entries with no position (e.g. E_r[nr][*]) are zero.
 *
 * Errors: every int-returning call returns FFPIC_OK (0) or a negative
 * status; ffpic_last_error() then describes the failure.  Errors raised by
 * kernels (non-finite momenta, a particle moving a whole cell in a step) are
 * recorded in a device error word and reported by the next synchronising
 * call (ffpic_sync, ffpic_get_*, ffpic_diagnostics).  No C++ exception
 * crosses this boundary.  A context is not thread-safe; use one context per
 * stream.
 */
#ifndef FFPIC_H
#define FFPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFPIC_MAX_SPECIES 4

enum ffpic_status {
    FFPIC_OK = 0,
    FFPIC_EINVAL = -1,    /* invalid argument or descriptor */
    FFPIC_ENOMEM = -2,    /* device or host allocation failed */
    FFPIC_EHIP = -3,      /* a HIP runtime call failed */
    FFPIC_ECAPACITY = -4, /* more particles than the species capacity */
    FFPIC_ENUMERIC = -5,  /* a kernel met a non-finite value or a CFL breach */
    FFPIC_ESTATE = -6     /* call not valid in the current state */
};

enum ffpic_precision {
    FFPIC_FP64 = 0,       /* fields, particles and currents in FP64 */
    FFPIC_FP32_MIXED = 1  /* int32 cell + FP32 in-cell offsets, FP32 momenta,
                             fields and currents; FP64 Psi and residuals */
};

enum ffpic_init {
    FFPIC_INIT_ZERO = 0,        /* all fields zero (load them yourself) */
    FFPIC_INIT_DIPOLE = 1,      /* Psi = mu sin^2(theta)/r, eq. (flux_dipole) */
    FFPIC_INIT_MONOPOLE = 2,    /* Psi = mu (1 - cos theta), Sect. 4 */
    FFPIC_INIT_MICHEL = 3,      /* monopole plus Michel B_phi, Sect. 4 */
    FFPIC_INIT_OPEN_DIPOLE = 4  /* dipole inside the light cylinder with the
                                   lines crossing it opened to a split monopole */
};
/* Every non-zero init sets poloidal B from nodal Psi differences (exactly
   divergence-free) and the corotation field E = -(Omega x r) x B in edge form
   (E = -Omega grad Psi); E_th and E_ph on the star stay at these values
   (corotation boundary, Sect. 4); E_th = E_ph = 0 on r = rmax. */

enum ffpic_component {
    FFPIC_ER = 0, FFPIC_ETH, FFPIC_EPH,
    FFPIC_BR, FFPIC_BTH, FFPIC_BPH,
    /* deposit accumulators of the last push (zeroed by the field update):
       JR = radial charge flux through dual faces over the step, JTH = polar
       charge flux, JPH = sum of Q v_phi S_xi S_eta per node (Q = charge) */
    FFPIC_JR, FFPIC_JTH, FFPIC_JPH,
    FFPIC_PSI,            /* flux function at nodes (FP64 in both modes) */
    FFPIC_F,              /* blending function at nodes */
    FFPIC_GAUSS,          /* node map of div E - 4 pi rho (read only) */
    FFPIC_DIVB,           /* primal-cell map of div B (read only) */
    FFPIC_NCOMP
};

/* Descriptor of one magnetosphere.  Reading of the paper's parameters:
   star and light cylinder (Sect. 2, 4), grid and CFL (Sect. 4, Table 1),
   species charge-to-mass and weight (Sect. 3, Table 1), force-free / PIC
   flux thresholds (eq. transition, Table 1), radiation-reaction strength
   (Sect. 3, Sect. 5.1 f_rad), absorbing layer (Sect. 4). */
typedef struct ffpic_desc {
    int32_t nr, nth;          /* cells in r and theta, each in [2, 65535] */
    double rmin, rmax;        /* radial extent, 0 < rmin < rmax */
    double r_lc;              /* light-cylinder radius; Omega = 1 / r_lc */
    double r_abs;             /* absorbing layer starts here; rmin < r_abs <= rmax */
    double mu;                /* dipole moment, or Psi_star for the monopoles */
    double cfl;               /* in (0, 1]: dt = cfl / sqrt(1/dr0^2 + 1/(r0 dth)^2) */
    double omega_b;           /* Lorentz coupling: du/dt = omega_b qm (E + beta x B) */
    double rr_coef;           /* radiation-reaction coefficient K_e (0 = off) */
    double psi_thr[4];        /* Psi_0 <= Psi_1 <= Psi_2 <= Psi_3 (+-inf allowed):
                                 f = 1 for Psi < Psi_0 and Psi >= Psi_3, linear on
                                 (Psi_0, Psi_1) and (Psi_2, Psi_3), 0 between */
    int32_t ff_enable;        /* 0: pure PIC (f = 0 everywhere) */
    int32_t precision;        /* enum ffpic_precision */
    int32_t init;             /* enum ffpic_init */
    int32_t sort_interval;    /* >= 1; 0 = the tuned values (see ffpic_autotune) */
    int32_t nspec;            /* 0 .. FFPIC_MAX_SPECIES */
    int32_t pad_;
    int64_t capacity[FFPIC_MAX_SPECIES]; /* particle slots per species */
    double qm[FFPIC_MAX_SPECIES];     /* charge-to-mass in units of e/m_e
                                         (-1 electrons, +1 positrons, 1/1836 protons) */
    double weight[FFPIC_MAX_SPECIES]; /* macro-particle charge magnitude */
    double inject_kappa;      /* surface pair injection (Sect. 4, monopole test):
                                 multiplicity kappa_inj, 0 = off.  Every step,
                                 each surface cell (i = 0) outside the pure
                                 force-free domain receives on average
                                 kappa_inj |rho_GJ| V / (q c^-1 dr0 / dt) pairs,
                                 |rho_GJ| = Omega |B_r| / 2 pi at the surface,
                                 q = weight[0]: floor(N) pairs plus one with
                                 probability frac(N), at uniform in-cell offsets,
                                 in corotation, one particle of every species
                                 at each position */
    uint64_t rng_seed;        /* key of the Philox4x32-10 generator of the
                                 injection draws (counter = step, cell, draw) */
    /* Plasma sources of the aligned dipole (Sect. 5).  All zero = off. */
    int32_t rr_ramp_n;        /* 0..4 knots of the radiation-reaction ramp:
                                 rr_coef is scaled by a factor that is
                                 piecewise linear through (rr_ramp_t[k],
                                 rr_ramp_f[k]) at t = step * dt, constant
                                 before the first knot and after the last
                                 (times non-decreasing, factors >= 0) */
    int32_t pad2_;
    double rr_ramp_t[4];
    double rr_ramp_f[4];
    double shell_r;           /* r < shell_r (the old position): after the
                                 Boris rotation and radiation reaction only
                                 the momentum along the local B is kept;
                                 0 = off */
    double gj_extract;        /* Goldreich-Julian extraction multiplicity,
                                 0 = off.  Every step, each surface cell
                                 (i = 0) outside the pure force-free domain
                                 holding less charge (sum over all species of
                                 weight x live particles) than
                                 gj_extract |rho_GJ| V (|rho_GJ| = Omega |B_r| /
                                 2 pi at the surface, V per radian of azimuth)
                                 receives ceil(deficit / (w_e + w_i)) pairs of
                                 an electron and an ion at uniform in-cell
                                 offsets (Philox draws, counter word 3 =
                                 0x676A6578), in corotation */
    int32_t gj_species[2];    /* extracted electron and ion species */
    double gamma_th;          /* pair creation threshold, 0 = off: after the
                                 push every particle of pair_species[0] or
                                 pair_species[1] with gamma > gamma_th adds
                                 one particle to each of the two species at
                                 its position, moving along its momentum
                                 with Lorentz factor gamma_s (parent kept;
                                 parents in species order, then slot order) */
    double gamma_s;           /* 1 <= gamma_s < gamma_th */
    int32_t pair_species[2];  /* electron and positron species */
} ffpic_desc;

typedef struct ffpic_diag {
    int64_t step;                         /* steps taken */
    int64_t alive[FFPIC_MAX_SPECIES];
    int64_t removed[FFPIC_MAX_SPECIES][4]; /* causes: 0 load, 1 force-free
                                              domain, 2 star, 3 absorber */
    double sum_gamma[FFPIC_MAX_SPECIES];
    double sum_u[FFPIC_MAX_SPECIES][3];   /* sums of u_r, u_theta, u_phi */
    double energy_e, energy_b;            /* sum of E^2 / 8pi, B^2 / 8pi times
                                             cell volume (2 pi dropped) */
    double gauss_max;                     /* max |div E - 4 pi rho| over interior nodes */
    double divb_max;                      /* max |div B| over primal cells */
    uint32_t error_word;                  /* device error bits (FFPIC_ERR_*) */
    uint32_t pad_;
} ffpic_diag;

#define FFPIC_ERR_NONFINITE 1u  /* non-finite momentum after a push */
#define FFPIC_ERR_CFL 2u        /* a particle crossed more than one cell */
#define FFPIC_ERR_CAPACITY 4u   /* injection, extraction or pair creation
                                   would exceed a species' capacity (nothing
                                   added by that phase in that step) */

#define FFPIC_DIAG_MOMENTS 1u
#define FFPIC_DIAG_ENERGY 2u
#define FFPIC_DIAG_RESIDUALS 4u
#define FFPIC_DIAG_POYNTING 8u
#define FFPIC_DIAG_ALL 15u

typedef struct ffpic_ctx ffpic_ctx;
typedef struct ffpic_batch ffpic_batch;

/* Validates d, builds the FP64 geometry tables, allocates all device memory
   (owned by the context), sets the initial fields and the mask.  `stream` is
   a hipStream_t borrowed for the life of the context (NULL = default
   stream).  On success *out receives the context.  EINVAL for a bad
   descriptor, ENOMEM, EHIP. */
int ffpic_create(const ffpic_desc *d, void *stream, ffpic_ctx **out);

/* Releases everything the context owns.  NULL is ignored. */
void ffpic_destroy(ffpic_ctx *ctx);

/* Message of the last failed call on this context (owned by the context,
   valid until its next call); a static string for ctx == NULL. */
const char *ffpic_last_error(const ffpic_ctx *ctx);

/* out[0..3] = dt, dlog, dtheta, Omega. */
int ffpic_info(const ffpic_ctx *ctx, double out[4]);

/* Replaces one field component (FFPIC_ER .. FFPIC_BPH) from an
   (nr+1)*(nth+1) FP64 array in host memory (src_on_device = 0) or device
   memory (1); the caller keeps ownership.  Loading a B component also makes
   it the reference state of the absorbing layer and rebuilds Psi and f. */
int ffpic_load_fields(ffpic_ctx *ctx, int comp, const double *src, int src_on_device);

/* Appends n particles of `species` given as FP64 arrays (r, theta, u_r,
   u_theta, u_phi) with u = gamma v / c, in host or device memory.
   Particles outside [rmin, r_abs) or theta outside [0, pi], with a
   non-finite value, or in a cell of the pure force-free domain are dropped
   (counted as removed at load); the species is then sorted by cell.
   ECAPACITY if the slots would overflow (nothing is loaded), EINVAL. */
int ffpic_load_particles(ffpic_ctx *ctx, int species, int64_t n, const double *r,
                         const double *th, const double *ur, const double *uth,
                         const double *uph, int src_on_device);

/* Advances nsteps time steps, asynchronously on the context's stream; no
   call reads from the device or waits for it (see ffpic_set_graph). */
int ffpic_step(ffpic_ctx *ctx, int32_t nsteps);

/* Test hook: runs single phases of a step without advancing the step
   counter (bit mask of FFPIC_PHASE_*), in the order mask, kill, sort,
   inject, extract, push, pairs, fields. */
#define FFPIC_PHASE_MASK 1u
#define FFPIC_PHASE_KILL 2u
#define FFPIC_PHASE_SORT 4u
#define FFPIC_PHASE_PUSH 8u
#define FFPIC_PHASE_FIELDS 16u
#define FFPIC_PHASE_INJECT 32u
#define FFPIC_PHASE_EXTRACT 64u
#define FFPIC_PHASE_PAIRS 128u
int ffpic_run_phases(ffpic_ctx *ctx, uint32_t phases);

/* Waits for the stream and returns the first recorded device error
   (ENUMERIC) or FFPIC_OK. */
int ffpic_sync(ffpic_ctx *ctx);

/* Copies one component (FFPIC_ER .. FFPIC_DIVB) as FP64 into an
   (nr+1)*(nth+1) caller buffer in host (0) or device (1) memory.
   Synchronises. */
int ffpic_get_field(ffpic_ctx *ctx, int comp, double *dst, int dst_on_device);

/* Number of particle slots of a species (live ones, plus dead slots not yet
   removed by a sort).  Synchronises. */
int ffpic_num_particles(ffpic_ctx *ctx, int species, int64_t *n);

/* Copies the particle slots of a species to host buffers of at least
   ffpic_num_particles entries (any pointer may be NULL).  cell = i*nth + j,
   or -1 for a dead slot.  Synchronises. */
int ffpic_get_particles(ffpic_ctx *ctx, int species, double *r, double *th,
                        double *ur, double *uth, double *uph, int32_t *cell);

/* As ffpic_get_particles for the slots [first, first + count) only; the
   range is clipped to the current slots and *count receives the number
   copied.  After a sort the slots of a range of cells are contiguous
   (ffpic_get_sort), so a band of cells can be read without copying the
   whole species.  EINVAL for a negative first or count.  Synchronises. */
int ffpic_get_particles_range(ffpic_ctx *ctx, int species, int64_t first, int64_t *count,
                              double *r, double *th, double *ur, double *uth, double *uph,
                              int32_t *cell);

/* Test hook: the current order of a species as cell offsets (nr*nth + 1
   int32 to host memory): cell_offsets[k] = number of live particles with
   cell < k (the particles are in cell order right after a sort).  perm
   (nullable, host memory) receives the permutation of the species' last
   sort: perm[k] = the slot, before that sort, of the particle now in slot
   k, for k below the live count after that sort, which goes to *nperm
   (nullable; call with perm NULL first to size it).  The sort is the
   stable sort by cell of Sect. 3's particle loop, dead and removed
   particles dropped.  Recording costs one 4-byte write per particle and
   sort and is off unless ffpic_record_sort(ctx, 1) was called before the
   sort; EINVAL for perm or nperm when the last sort of that species was
   not recorded, for a species out of range or NULL offsets.  Synchronises. */
int ffpic_get_sort(ffpic_ctx *ctx, int species, int32_t *cell_offsets, int32_t *perm,
                   int64_t *nperm);

/* Turns the recording of the sort permutation (see ffpic_get_sort) on or
   off for the sorts that follow; turning it on allocates one int32 per
   particle slot of every species.  Not to be called while a step is being
   captured. */
int ffpic_record_sort(ffpic_ctx *ctx, int on);

/* Test hooks, host only (no device is touched, no context is made): what
   ffpic_create builds on the host for descriptor d, so that it can be
   checked without a GPU.
   ffpic_host_table copies the FP64 geometry table `table` (FFPIC_TAB_*) to
   out (nullable) and its length to *n.  The grid of Sect. 4: r_i = rmin
   exp(i dlog), dlog = ln(rmax/rmin)/nr, theta_j = j pi/nth; half points at
   i+1/2 and j+1/2; the dual cell of node (i, j) spans [r_lo, r_hi] x
   [theta_lo, theta_hi] (half points, clipped to the grid ends and to
   [0, pi] on the axis).
   ffpic_host_initial_field copies initial field component comp
   (FFPIC_ER .. FFPIC_BPH) as an (nr+1)*(nth+1) node-shaped FP64 array.
   EINVAL for a rejected descriptor, a table or component out of range or a
   NULL pointer. */
enum ffpic_table {
    FFPIC_TAB_RN = 0,   /* r_i [nr+1] */
    FFPIC_TAB_RH,       /* r_{i+1/2} [nr] */
    FFPIC_TAB_RN2,      /* r_i^2 [nr+1] */
    FFPIC_TAB_RH2,      /* r_{i+1/2}^2 [nr] */
    FFPIC_TAB_DRN,      /* r_{i+1} - r_i [nr] */
    FFPIC_TAB_DRH,      /* r_{i+1/2} - r_{i-1/2} [nr+1], 0 at both ends */
    FFPIC_TAB_DR2N,     /* (r_{i+1}^2 - r_i^2)/2 [nr] */
    FFPIC_TAB_DR2H,     /* (r_hi^2 - r_lo^2)/2 [nr+1] */
    FFPIC_TAB_DR3H,     /* (r_hi^3 - r_lo^3)/3 [nr+1] */
    FFPIC_TAB_DR3N,     /* (r_{i+1}^3 - r_i^3)/3 [nr] */
    FFPIC_TAB_LAMN,     /* absorber factor at r_i [nr+1] */
    FFPIC_TAB_LAMH,     /* absorber factor at r_{i+1/2} [nr] */
    FFPIC_TAB_SN,       /* sin theta_j [nth+1], 0 at both poles */
    FFPIC_TAB_CN,       /* cos theta_j [nth+1], +1 and -1 at the poles */
    FFPIC_TAB_SH,       /* sin theta_{j+1/2} [nth] */
    FFPIC_TAB_DCN,      /* cos theta_j - cos theta_{j+1} [nth] */
    FFPIC_TAB_DCD,      /* cos theta_lo - cos theta_hi [nth+1] */
    FFPIC_TAB_DTHD,     /* theta_hi - theta_lo [nth+1] */
    FFPIC_TAB_THN,      /* theta_j [nth+1] */
    FFPIC_NTAB
};
int ffpic_host_table(const ffpic_desc *d, int table, double *out, int64_t *n);
int ffpic_host_initial_field(const ffpic_desc *d, int comp, double *out);

/* Diagnostics selected by `what` (FFPIC_DIAG_*); L_of_r (nullable, nr+1
   doubles, host) receives the Poynting flux through each sphere r_i
   (Sect. 4, eq. michel_spindown form).  Synchronises. */
int ffpic_diagnostics(ffpic_ctx *ctx, uint32_t what, ffpic_diag *out, double *L_of_r);

/* For callers that cannot allocate device memory (code that must not call
   hipMalloc, tight serving loops, harnesses that forbid allocation): the
   same diagnostics as ffpic_diagnostics, same arguments and results, with
   no device allocation.  Its device scratch (partial sums, result slots,
   the node charge map of the Gauss residual, L(r)) is one static 32 MiB
   array per GPU, held until the process ends.  The Gauss residual
   (FFPIC_DIAG_RESIDUALS) needs nn = (nr+1)(nth+1) doubles of it: EINVAL,
   with the limit in ffpic_last_error, for a grid of more than about 4.1
   million nodes; the other diagnostics have no size limit.  EINVAL also
   when the context's device is not the current device.  Calls on one GPU
   share the array: calls that overlap in time (several host threads) race
   on it.  Synchronises. */
int ffpic_diagnostics_noalloc(ffpic_ctx *ctx, uint32_t what, ffpic_diag *out, double *L_of_r);

/* Spectra of one species over a region of the meridional plane (the
   observables of Sect. 5: particle energy spectra and the synchrotron
   spectral energy distribution).  A live particle counts when
   rmin <= r < rmax and thmin <= theta < thmax.  With w the species' weight,
   gamma = sqrt(1 + u.u) and Bperp of eq. (bperp) from E and B gathered at
   the particle as in the push:
     dN[m]  (ngamma doubles, host): summed w of the particles with gamma in
            [gmin (gmax/gmin)^(m/ngamma), gmin (gmax/gmin)^((m+1)/ngamma));
     prad   (1 double, host): summed w P, P = K gamma^2 Bperp^2 the leading
            power of the radiation-reaction force g, K the coefficient the
            push applies at the current step (ramp included);
     sed[k] (nnu doubles, host): summed w nu dP/dnu at
            nu_k = numin (numax/numin)^(k/(nnu-1)) (code frequency units),
            nu dP/dnu = P x F(x) 9 sqrt(3) / (8 pi), x = nu / nu_c,
            nu_c = 3/(4 pi) gamma^2 omega_b |qm| Bperp, F the synchrotron
            function x int_x^inf K_{5/3}: the single-particle synchrotron
            spectrum normalised to P (F from a table, about 1e-5 relative).
   EINVAL for a bad species, a NULL output, an empty region or range, or
   ngamma / nnu outside [1, FFPIC_SPEC_MAX].  Synchronises. */
#define FFPIC_SPEC_MAX 256
typedef struct ffpic_spectra_req {
    double rmin, rmax, thmin, thmax;
    double gmin, gmax;
    double numin, numax;
    int32_t ngamma, nnu;
} ffpic_spectra_req;
int ffpic_spectra(ffpic_ctx *ctx, int species, const ffpic_spectra_req *req, double *dN,
                  double *sed, double *prad);

/* Checkpoint: with buf == NULL writes the required size to *len; otherwise
   serialises fields, Psi, f, particles, counters and the step number into
   buf (at least *len bytes, host memory).  Restore requires a context
   created from the same descriptor.  Synchronises. */
int ffpic_save(ffpic_ctx *ctx, void *buf, size_t *len);
int ffpic_restore(ffpic_ctx *ctx, const void *buf, size_t len);

/* Tuning of the fused field step: radial rows per workgroup (each
   workgroup owns a strip of theta columns and a slab of that many rows);
   0 = automatic (enough slabs to fill the GPU once, at least 32 rows).
   Results do not depend on it.  EINVAL for a negative value. */
int ffpic_set_field_rows(ffpic_ctx *ctx, int32_t rows);

/* Tuning of the FP32 push: particles per thread of a workgroup's chunk
   (8, 16 or 32; chunks of 256 threads).  Larger chunks share one field and
   one current patch among more particles; smaller ones make more
   workgroups for small systems.  Ignored by the FP64 push.  Results do not
   depend on it beyond the order of floating-point atomic additions.
   EINVAL for another value. */
int ffpic_set_push_chunk(ffpic_ctx *ctx, int32_t ppt);

/* Graph capture of ffpic_step (on by default).  A call of ffpic_step runs
   every whole sort cycle it contains (sort_interval steps from a step that
   sorts) as one HIP graph: captured on the first cycle that starts from a
   given host state (buffer roles, sort bookkeeping, slot bounds), then
   replayed for every later cycle from the same state (the buffers
   alternate, so a steady run replays two or four graphs).  Other steps,
   cycles whose kernel arguments change every step (surface injection or
   extraction, a radiation-reaction ramp), the first cycle after a load and
   steps timed with ffpic_set_timing are launched one by one.  Results do
   not depend on it.  ffpic_graph_stats reports the graphs captured and
   launched so far (either pointer nullable). */
int ffpic_set_graph(ffpic_ctx *ctx, int on);
int ffpic_graph_stats(ffpic_ctx *ctx, int64_t *builds, int64_t *launches);

/* Device time of each phase of the last ffpic_step call, in ms, summed over
   its steps: out[0] mask, [1] sort, [2] push+deposit, [3] fields.
   Requires ffpic_set_timing(ctx, 1) before the step. */
int ffpic_set_timing(ffpic_ctx *ctx, int enable);
int ffpic_phase_times(ffpic_ctx *ctx, float out[4]);


/* ---------------------------------------------------------------------
 * Batches of independent magnetospheres (many small systems on one GPU).
 *
 * ffpic_batch_create builds n systems from the n descriptors d[0..n-1].
 * Their kernels run on up to four library-owned streams, so that the
 * small grids run concurrently.  Systems are assigned to streams by
 * longest-processing-time-first packing on particles plus grid nodes.
 * `stream` is the caller's stream (borrowed; NULL = default stream):
 * ffpic_batch_step is ordered after the work already queued on it, and
 * work queued on it afterwards waits for the whole batch step.  EINVAL for
 * n < 1 or a rejected descriptor, ENOMEM, EHIP; on failure nothing is left
 * allocated.
 *
 * ffpic_batch_view gives system k as an ordinary context (non-owning):
 * every ffpic_* call works on it (loading particles, diagnostics, fields,
 * checkpoints, autotune).  ffpic_destroy on a view does nothing; the views
 * are released by ffpic_batch_destroy, which first drains the streams.
 * ffpic_batch_sync returns the first device error of any system.
 */
int ffpic_batch_create(int n, const ffpic_desc *d, void *stream, ffpic_batch **out);
int ffpic_batch_view(ffpic_batch *b, int k, ffpic_ctx **view);
int ffpic_batch_size(const ffpic_batch *b);
int ffpic_batch_step(ffpic_batch *b, int32_t nsteps);
int ffpic_batch_sync(ffpic_batch *b);

/* Graph capture of batch steps.  When every system stands at the start of
   one of its sort cycles and each could replay its own cycle from a graph
   (see ffpic_set_graph), ffpic_batch_step runs the least common multiple of
   the systems' sort intervals (up to 64 steps) of all systems as one HIP
   graph, captured once per host state of all systems and replayed
   afterwards.  Other steps are launched one by one.  `mode`:
     0  no graphs;
     1  the graph holds every system's own launches, each system's chain on
        its stream's branch;
     2  (default) where every system is FP32-mixed and has no plasma sources
        (injection, extraction, pair creation): the graph holds, per step,
        ONE launch of persistent workgroups for the flux functions of all
        systems, one for their masks, one per push kernel instance for all
        systems' pushes and one per field-step instance for all their field
        steps (each workgroup takes work items, such as a 4096-particle chunk
        of one system, from a counter in device memory until none is left);
        only the sorts stay per system.  The job tables those launches read
        are owned by the graph (device memory, freed with it).  Other
        batches fall back to mode 1.
   Results do not depend on the mode beyond the order of floating-point
   atomic additions in the deposit.  EINVAL for another mode.
   ffpic_batch_graph_stats: graphs captured and graph launches so far;
   ffpic_batch_grouped_launches: how many of the launches were mode-2
   graphs. */
int ffpic_batch_set_graph(ffpic_batch *b, int mode);
int ffpic_batch_graph_stats(ffpic_batch *b, int64_t *builds, int64_t *launches);
int ffpic_batch_grouped_launches(const ffpic_batch *b, int64_t *launches);
/* Particles per thread of the grouped pushes (mode 2): 8, 16 or 32 for every
   system, or 0 (the default) for each system's own setting (see
   ffpic_set_push_chunk).  A system's own setting is tuned for that system
   filling the GPU alone; grouped, the systems fill it together.  The
   arithmetic does not change (see ffpic_set_push_chunk).  EINVAL for another
   value. */
int ffpic_batch_set_grouped_chunk(ffpic_batch *b, int32_t ppt);
/* The graph mode in use (after ffpic_batch_autotune: the one it chose), when
   grouped_ppt is not NULL the grouped push chunk in use (0: each system's
   own), and, when ms_per_step is not NULL, the batch-step times the tuner
   measured for modes 0, 1, 2 (0 where not measured; for mode 2 the faster of
   its two chunk settings). */
int ffpic_batch_get_graph(const ffpic_batch *b, int32_t *mode, int32_t *grouped_ppt,
                          double ms_per_step[3]);
const char *ffpic_batch_last_error(const ffpic_batch *b);
int ffpic_batch_destroy(ffpic_batch *b);

/* ---------------------------------------------------------------------
 * Autotuning of the sort interval and the kernels' tile sizes.
 *
 * A sort costs one pass over all particle state.  Sorted particles make the
 * push's field gather and current deposit local.  The best interval depends
 * on the workload, and so do the tile sizes of the FP32 push (particles per
 * thread of a workgroup's chunk, which sets how many particles share one
 * field patch and one current patch) and of the fused field step (radial
 * rows of a workgroup's slab, see ffpic_set_field_rows).  ffpic_autotune
 * checkpoints the context to host memory (as ffpic_save) and, from that
 * state, times whole sort cycles of each candidate (after one untimed
 * cycle: a restored context's first sort is a full one, later sorts are
 * incremental), one parameter after the other, keeping the best value of
 * each before trying the next:
 *   1. the sort interval: 8, 4, 16, 2, 32, 1;
 *   2. the field step's slab rows: 0 (automatic), 32, 64, 128, 16;
 *   3. (FP32) the push's particles per thread: 16, 8, 32;
 * while the wall time stays within budget_ms (the first candidate of each
 * parameter is always timed).  It then restores the checkpoint and keeps
 * the chosen values.
 *
 * The state after the call equals the state before it.  None of the
 * parameters changes the arithmetic: results change by the order of
 * floating-point atomic additions in the deposit and in no other way.
 *
 * If the environment variable FFPIC_TUNING_CACHE names a file, a line
 * "nr nth precision nspec slots interval rows ppt" is appended to it.
 * ffpic_create with sort_interval = 0 takes the last matching line (same
 * nr, nth, precision, nspec) for all three, else 8, 0 and 16.
 *
 * Errors: EINVAL for a non-positive budget; a context in error
 * (ffpic_sync fails) is not tuned.  ffpic_batch_autotune tunes every system
 * with an equal share of the budget and writes n entries to out.  Then, for
 * a batch that can run as grouped launches (see ffpic_batch_set_graph) with
 * graphs on, it checkpoints every system, times whole batch cycles with
 * per-system graphs (mode 1), with grouped launches (mode 2) using each
 * system's push chunk and with grouped launches using 16 particles per thread
 * for every system, from that same state (each candidate twice, alternating,
 * its faster timing kept), restores the checkpoints and keeps the fastest
 * (ffpic_batch_get_graph reports the choice and the times).  The systems' states after
 * the call are those before it.
 */
#define FFPIC_TUNE_MAX 16
enum ffpic_tune_kind {
    FFPIC_TUNE_SORT_INTERVAL = 0,
    FFPIC_TUNE_FIELD_ROWS = 1,
    FFPIC_TUNE_PUSH_PPT = 2
};
typedef struct ffpic_tuning {
    int32_t sort_interval;               /* the values chosen (and now in use) */
    int32_t field_rows;
    int32_t push_ppt;                    /* 0 for FP64 contexts */
    int32_t ncand;                       /* candidates timed */
    int32_t cand_kind[FFPIC_TUNE_MAX];   /* the parameter of each (ffpic_tune_kind) */
    int32_t cand[FFPIC_TUNE_MAX];        /* its value */
    double ms_per_step[FFPIC_TUNE_MAX];  /* measured GPU time per step */
    double total_ms;                     /* wall time spent tuning */
} ffpic_tuning;

int ffpic_autotune(ffpic_ctx *ctx, double budget_ms, ffpic_tuning *out);
int ffpic_batch_autotune(ffpic_batch *b, double budget_ms, ffpic_tuning *out);

#ifdef __cplusplus
}
#endif
#endif
