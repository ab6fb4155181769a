// Internal declarations of the MI355X hybrid force-free / PIC library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ffpic.h"
#include "sort_view.h"

namespace ffpic {

constexpr double kPi = 3.14159265358979323846;

// Geometry of the spherical Yee grid as 1-D tables (all computed on the host
// in FP64, stored in the working precision R).  Index conventions:
//   radial node i in [0, nr], half node i+1/2 stored at i in [0, nr);
//   polar node j in [0, nth], half node j+1/2 stored at j in [0, nth).
// Dual cell of node (i, j): r in [r_lo(i), r_hi(i)], theta in
// [theta_lo(j), theta_hi(j)] with r_lo(0) = r_0, r_hi(nr) = r_nr and the
// theta range clipped to [0, pi] on the axis.
template <typename R>
struct Geo {
    int nr, nth, ld;        // ld = nth + 1 (row stride of every field array)
    R dt, dth;
    const R *rn;    // r_i                        [nr+1]
    const R *rh;    // r_{i+1/2}                  [nr]
    const R *rn2;   // r_i^2                      [nr+1]
    const R *rh2;   // r_{i+1/2}^2                [nr]
    const R *drn;   // r_{i+1} - r_i              [nr]
    const R *drh;   // r_{i+1/2} - r_{i-1/2}      [nr+1] (entry 0 unused)
    const R *dr2n;  // (r_{i+1}^2 - r_i^2) / 2    [nr]
    const R *dr2h;  // (r_hi^2 - r_lo^2) / 2      [nr+1]
    const R *dr3h;  // (r_hi^3 - r_lo^3) / 3      [nr+1]
    const R *dr3n;  // (r_{i+1}^3 - r_i^3) / 3    [nr]
    const R *lamn;  // absorber factor at r_i     [nr+1]
    const R *lamh;  // absorber factor at r_{i+1/2} [nr]
    const R *sn;    // sin(theta_j)               [nth+1]
    const R *cn;    // cos(theta_j)               [nth+1]
    const R *sh;    // sin(theta_{j+1/2})         [nth]
    const R *dcn;   // cos(theta_j) - cos(theta_{j+1})   [nth]
    const R *dcd;   // cos(theta_lo) - cos(theta_hi)     [nth+1]
    const R *dthd;  // theta_hi - theta_lo               [nth+1]
};

enum { T_RN, T_RH, T_RN2, T_RH2, T_DRN, T_DRH, T_DR2N, T_DR2H, T_DR3H, T_DR3N,
       T_LAMN, T_LAMH, T_SN, T_CN, T_SH, T_DCN, T_DCD, T_DTHD, T_THN, T_NTAB };
static_assert(T_RN == FFPIC_TAB_RN && T_DCN == FFPIC_TAB_DCN && T_THN == FFPIC_TAB_THN &&
                  T_NTAB == FFPIC_NTAB,
              "the internal table order is the one ffpic_host_table exports");

struct Species {
    int64_t cap = 0;
    int64_t nub = 0;          // host upper bound of the slots in use
    void *cur[6] = {};        // FP64: r, th, ur, uth, uph | FP32: cell, a, b, ur, uth, uph
    void *alt[6] = {};
    int narr = 0;
    double qm = 0, weight = 0;
};

// The host state that one sort cycle of steps reads into its kernels'
// arguments and changes: buffer pointers that swap, sort bookkeeping, slot
// bounds.  A captured cycle is replayed only from the state it was captured
// in, and leaves the state its capture left.
struct CycleState {
    void *cur[FFPIC_MAX_SPECIES][6], *alt[FFPIC_MAX_SPECIES][6];
    int64_t nub[FFPIC_MAX_SPECIES];
    int sort_cur[FFPIC_MAX_SPECIES];
    bool sort_valid[FFPIC_MAX_SPECIES], perm_valid[FFPIC_MAX_SPECIES];
    void *E[3], *B[3], *J[3], *dE[3], *dB[3], *stAlt[6], *Jalt[3];
    int fused_rows, push_ppt;        // settings the launches depend on
    bool record_perm, incremental_sort;
};

struct CycleGraph {
    int steps = 0;
    CycleState pre{}, post{};
    hipGraphExec_t exec = nullptr;
};

}  // namespace ffpic

struct ffpic_ctx {
    ffpic_desc d{};
    hipStream_t stream = nullptr;
    int nr = 0, nth = 0, ld = 0;
    size_t nn = 0;
    double dlog = 0, dth = 0, dt = 0, omega = 0;
    bool fp64 = true;
    std::vector<double> tab[ffpic::T_NTAB];   // host FP64 tables
    void *dtab[ffpic::T_NTAB] = {};           // device tables in working precision
    double *dtab64[ffpic::T_NTAB] = {};       // device FP64 tables
    size_t rsz = 8;                           // sizeof(R)
    void *E[3] = {}, *B[3] = {}, *B0[3] = {}, *J[3] = {};
    // FP32 mode: perturbation state about the FP64 background (see
    // fields_fused.h) and the background's rates evaluated in FP64
    void *dE[3] = {}, *dB[3] = {}, *E0[3] = {}, *rE0[3] = {}, *rB0[3] = {}, *rho0 = nullptr;
    // FP32 mode: FP64 device copies of the background E_r, E_th, B_r, B_th
    // (the FP64 Gauss and div B residuals are formed from them plus dE, dB)
    double *E0d[2] = {}, *B0d[2] = {};
    // the fused field step reads one state buffer and writes the other
    // (FP64: E, B; FP32: dE, dB), and clears the second set of deposit
    // accumulators for the next push; the pointers swap after each step
    void *stAlt[6] = {}, *Jalt[3] = {};
    bool rE0_zero[3] = {}, rB0_zero[3] = {};  // FP32: background rate identically zero
    int fused_rows = 0;                       // slab height (0 = from fused_slots)
    int push_ppt = 16;                        // FP32 push: particles per thread (8, 16, 32)
    int fused_slots = 0;                      // workgroups resident on the GPU at once
    void *fz_rowc = nullptr, *fz_colc = nullptr;   // FP32 field step: row / column coefficients
    int device = 0;                           // HIP device the context was created on
    size_t cstride = 0;                       // elements between the components of a field
    std::vector<double> hE0[3], hB0[3];       // FP64 background (host)
    int absorb_row0 = 0;                      // first grid row with damping below 1
    // surface pair injection: expected pairs per step of each surface cell
    // (FP64, host-computed), per-cell counts and their scan
    double *inj_rate = nullptr;
    int32_t *inj_cnt = nullptr, *inj_off = nullptr;
    int64_t inj_bound = 0;                    // most pairs one step can add
    // Goldreich-Julian extraction: target charge of each surface cell (FP64,
    // host-computed), per-species particle counts of the surface cells
    double *gj_target = nullptr;
    int32_t *gj_have = nullptr;               // [nspec][nth]
    int64_t gj_bound = 0;                     // most pairs one step can add
    // threshold pair creation: per-block parent counts of both parent
    // species and their exclusive scan
    int32_t *pair_cnt = nullptr, *pair_off = nullptr;
    int64_t pair_blocks = 0;                  // capacity of pair_cnt (entries - 1)
    // spectra: table of ln F of the synchrotron function, the gamma bin
    // edges and frequencies of the last request
    double *spec_tab = nullptr, *spec_edge = nullptr, *spec_nu = nullptr;
    double *psi = nullptr;
    void *f = nullptr;
    uint8_t *kill = nullptr;
    ffpic::Species sp[FFPIC_MAX_SPECIES];
    uint32_t *keys[2] = {}, *vals[2] = {};
    // incremental re-sort: per species the cell offsets of the last sort
    // (double-buffered), plus shared scratch
    int32_t *soff[FFPIC_MAX_SPECIES][2] = {};
    int sort_cur[FFPIC_MAX_SPECIES] = {};
    bool sort_valid[FFPIC_MAX_SPECIES] = {};
    bool incremental_sort = true;
    // per species (see sort_alloc): class words, counts, key offsets of the
    // stayers, the movers' places
    uint64_t *sort_smask[FFPIC_MAX_SPECIES] = {}, *sort_mmask[FFPIC_MAX_SPECIES] = {};   // [cap/64 + 1]
    uint32_t *sort_wsm[FFPIC_MAX_SPECIES] = {};   // counts before each word in its tile
    uint2 *sort_tc[FFPIC_MAX_SPECIES] = {}, *sort_ts[FFPIC_MAX_SPECIES] = {},
          *sort_gs[FFPIC_MAX_SPECIES] = {};   // tile / group counts
    uint32_t *sort_aux = nullptr;             // sorted mover slots [cap]
    int32_t *sort_mst[FFPIC_MAX_SPECIES] = {};   // movers before each key's stayers [nr*nth + 1]
    int32_t *sort_kcnt = nullptr;             // movers per key, zero between sorts [nr*nth + 1]
    void *sort_cbuf = nullptr;                // movers' state, compacted [narr * cbuf_n]
    int64_t sort_cbuf_n = 0;
    uint32_t *sort_tot[FFPIC_MAX_SPECIES] = {};  // stayers, movers, slots before the sort
    int32_t *sort_dest[FFPIC_MAX_SPECIES] = {};   // FP32: place of each slot's particle [cap]
    bool sort_pending[FFPIC_MAX_SPECIES] = {};   // the next push places the sort
    ffpic::SortPlace place[FFPIC_MAX_SPECIES] = {};
    uint32_t *rs_hist = nullptr, *rs_dtot = nullptr;   // radix sort: digit counts per tile
    int rs_stride = 0;                        // tiles per digit row of rs_hist
    int32_t *rs_n = nullptr;                  // radix sort: pair count (device)
    int32_t *scan_part = nullptr;             // block sums of exclusive_scan_i32
    int64_t scan_part_n = 0;
    // sort permutation of the last sort of each species (ffpic_record_sort)
    bool record_perm = false;
    int32_t *perm[FFPIC_MAX_SPECIES] = {};
    bool perm_valid[FFPIC_MAX_SPECIES] = {};
    int64_t sort_cap = 0;
    int32_t *nslots = nullptr;                // device [FFPIC_MAX_SPECIES]
    int32_t *nsorted = nullptr;               // device: live count at each species' last sort
    int32_t *nalive = nullptr;                // device [FFPIC_MAX_SPECIES]
    unsigned long long *removed = nullptr;    // device [FFPIC_MAX_SPECIES][4]
    uint32_t *err = nullptr;                  // device error word
    double *red = nullptr;                    // reduction scratch (device)
    size_t red_len = 0;
    int64_t step = 0;
    bool sorted_once[FFPIC_MAX_SPECIES] = {};
    int timing = 0;
    hipEvent_t ev[8] = {};
    std::vector<hipEvent_t> evpool;           // 5 per timed step
    float phase_ms[4] = {};
    bool batch_owned = false;                 // a view of a batch system
    // graph-captured sort cycles (see ffpic_set_graph): the graphs made so
    // far, each with the host state it starts from and leaves behind
    bool use_graph = true;
    hipStream_t gstream = nullptr;            // capture stream (forked from stream)
    hipEvent_t gfork = nullptr, gjoin = nullptr;
    std::vector<ffpic::CycleGraph> graphs;
    int64_t graph_builds = 0, graph_launches = 0;
    std::string last_error;
};

namespace ffpic {

template <typename R>
Geo<R> geo(const ffpic_ctx *c);

// kernels (launchers); all enqueue on c->stream
void psi_mask(ffpic_ctx *c);
// kill + stable sort by cell; with defer (FP32, incremental sorts) the
// particles are placed in the new order by the species' next push
void sort_species(ffpic_ctx *c, int s, bool defer = false);
void kill_species(ffpic_ctx *c, int s);           // kill without sorting
void push_species(ffpic_ctx *c, int s);
void field_step(ffpic_ctx *c);
void convert_loaded(ffpic_ctx *c, int s, int64_t off, int64_t n, const double *r,
                    const double *th, const double *ur, const double *uth, const double *uph);
void export_particles(ffpic_ctx *c, int s, int64_t first, int64_t n, double *r, double *th, double *ur,
                      double *uth, double *uph, int32_t *cell);   // device outputs
void to_f64(ffpic_ctx *c, const void *src, double *dst, size_t n);
void from_f64(ffpic_ctx *c, const double *src, void *dst, size_t n);
void sort_offsets(ffpic_ctx *c, int s, int32_t *dev_off);
// FP64 diagnostics.  `part` holds diag_partials() * 5 doubles of per-block
// partial results (device scratch), `out*` device result slots.
int diag_partials();
void moments(ffpic_ctx *c, int s, double *part, double *dev_out5);
// Gauss residual: node charges into qn (nn doubles, cleared here), then the
// map (nullable) and/or the per-block maxima of |G| (part, nullable)
void gauss(ffpic_ctx *c, double *qn, double *dev_map, double *part);
void divb(ffpic_ctx *c, double *dev_map, double *part);
void poynting(ffpic_ctx *c, double *dev_L);
void energies(ffpic_ctx *c, double *part, double *dev_out2);
// device scratch of one diagnostics call
struct DiagBufs {
    double *part = nullptr;   // diag_partials() * 5
    double *out = nullptr;    // 16 result slots
    double *qn = nullptr;     // nn node charges (residuals only)
    double *L = nullptr;      // nr + 1 (Poynting flux only)
};
// everything of ffpic_diagnostics but the scratch: synchronises, fills *out
// and (nullable) the host array L_of_r; allocates nothing on the device
void run_diagnostics(ffpic_ctx *c, uint32_t what, ffpic_diag *out, double *L_of_r,
                     const DiagBufs &b);
// the same, returning a status (and setting the context's error message)
// instead of throwing
void fused32_tables(const ffpic_ctx *c, std::vector<float> &rowc, std::vector<float> &colc);
int run_diagnostics_checked(ffpic_ctx *c, uint32_t what, ffpic_diag *out, double *L_of_r,
                            const DiagBufs &b);
void sort_alloc(ffpic_ctx *c, int64_t cap, void *(*dmalloc)(size_t));
int sort_key_bits(const ffpic_ctx *c);
// exclusive scan of n int32 values on the device (block sums in scan_part,
// which must hold scan_part_len(n) entries)
void exclusive_scan_i32(ffpic_ctx *c, const int32_t *in, int32_t *out, int64_t n);
int64_t scan_part_len(int64_t n);
void zero_counters(ffpic_ctx *c, int32_t *p, int n);
void tuned_settings(const ffpic_desc *d, int *interval, int *rows, int *ppt);
void inject_pairs(ffpic_ctx *c);
void extract_gj(ffpic_ctx *c);
void create_pairs(ffpic_ctx *c);
int pair_block_slots();
double rr_factor(const ffpic_ctx *c);   // radiation-reaction ramp at this step
// steps launched one by one (no graph), for callers that capture themselves
void steps_one_by_one(ffpic_ctx *c, int n);
// whether the next sort cycle can be replayed from a graph, and the host
// state such a replay starts from and leaves (see CycleState)
bool graphable_cycle(const ffpic_ctx *c);
bool step_sorts(const ffpic_ctx *c);    // the step about to be taken sorts
CycleState get_cycle_state(const ffpic_ctx *c);
void put_cycle_state(ffpic_ctx *c, const CycleState &st);
// dev_out: ngamma + nnu + 1 doubles (dN, sed, prad)
void spectra(ffpic_ctx *c, int s, const ffpic_spectra_req *req, double *dev_out);

// Grouped launches over several FP32-mixed contexts: each *_job call writes
// one context's job (the arguments its launch would take) into out, does
// the host bookkeeping that follows the launch, and returns the job's number
// of work items; the *_group_launch calls run the jobs of a table in device
// memory (job k owns items [starts[k], starts[k + 1])) on persistent
// workgroups (grid of them) that take items from the counter pair ctr
// (zero before the launch, zero again after it).
size_t push_job_bytes();
// ppt: particles per thread of the grouped push (8, 16, 32), 0 = the
// context's own setting
int push_group_key(const ffpic_ctx *c, int s, int ppt);   // kernel instance, 0..11
int push_job(ffpic_ctx *c, int s, void *out, int ppt);
int push_group_slots(int key);
void push_group_launch(hipStream_t st, int key, const void *jobs, const int *starts, int njobs,
                       int grid, int *ctr);
size_t field_job_bytes();
int field_job(ffpic_ctx *c, void *out, int *key); // key: kernel instance, 0..7
int field_group_slots(int key);
void field_group_launch(hipStream_t st, int key, const void *jobs, const int *starts, int njobs,
                        int grid, int *ctr);
size_t psi_job_bytes();
size_t mask_job_bytes();
int psi_job32(const ffpic_ctx *c, void *out);
int mask_job32(const ffpic_ctx *c, void *out);
int psi_group_slots();
void psi_group_launch(hipStream_t st, const void *jobs, const int *starts, int njobs, int grid,
                      int *ctr);
void mask_group_launch(hipStream_t st, const void *jobs, const int *starts, int njobs, int grid);

}  // namespace ffpic

#define FFPIC_LAUNCH_CHECK()                                                     \
    do {                                                                         \
        hipError_t e_ = hipGetLastError();                                       \
        if (e_ != hipSuccess) throw std::runtime_error(hipGetErrorString(e_));   \
    } while (0)
