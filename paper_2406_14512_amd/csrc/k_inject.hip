// Particle sources at the stellar surface: the pair injection of the
// monopole test (Sect. 4) and the Goldreich-Julian extraction of electrons
// and ions of the dipole (Sect. 5).
//
// Pair injection: electron-positron pairs injected with multiplicity
// kappa_inj in the first layer of cells above the star, PIC domain only.
// Every step, surface cell (0, j) outside the pure force-free domain gets
// floor(N_j) pairs plus one more with probability frac(N_j), where N_j (a
// host table, FP64) is kappa_inj times the Goldreich-Julian number density
// Omega |B_r| / (2 pi q) in the cell volume, renewed once per crossing time
// of the cell.  Positions are uniform in the cell's logical offsets, the
// momentum is corotation (u_phi = gamma Omega r sin theta), and every
// species gets one particle at each position (a pair carries no net charge).
//
// Random numbers: Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw
// 2011), counter = (step, cell, draw, tag), key = the descriptor's seed, so
// the draws do not depend on the order in which threads run.  The new
// particles are appended behind the current slots in (cell, draw) order: a
// per-cell count, an exclusive scan, then one writer per cell.
//
// Extraction: the charge held by each surface cell outside the pure
// force-free domain (every species' weight times its live particles in the
// cell, species in order) is topped up to gj_extract |rho_GJ| V with
// ceil(deficit / (w_e + w_i)) electron-ion pairs, placed and appended like
// the injected pairs (counter word 3 = kExtTag).

#include "device_common.h"

namespace ffpic {

constexpr uint32_t kInjTag = 0x696E6A63u;            // counter word 3 of the injection draws
constexpr uint32_t kExtTag = 0x676A6578u;            // ... and of the extraction draws
constexpr double kNear1 = 0.99999994039535522;       // largest float below 1

__device__ __forceinline__ void philox4x32(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c[0] = hi1 ^ c[1] ^ k0;
        c[1] = lo1;
        c[2] = hi0 ^ c[3] ^ k1;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double u01(uint32_t x) { return (double)x * (1.0 / 4294967296.0); }

// number of pairs of each surface cell this step (cnt[nth] = 0 so that the
// exclusive scan's last entry is the total)
__global__ void k_inject_count(int nth, const uint8_t *__restrict__ kill,
                               const double *__restrict__ rate, uint32_t step, uint32_t k0,
                               uint32_t k1, int32_t *__restrict__ cnt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > nth) return;
    int n = 0;
    if (j < nth && !kill[j]) {
        const double N = rate[j];
        const double fl = floor(N);
        uint32_t c[4] = {step, (uint32_t)j, 0u, kInjTag};
        philox4x32(c, k0, k1);
        n = (int)fl + (u01(c[0]) < N - fl ? 1 : 0);
    }
    cnt[j] = n;
}

struct InjSpecies {
    void *arr[6];          // state arrays (FP64: r, th, ur, uth, uph; FP32: cell, a, b, u x3)
    int32_t *nslots;
    int64_t cap;
};

// the species that receive one particle at each drawn position
struct InjArgs {
    InjSpecies sp[FFPIC_MAX_SPECIES];
    int nspec, nth, nr;
    double rn0, dlog, dth, omega;
    const double *thn;
    uint32_t step, k0, k1, tag;
};

// all species fit, else nothing is injected this step
__device__ __forceinline__ bool inject_fits(const InjArgs &A, int total) {
    bool ok = true;
    for (int s = 0; s < A.nspec; s++) ok = ok && (int64_t)A.sp[s].nslots[0] + total <= A.sp[s].cap;
    return ok;
}

template <bool FP64>
__global__ void k_inject_write(const int32_t *__restrict__ cnt, const int32_t *__restrict__ off,
                               InjArgs A) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A.nth) return;
    const int n = cnt[j];
    if (n == 0 || !inject_fits(A, off[A.nth])) return;
    for (int p = 0; p < n; p++) {
        uint32_t c[4] = {A.step, (uint32_t)j, (uint32_t)(p + 1), A.tag};
        philox4x32(c, A.k0, A.k1);
        const double a = u01(c[0]), b = u01(c[1]);
        const double r = A.rn0 * exp(a * A.dlog);
        const double th = A.thn[j] + b * A.dth;
        const double v = A.omega * r * sin(th);
        const double uph = v / sqrt(1.0 - v * v);
        for (int s = 0; s < A.nspec; s++) {
            const int64_t q = (int64_t)A.sp[s].nslots[0] + off[j] + p;
            if (FP64) {
                double **d = (double **)A.sp[s].arr;
                d[0][q] = r; d[1][q] = th; d[2][q] = 0.0; d[3][q] = 0.0; d[4][q] = uph;
            } else {
                // cell and FP32 offsets; an offset that rounds up to 1 moves
                // to the next cell (as for loaded particles)
                int i = 0, jj = j;
                float af = (float)a, bf = (float)b;
                if (af >= 1.f) {
                    if (A.nr > 1) { i = 1; af = 0.f; } else { af = (float)kNear1; }
                }
                if (bf >= 1.f) {
                    if (jj < A.nth - 1) { jj++; bf = 0.f; } else { bf = (float)kNear1; }
                }
                ((int32_t *)A.sp[s].arr[0])[q] = (i << 16) | jj;
                ((float *)A.sp[s].arr[1])[q] = af;
                ((float *)A.sp[s].arr[2])[q] = bf;
                ((float *)A.sp[s].arr[3])[q] = 0.f;
                ((float *)A.sp[s].arr[4])[q] = 0.f;
                ((float *)A.sp[s].arr[5])[q] = (float)uph;
            }
        }
    }
}

// the new slots join the species (or the capacity error is recorded)
__global__ void k_inject_commit(const int32_t *__restrict__ off, InjArgs A,
                                uint32_t *__restrict__ err) {
    const int total = off[A.nth];
    if (total == 0) return;
    if (!inject_fits(A, total)) {
        atomicOr(err, FFPIC_ERR_CAPACITY);
        return;
    }
    for (int s = 0; s < A.nspec; s++) A.sp[s].nslots[0] += total;
}

namespace {

InjArgs inj_args(ffpic_ctx *c, const int *targets, int ntargets, uint32_t tag) {
    InjArgs A{};
    A.nspec = ntargets;
    A.nth = c->nth;
    A.nr = c->nr;
    A.rn0 = c->tab[T_RN][0];
    A.dlog = c->dlog;
    A.dth = c->dth;
    A.omega = c->omega;
    A.thn = c->dtab64[T_THN];
    A.step = (uint32_t)c->step;
    A.k0 = (uint32_t)c->d.rng_seed;
    A.k1 = (uint32_t)(c->d.rng_seed >> 32);
    A.tag = tag;
    for (int t = 0; t < ntargets; t++) {
        const int s = targets[t];
        for (int a = 0; a < c->sp[s].narr; a++) A.sp[t].arr[a] = c->sp[s].cur[a];
        A.sp[t].nslots = c->nslots + s;
        A.sp[t].cap = c->sp[s].cap;
    }
    return A;
}

// scan of the per-cell counts in c->inj_cnt, then the ordered append and
// the commit (or the capacity error)
void append_surface(ffpic_ctx *c, const int *targets, int ntargets, uint32_t tag,
                    int64_t bound) {
    const InjArgs A = inj_args(c, targets, ntargets, tag);
    const int nth = c->nth;
    const int nb = (nth + 1 + 255) / 256;
    exclusive_scan_i32(c, c->inj_cnt, c->inj_off, (int64_t)nth + 1);
    if (c->fp64)
        hipLaunchKernelGGL(k_inject_write<true>, dim3(nb), dim3(256), 0, c->stream, c->inj_cnt,
                           c->inj_off, A);
    else
        hipLaunchKernelGGL(k_inject_write<false>, dim3(nb), dim3(256), 0, c->stream, c->inj_cnt,
                           c->inj_off, A);
    hipLaunchKernelGGL(k_inject_commit, dim3(1), dim3(1), 0, c->stream, c->inj_off, A, c->err);
    FFPIC_LAUNCH_CHECK();
    // host upper bound of the slots in use
    for (int t = 0; t < ntargets; t++) {
        ffpic::Species &S = c->sp[targets[t]];
        S.nub = std::min<int64_t>(S.nub + bound, S.cap);
    }
}

// live particles of one species in each surface cell (i = 0)
template <bool FP64>
__global__ void k_surface_count(int nub, const int32_t *__restrict__ nslots, int nr, int nth,
                                double rmin, double dlog, double dth,
                                const double *__restrict__ rn, const double *__restrict__ thn,
                                const void *__restrict__ a0, const void *__restrict__ a1,
                                int32_t *__restrict__ have) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub || q >= nslots[0]) return;
    if (FP64) {
        const double r = ((const double *)a0)[q];
        if (!(r > 0.0) || !(r < rn[1])) return;
        int i, j;
        double a, b;
        locate64(nr, nth, rmin, dlog, dth, rn, thn, r, ((const double *)a1)[q], i, j, a, b);
        if (i == 0) atomicAdd(&have[j], 1);
    } else {
        const int cell = ((const int32_t *)a0)[q];
        if (cell >= 0 && (cell >> 16) == 0) atomicAdd(&have[cell & 0xffff], 1);
    }
}

struct ExtArgs {
    double w[FFPIC_MAX_SPECIES];
    double wpair;
    int nspec, nth;
};

// pairs to extract per surface cell (cnt[nth] = 0 for the scan's total)
__global__ void k_extract_count(ExtArgs X, const uint8_t *__restrict__ kill,
                                const double *__restrict__ target,
                                const int32_t *__restrict__ have, int32_t *__restrict__ cnt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > X.nth) return;
    int n = 0;
    if (j < X.nth && !kill[j]) {
        double held = 0.0;
        for (int s = 0; s < X.nspec; s++) held += X.w[s] * (double)have[s * X.nth + j];
        const double deficit = target[j] - held;
        if (deficit > 0.0) n = (int)ceil(deficit / X.wpair);
    }
    cnt[j] = n;
}

}  // namespace

void inject_pairs(ffpic_ctx *c) {
    if (!(c->d.inject_kappa > 0.0) || c->d.nspec == 0) return;
    const int nth = c->nth;
    const uint32_t k0 = (uint32_t)c->d.rng_seed, k1 = (uint32_t)(c->d.rng_seed >> 32);
    const uint32_t step = (uint32_t)c->step;
    const int nb = (nth + 1 + 255) / 256;
    hipLaunchKernelGGL(k_inject_count, dim3(nb), dim3(256), 0, c->stream, nth, c->kill,
                       c->inj_rate, step, k0, k1, c->inj_cnt);
    int all[FFPIC_MAX_SPECIES];
    for (int s = 0; s < c->d.nspec; s++) all[s] = s;
    append_surface(c, all, c->d.nspec, kInjTag, c->inj_bound);
}

void extract_gj(ffpic_ctx *c) {
    if (!(c->d.gj_extract > 0.0)) return;
    const int nth = c->nth, ns = c->d.nspec;
    zero_counters(c, c->gj_have, ns * nth);
    for (int s = 0; s < ns; s++) {
        const ffpic::Species &S = c->sp[s];
        if (S.nub == 0) continue;
        const int nbs = (int)((S.nub + 255) / 256);
        hipLaunchKernelGGL(c->fp64 ? k_surface_count<true> : k_surface_count<false>, dim3(nbs),
                           dim3(256), 0, c->stream, (int)S.nub, c->nslots + s, c->nr, nth,
                           c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN], c->dtab64[T_THN],
                           S.cur[0], S.cur[1], c->gj_have + (size_t)s * nth);
    }
    ExtArgs X{};
    for (int s = 0; s < ns; s++) X.w[s] = c->d.weight[s];
    X.wpair = c->d.weight[c->d.gj_species[0]] + c->d.weight[c->d.gj_species[1]];
    X.nspec = ns;
    X.nth = nth;
    hipLaunchKernelGGL(k_extract_count, dim3((nth + 1 + 255) / 256), dim3(256), 0, c->stream, X,
                       c->kill, c->gj_target, c->gj_have, c->inj_cnt);
    FFPIC_LAUNCH_CHECK();
    append_surface(c, c->d.gj_species, 2, kExtTag, c->gj_bound);
}

}  // namespace ffpic
