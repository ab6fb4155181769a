// Surface pair injection (Sect. 4, monopole test: electron-positron pairs
// injected with multiplicity kappa_inj in the first layer of cells above the
// star, in the PIC domain only).
//
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
#include <rocprim/device/device_scan.hpp>

#include "device_common.h"

namespace ffpic {

constexpr uint32_t kInjTag = 0x696E6A63u;            // counter word 3 of the draws
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

struct InjArgs {
    InjSpecies sp[FFPIC_MAX_SPECIES];
    int nspec, nth, nr;
    double rn0, dlog, dth, omega;
    const double *thn;
    uint32_t step, k0, k1;
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
        uint32_t c[4] = {A.step, (uint32_t)j, (uint32_t)(p + 1), kInjTag};
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

size_t inject_scan_bytes(int nth) {
    size_t bytes = 0;
    hipError_t e = rocprim::exclusive_scan((void *)nullptr, bytes, (int32_t *)nullptr,
                                           (int32_t *)nullptr, 0, (size_t)nth + 1,
                                           rocprim::plus<int32_t>());
    if (e != hipSuccess) throw std::runtime_error("rocprim scan size query failed");
    return bytes;
}

void inject_pairs(ffpic_ctx *c) {
    if (!(c->d.inject_kappa > 0.0) || c->d.nspec == 0) return;
    const int nth = c->nth;
    const uint32_t k0 = (uint32_t)c->d.rng_seed, k1 = (uint32_t)(c->d.rng_seed >> 32);
    const uint32_t step = (uint32_t)c->step;
    const int nb = (nth + 1 + 255) / 256;
    hipLaunchKernelGGL(k_inject_count, dim3(nb), dim3(256), 0, c->stream, nth, c->kill,
                       c->inj_rate, step, k0, k1, c->inj_cnt);
    size_t bytes = c->inj_scan_bytes;
    if (rocprim::exclusive_scan(c->inj_scan_tmp, bytes, c->inj_cnt, c->inj_off, 0,
                                (size_t)nth + 1, rocprim::plus<int32_t>(),
                                c->stream) != hipSuccess)
        throw std::runtime_error("rocprim scan failed");
    InjArgs A{};
    A.nspec = c->d.nspec;
    A.nth = nth;
    A.nr = c->nr;
    A.rn0 = c->tab[T_RN][0];
    A.dlog = c->dlog;
    A.dth = c->dth;
    A.omega = c->omega;
    A.thn = c->dtab64[T_THN];
    A.step = step;
    A.k0 = k0;
    A.k1 = k1;
    for (int s = 0; s < c->d.nspec; s++) {
        for (int a = 0; a < c->sp[s].narr; a++) A.sp[s].arr[a] = c->sp[s].cur[a];
        A.sp[s].nslots = c->nslots + s;
        A.sp[s].cap = c->sp[s].cap;
    }
    if (c->fp64)
        hipLaunchKernelGGL(k_inject_write<true>, dim3(nb), dim3(256), 0, c->stream, c->inj_cnt,
                           c->inj_off, A);
    else
        hipLaunchKernelGGL(k_inject_write<false>, dim3(nb), dim3(256), 0, c->stream, c->inj_cnt,
                           c->inj_off, A);
    hipLaunchKernelGGL(k_inject_commit, dim3(1), dim3(1), 0, c->stream, c->inj_off, A, c->err);
    FFPIC_LAUNCH_CHECK();
    // host upper bound of the slots in use
    for (int s = 0; s < c->d.nspec; s++)
        c->sp[s].nub = std::min<int64_t>(c->sp[s].nub + c->inj_bound, c->sp[s].cap);
}

}  // namespace ffpic
