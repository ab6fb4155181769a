// Threshold pair creation (Sect. 5, aligned dipole): after the push, every
// particle of the two lepton species whose Lorentz factor exceeds gamma_th
// creates one electron and one positron at its own position, moving along
// its momentum with Lorentz factor gamma_s.  The parent keeps its state.
//
// The new particles are appended in a fixed order, independent of thread
// scheduling: parent species in order, then parent slots in order.  Three
// launches per parent species and one scan:
//   1. per block of kPairSlots slots, the number of parents;
//   2. an exclusive scan over the blocks of both species (plus one zero
//      entry, whose scanned value is the total);
//   3. per block, the parents are found again and ranked in slot order (a
//      ballot per wavefront, the wavefronts' counts through LDS) and their
//      pairs written behind the current slots of both target species;
// then one thread commits the new slot counts, or records the capacity
// error if either species would overflow (nothing is added that step).
// The parent test 1 + |u|^2 > gamma_th^2 is evaluated by the same code in
// launches 1 and 3, and this file is compiled without FP contraction, so
// both launches take the same decision for every particle.

#include "device_common.h"

namespace ffpic {

namespace {

constexpr int kPairWG = 256;
constexpr int kPairPPT = 4;
constexpr int kPairSlots = kPairWG * kPairPPT;

struct PairTarget {
    void *arr[6];          // FP64: r, th, ur, uth, uph; FP32: cell, a, b, ur, uth, uph
    int32_t *nslots;
    int64_t cap;
};

struct PairArgs {
    PairTarget t[2];       // electron and positron species
    double gth2;           // gamma_th^2
    double us;             // |u| of a created particle, sqrt(gamma_s^2 - 1)
    int nblk_total;        // blocks of both parent species
};

template <bool FP64>
__device__ __forceinline__ bool is_parent(void *const *arr, unsigned q, double gth2, float gth2f,
                                          double &f64, float &f32, double us, float usf) {
    if (FP64) {
        const double r = ((const double *)arr[0])[q];
        if (!(r > 0.0)) return false;
        const double ur = ((const double *)arr[2])[q], ut = ((const double *)arr[3])[q],
                     up = ((const double *)arr[4])[q];
        const double u2 = ur * ur + ut * ut + up * up;
        if (!(1.0 + u2 > gth2)) return false;
        f64 = us / sqrt(u2);
        return true;
    } else {
        if (((const int32_t *)arr[0])[q] < 0) return false;
        const float ur = ((const float *)arr[3])[q], ut = ((const float *)arr[4])[q],
                    up = ((const float *)arr[5])[q];
        const float u2 = ur * ur + ut * ut + up * up;
        if (!(1.f + u2 > gth2f)) return false;
        f32 = usf / sqrtf(u2);
        return true;
    }
}

// launch 1: parents per block of slots
template <bool FP64>
__global__ void __launch_bounds__(kPairWG)
    k_pair_count(PairTarget P, int nub, const int32_t *__restrict__ nslots, double gth2,
                 int32_t *__restrict__ cnt) {
    __shared__ int wsum[kPairWG / 64];
    const int tid = threadIdx.x;
    const int n = min(nub, nslots[0]);
    const int base = blockIdx.x * kPairSlots;
    int mine = 0;
    double f64;
    float f32;
    for (int k = 0; k < kPairPPT; k++) {
        const int q = base + k * kPairWG + tid;
        if (q < n && is_parent<FP64>(P.arr, (unsigned)q, gth2, (float)gth2, f64, f32, 0.0, 0.f))
            mine++;
    }
    for (int o = 32; o >= 1; o >>= 1) mine += __shfl_xor(mine, o, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = mine;
    __syncthreads();
    if (tid == 0) {
        int t = 0;
        for (int w = 0; w < kPairWG / 64; w++) t += wsum[w];
        cnt[blockIdx.x] = t;
    }
}

// launch 3: the ordered write of the pairs of one parent species' blocks
template <bool FP64>
__global__ void __launch_bounds__(kPairWG)
    k_pair_write(PairTarget P, int nub, const int32_t *__restrict__ nslots,
                 const int32_t *__restrict__ off, const int32_t *__restrict__ tot, PairArgs A) {
    __shared__ int wcnt[kPairWG / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // off: the scanned counts of this species' blocks; tot: the total of
    // both species
    const int total = tot[0];
    // every target species must take all of this step's pairs
    for (int t = 0; t < 2; t++)
        if ((int64_t)A.t[t].nslots[0] + total > A.t[t].cap) return;
    const int n = min(nub, nslots[0]);
    const int base = blockIdx.x * kPairSlots;
    int run = off[blockIdx.x];
    const float usf = (float)A.us;
    for (int k = 0; k < kPairPPT; k++) {
        const int q = base + k * kPairWG + tid;
        double f64 = 0.0;
        float f32 = 0.f;
        const bool par = q < n && is_parent<FP64>(P.arr, (unsigned)q, A.gth2, (float)A.gth2,
                                                  f64, f32, A.us, usf);
        const unsigned long long m = __ballot(par);
        if (lane == 0) wcnt[wave] = __popcll(m);
        __syncthreads();
        int before = 0, all = 0;
        for (int w = 0; w < kPairWG / 64; w++) {
            before += w < wave ? wcnt[w] : 0;
            all += wcnt[w];
        }
        if (par) {
            const unsigned long long below = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
            const int rank = run + before + __popcll(below);
            for (int t = 0; t < 2; t++) {
                const int64_t d = (int64_t)A.t[t].nslots[0] + rank;
                if (FP64) {
                    const double *src[5] = {(const double *)P.arr[0], (const double *)P.arr[1],
                                            (const double *)P.arr[2], (const double *)P.arr[3],
                                            (const double *)P.arr[4]};
                    double **dst = (double **)A.t[t].arr;
                    dst[0][d] = src[0][q];
                    dst[1][d] = src[1][q];
                    dst[2][d] = src[2][q] * f64;
                    dst[3][d] = src[3][q] * f64;
                    dst[4][d] = src[4][q] * f64;
                } else {
                    ((int32_t *)A.t[t].arr[0])[d] = ((const int32_t *)P.arr[0])[q];
                    ((float *)A.t[t].arr[1])[d] = ((const float *)P.arr[1])[q];
                    ((float *)A.t[t].arr[2])[d] = ((const float *)P.arr[2])[q];
                    for (int c = 3; c < 6; c++)
                        ((float *)A.t[t].arr[c])[d] = ((const float *)P.arr[c])[q] * f32;
                }
            }
        }
        run += all;
        __syncthreads();   // wcnt is rewritten by the next k
    }
}

__global__ void k_pair_commit(const int32_t *__restrict__ off, PairArgs A,
                              uint32_t *__restrict__ err) {
    const int total = off[A.nblk_total];
    if (total == 0) return;
    for (int t = 0; t < 2; t++)
        if ((int64_t)A.t[t].nslots[0] + total > A.t[t].cap) {
            atomicOr(err, FFPIC_ERR_CAPACITY);
            return;
        }
    A.t[0].nslots[0] += total;
    A.t[1].nslots[0] += total;
}

PairTarget target(ffpic_ctx *c, int s) {
    PairTarget T{};
    for (int a = 0; a < c->sp[s].narr; a++) T.arr[a] = c->sp[s].cur[a];
    T.nslots = c->nslots + s;
    T.cap = c->sp[s].cap;
    return T;
}

}  // namespace

int pair_block_slots() { return kPairSlots; }

void create_pairs(ffpic_ctx *c) {
    if (!(c->d.gamma_th > 0.0)) return;
    const int sp[2] = {c->d.pair_species[0], c->d.pair_species[1]};
    // the number of new slots is known only on the device: from here on the
    // launches of both species cover all their slots (each kernel stops at
    // the device count)
    for (int h = 0; h < 2; h++) c->sp[sp[h]].nub = c->sp[sp[h]].cap;
    int nb[2];
    for (int h = 0; h < 2; h++) nb[h] = (int)((c->sp[sp[h]].nub + kPairSlots - 1) / kPairSlots);
    const int ntot = nb[0] + nb[1];
    if (ntot > c->pair_blocks) throw std::runtime_error("pair block table too small");
    PairArgs A{};
    A.t[0] = target(c, sp[0]);
    A.t[1] = target(c, sp[1]);
    A.gth2 = c->d.gamma_th * c->d.gamma_th;
    A.us = sqrt(c->d.gamma_s * c->d.gamma_s - 1.0);
    A.nblk_total = ntot;
    // block counts of parent species 0, then 1, then the zero entry
    zero_counters(c, c->pair_cnt + ntot, 1);
    int first = 0;
    for (int h = 0; h < 2; h++) {
        if (nb[h] > 0) {
            auto k = c->fp64 ? k_pair_count<true> : k_pair_count<false>;
            hipLaunchKernelGGL(k, dim3(nb[h]), dim3(kPairWG), 0, c->stream, target(c, sp[h]),
                               (int)c->sp[sp[h]].nub, c->nslots + sp[h], A.gth2,
                               c->pair_cnt + first);
        }
        first += nb[h];
    }
    exclusive_scan_i32(c, c->pair_cnt, c->pair_off, (int64_t)ntot + 1);
    first = 0;
    for (int h = 0; h < 2; h++) {
        if (nb[h] > 0) {
            auto k = c->fp64 ? k_pair_write<true> : k_pair_write<false>;
            hipLaunchKernelGGL(k, dim3(nb[h]), dim3(kPairWG), 0, c->stream, target(c, sp[h]),
                               (int)c->sp[sp[h]].nub, c->nslots + sp[h], c->pair_off + first,
                               c->pair_off + ntot, A);
        }
        first += nb[h];
    }
    hipLaunchKernelGGL(k_pair_commit, dim3(1), dim3(1), 0, c->stream, c->pair_off, A, c->err);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
