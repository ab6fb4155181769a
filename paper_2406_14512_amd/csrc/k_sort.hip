// Stable sort of each species by cell (key = i*nth + j), with the removal
// of particles in the pure force-free domain folded into the key pass.
//
// 1. key pass: one thread per slot; dead slots and particles in kill cells
//    get the dead key (larger than every live key, so they sort last and
//    are dropped), live ones their cell.  Live particles lie inside the
//    absorbing radius, so the dead key is the first cell of the row past
//    it, which keeps the key within 24 bits on a 4096^2 grid (three 8-bit
//    radix passes instead of four).
// 2. rocPRIM LSD radix sort of (key, slot) pairs over the key's bit range:
//    LSD radix sort is stable, so equal keys keep their slot order.
// 3. the live count is the position of the first dead key in the sorted
//    keys (binary search), so no pass of the sort contends on a counter.
// 4. gather pass: the SoA state is permuted into the second buffer.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "device_common.h"

namespace ffpic {

__global__ void k_key64(int nub, const int32_t *__restrict__ nslots, int nr, int nth, double rmin,
                        double dlog, double dth, const double *__restrict__ rn,
                        const double *__restrict__ thn, const uint8_t *__restrict__ kill,
                        uint32_t dead, double *__restrict__ R, const double *__restrict__ TH,
                        uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                        unsigned long long *__restrict__ removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t key = dead;
    bool killed = false;
    if (q < nslots[0]) {
        double r = R[q];
        if (r > 0.0) {
            int i, j;
            double a, b;
            locate64(nr, nth, rmin, dlog, dth, rn, thn, r, TH[q], i, j, a, b);
            if (kill[(size_t)i * nth + j]) {
                killed = true;
                R[q] = -1.0;
            } else {
                key = (uint32_t)i * (uint32_t)nth + (uint32_t)j;
            }
        }
    }
    keys[q] = key;
    vals[q] = (uint32_t)q;
    count_wave(&removed[1], killed);
}

__global__ void k_key32(int nub, const int32_t *__restrict__ nslots, int nth,
                        const uint8_t *__restrict__ kill, uint32_t dead,
                        int32_t *__restrict__ CELL, uint32_t *__restrict__ keys,
                        uint32_t *__restrict__ vals, unsigned long long *__restrict__ removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t key = dead;
    bool killed = false;
    if (q < nslots[0]) {
        int c = CELL[q];
        if (c >= 0) {
            int i = c >> 16, j = c & 0xffff;
            if (kill[(size_t)i * nth + j]) {
                killed = true;
                CELL[q] = -1;
            } else {
                key = (uint32_t)i * (uint32_t)nth + (uint32_t)j;
            }
        }
    }
    keys[q] = key;
    vals[q] = (uint32_t)q;
    count_wave(&removed[1], killed);
}

// number of live keys = index of the first dead key in the sorted keys
__global__ void k_count_sorted(int nub, const uint32_t *__restrict__ keys, uint32_t dead,
                               int32_t *__restrict__ nalive, int32_t *__restrict__ nslots) {
    int lo = 0, hi = nub;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (keys[mid] < dead) lo = mid + 1; else hi = mid;
    }
    nalive[0] = lo;
    if (nslots) nslots[0] = lo;
}

// live count of unsorted keys: block reduction, one atomic per block
__global__ void __launch_bounds__(256) k_count_live(int nub, const uint32_t *__restrict__ keys,
                                                    uint32_t dead, int32_t *__restrict__ nalive) {
    __shared__ int part[4];
    int c = 0;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < nub; q += gridDim.x * 256) c += keys[q] < dead;
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(nalive, part[0] + part[1] + part[2] + part[3]);
}

// permutes all state arrays of a species in one pass over the permutation
template <typename T, int NA>
struct PtrSet {
    const T *src[NA];
    T *dst[NA];
};

template <typename T, int NA>
__global__ void k_gather_set(int nub, const int32_t *__restrict__ nalive,
                             const uint32_t *__restrict__ perm, PtrSet<T, NA> P) {
    const int n = min(nub, nalive[0]);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const uint32_t s = perm[q];
        T v[NA];
#pragma unroll
        for (int a = 0; a < NA; a++) v[a] = P.src[a][s];
#pragma unroll
        for (int a = 0; a < NA; a++) P.dst[a][q] = v[a];
    }
}

__global__ void k_zero_i32(int32_t *p, int n) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0;
}

void zero_counters(ffpic_ctx *c, int32_t *p, int n) {
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 63) / 64), dim3(64), 0, c->stream, p, n);
}

// first key past every live one (see the header comment)
static uint32_t dead_key(const ffpic_ctx *c) {
    double xa = std::log(c->d.r_abs / c->d.rmin) / c->dlog;
    int64_t iabs = (int64_t)std::floor(xa);
    int64_t k = (iabs + 1) * (int64_t)c->nth;
    int64_t all = (int64_t)c->nr * c->nth;
    return (uint32_t)(iabs + 1 < c->nr ? k : all);
}

int sort_key_bits(const ffpic_ctx *c) {
    uint64_t dead = dead_key(c);
    int bits = 1;
    while ((1ull << bits) <= dead) bits++;
    return bits;
}

size_t sort_temp_bytes(int64_t cap, int bits) {
    size_t bytes = 0;
    if (cap <= 0) return 0;
    hipError_t e = rocprim::radix_sort_pairs((void *)nullptr, bytes, (uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (unsigned int)cap, 0, bits);
    if (e != hipSuccess) throw std::runtime_error("rocprim temp size query failed");
    return bytes;
}

static void key_pass(ffpic_ctx *c, int s, uint32_t dead) {
    ffpic::Species &S = c->sp[s];
    int nub = (int)S.nub;
    int nb = (nub + 255) / 256;
    if (c->fp64) {
        hipLaunchKernelGGL(k_key64, dim3(nb), dim3(256), 0, c->stream, nub, c->nslots + s, c->nr,
                           c->nth, c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN], c->dtab64[T_THN],
                           c->kill, dead, (double *)S.cur[0], (const double *)S.cur[1],
                           c->keys[0], c->vals[0], c->removed + 4 * s);
    } else {
        hipLaunchKernelGGL(k_key32, dim3(nb), dim3(256), 0, c->stream, nub, c->nslots + s, c->nth,
                           c->kill, dead, (int32_t *)S.cur[0], c->keys[0], c->vals[0],
                           c->removed + 4 * s);
    }
    FFPIC_LAUNCH_CHECK();
}

void sort_species(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    int nub = (int)S.nub;
    if (nub == 0) return;
    uint32_t dead = dead_key(c);
    key_pass(c, s, dead);
    size_t bytes = c->sort_tmp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(c->sort_tmp, bytes, c->keys[0], c->keys[1],
                                             c->vals[0], c->vals[1], (unsigned int)nub, 0,
                                             sort_key_bits(c), c->stream);
    if (e != hipSuccess) throw std::runtime_error("rocprim radix sort failed");
    int32_t *nal = c->nalive + s;
    hipLaunchKernelGGL(k_count_sorted, dim3(1), dim3(1), 0, c->stream, nub, c->keys[1], dead, nal,
                       c->nslots + s);
    int nb = std::min((nub + 255) / 256, 65536);
    if (c->fp64) {
        PtrSet<uint64_t, 5> P;
        for (int a = 0; a < 5; a++) { P.src[a] = (const uint64_t *)S.cur[a]; P.dst[a] = (uint64_t *)S.alt[a]; }
        hipLaunchKernelGGL((k_gather_set<uint64_t, 5>), dim3(nb), dim3(256), 0, c->stream, nub,
                           nal, c->vals[1], P);
    } else {
        PtrSet<uint32_t, 6> P;
        for (int a = 0; a < 6; a++) { P.src[a] = (const uint32_t *)S.cur[a]; P.dst[a] = (uint32_t *)S.alt[a]; }
        hipLaunchKernelGGL((k_gather_set<uint32_t, 6>), dim3(nb), dim3(256), 0, c->stream, nub,
                           nal, c->vals[1], P);
    }
    FFPIC_LAUNCH_CHECK();
    for (int a = 0; a < S.narr; a++) std::swap(S.cur[a], S.alt[a]);
}

// removal of particles in force-free cells without reordering
void kill_species(ffpic_ctx *c, int s) {
    if (c->sp[s].nub == 0) return;
    key_pass(c, s, dead_key(c));
}

// cell offsets from the current (sorted) order: off[k] = first slot whose
// key is >= k, found by binary search over the live slots
__global__ void k_offsets(int nalive_host, const uint32_t *__restrict__ keys, int nkeys,
                          int32_t *__restrict__ off) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nkeys) return;
    int lo = 0, hi = nalive_host;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((int)keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    off[k] = lo;
}

void sort_offsets(ffpic_ctx *c, int s, int32_t *dev_off) {
    // keys of the current order (no removal): all-zero kill flags
    ffpic::Species &S = c->sp[s];
    int nkeys = c->nr * c->nth;
    int nal = 0;
    if (S.nub > 0) {
        uint8_t *nok = nullptr;
        size_t ncell = (size_t)c->nr * c->nth;
        if (hipMalloc(&nok, ncell) != hipSuccess) throw std::runtime_error("hipMalloc failed");
        (void)hipMemsetAsync(nok, 0, ncell, c->stream);
        uint8_t *saved = c->kill;
        c->kill = nok;
        uint32_t dead = dead_key(c);
        key_pass(c, s, dead);
        c->kill = saved;
        zero_counters(c, c->nalive + s, 1);
        hipLaunchKernelGGL(k_count_live, dim3(256), dim3(256), 0, c->stream, (int)S.nub,
                           c->keys[0], dead, c->nalive + s);
        (void)hipMemcpyAsync(&nal, c->nalive + s, sizeof(int), hipMemcpyDeviceToHost, c->stream);
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(nok);
    }
    hipLaunchKernelGGL(k_offsets, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream, nal,
                       c->keys[0], nkeys, dev_off);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
