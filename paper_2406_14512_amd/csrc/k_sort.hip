// Stable sort of each species by cell (key = i*nth + j), with the removal
// of particles in the pure force-free domain folded into the key pass.
//
// 1. key pass: one thread per slot; dead slots and particles in kill cells
//    get key nr*nth (they sort last and are dropped), live ones their cell;
//    live particles are counted (wave-aggregated atomics).
// 2. rocPRIM LSD radix sort of (key, slot) pairs over the key's bit range:
//    LSD radix sort is stable, so equal keys keep their slot order.
// 3. gather pass: the SoA state is permuted into the second buffer.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "device_common.h"

namespace ffpic {

__global__ void k_key64(int nub, const int32_t *__restrict__ nslots, int nr, int nth, double rmin,
                        double dlog, double dth, const double *__restrict__ rn,
                        const double *__restrict__ thn, const uint8_t *__restrict__ kill,
                        double *__restrict__ R, const double *__restrict__ TH,
                        uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                        int32_t *__restrict__ nalive, unsigned long long *__restrict__ removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t dead = (uint32_t)nr * (uint32_t)nth;
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
    count_wave_i(nalive, key != dead);
    count_wave(&removed[1], killed);
}

__global__ void k_key32(int nub, const int32_t *__restrict__ nslots, int nr, int nth,
                        const uint8_t *__restrict__ kill, int32_t *__restrict__ CELL,
                        uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                        int32_t *__restrict__ nalive, unsigned long long *__restrict__ removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t dead = (uint32_t)nr * (uint32_t)nth;
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
    count_wave_i(nalive, key != dead);
    count_wave(&removed[1], killed);
}

template <typename T>
__global__ void k_gather(int nub, const int32_t *__restrict__ nalive,
                         const uint32_t *__restrict__ perm, const T *__restrict__ src,
                         T *__restrict__ dst) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub || q >= nalive[0]) return;
    dst[q] = src[perm[q]];
}

__global__ void k_set_slots(int32_t *nslots, const int32_t *nalive) { nslots[0] = nalive[0]; }

__global__ void k_zero_i32(int32_t *p, int n) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0;
}

void zero_counters(ffpic_ctx *c, int32_t *p, int n) {
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 63) / 64), dim3(64), 0, c->stream, p, n);
}

static int key_bits(const ffpic_ctx *c) {
    uint64_t dead = (uint64_t)c->nr * (uint64_t)c->nth;
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

static void sort_common(ffpic_ctx *c, int s, bool do_sort) {
    ffpic::Species &S = c->sp[s];
    int nub = (int)S.nub;
    if (nub == 0) return;
    int nb = (nub + 255) / 256;
    int32_t *nal = c->nalive + s;
    zero_counters(c, nal, 1);
    if (c->fp64) {
        hipLaunchKernelGGL(k_key64, dim3(nb), dim3(256), 0, c->stream, nub, c->nslots + s, c->nr,
                           c->nth, c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN], c->dtab64[T_THN],
                           c->kill, (double *)S.cur[0], (const double *)S.cur[1], c->keys[0],
                           c->vals[0], nal, c->removed + 4 * s);
    } else {
        hipLaunchKernelGGL(k_key32, dim3(nb), dim3(256), 0, c->stream, nub, c->nslots + s, c->nr,
                           c->nth, c->kill, (int32_t *)S.cur[0], c->keys[0], c->vals[0], nal,
                           c->removed + 4 * s);
    }
    FFPIC_LAUNCH_CHECK();
    if (!do_sort) return;
    size_t bytes = c->sort_tmp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(c->sort_tmp, bytes, c->keys[0], c->keys[1],
                                             c->vals[0], c->vals[1], (unsigned int)nub, 0,
                                             key_bits(c), c->stream);
    if (e != hipSuccess) throw std::runtime_error("rocprim radix sort failed");
    for (int a = 0; a < S.narr; a++) {
        if (c->fp64)
            hipLaunchKernelGGL(k_gather<uint64_t>, dim3(nb), dim3(256), 0, c->stream, nub, nal,
                               c->vals[1], (const uint64_t *)S.cur[a], (uint64_t *)S.alt[a]);
        else
            hipLaunchKernelGGL(k_gather<uint32_t>, dim3(nb), dim3(256), 0, c->stream, nub, nal,
                               c->vals[1], (const uint32_t *)S.cur[a], (uint32_t *)S.alt[a]);
    }
    FFPIC_LAUNCH_CHECK();
    for (int a = 0; a < S.narr; a++) std::swap(S.cur[a], S.alt[a]);
    hipLaunchKernelGGL(k_set_slots, dim3(1), dim3(1), 0, c->stream, c->nslots + s, nal);
    FFPIC_LAUNCH_CHECK();
}

void sort_species(ffpic_ctx *c, int s) { sort_common(c, s, true); }
void kill_species(ffpic_ctx *c, int s) { sort_common(c, s, false); }

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
    // recompute keys of the current order without killing or sorting
    ffpic::Species &S = c->sp[s];
    int nkeys = c->nr * c->nth;
    int nal = 0;
    if (S.nub > 0) {
        // a key pass on a copy of the kill-free state: use an all-zero kill
        uint8_t *nok = nullptr;
        size_t ncell = (size_t)c->nr * c->nth;
        if (hipMalloc(&nok, ncell) != hipSuccess) throw std::runtime_error("hipMalloc failed");
        (void)hipMemsetAsync(nok, 0, ncell, c->stream);
        uint8_t *saved = c->kill;
        c->kill = nok;
        sort_common(c, s, false);
        c->kill = saved;
        (void)hipMemcpyAsync(&nal, c->nalive + s, sizeof(int), hipMemcpyDeviceToHost, c->stream);
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(nok);
    }
    hipLaunchKernelGGL(k_offsets, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream, nal,
                       c->keys[0], nkeys, dev_off);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
