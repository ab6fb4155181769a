// Device helpers shared by the kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ffpic_internal.h"

namespace ffpic {

__device__ __forceinline__ size_t ix(int ld, int i, int j) {
    return (size_t)i * (size_t)ld + (size_t)j;
}

// hardware float / double atomic add to global memory, device scope,
// no return value
template <typename R>
__device__ __forceinline__ void gadd(R *p, R v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// blending function of eq. (transition) with the two force-free domains of
// Table 1 (see ffpic_desc::psi_thr); evaluated in FP64
__device__ __forceinline__ double blend(double psi, double t0, double t1, double t2, double t3) {
    if (psi >= t3) return 1.0;
    if (psi < t0) return 1.0;
    if (psi < t1) return (t1 - psi) / (t1 - t0);
    if (psi > t2) return (psi - t2) / (t3 - t2);
    return 0.0;
}

// wave-aggregated increment of a 64-bit counter: one atomic per wave
__device__ __forceinline__ void count_wave(unsigned long long *ctr, bool pred) {
    unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    int leader = __ffsll((long long)m) - 1;
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

__device__ __forceinline__ int count_wave_i(int *ctr, bool pred) {
    unsigned long long m = __ballot(pred);
    if (m == 0ull) return 0;
    int leader = __ffsll((long long)m) - 1;
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(ctr, (int)__popcll(m));
    return (int)__popcll(m);
}

// The job of a grouped launch that holds work item `item` (job k owns items
// [starts[k], starts[k + 1]), starts ascending): the workgroup's threads test
// the jobs side by side and the one that matches writes its index to *slot,
// to be read after the next barrier.  One round of loads, where a bisection
// would wait for one load per halving.
__device__ __forceinline__ void find_job(const int *__restrict__ starts, int njobs, int item,
                                         int *slot) {
    for (int t = (int)threadIdx.x; t < njobs; t += (int)blockDim.x)
        if (starts[t] <= item && item < starts[t + 1]) *slot = t;
}

// A table entry that every lane reads alike (the job of a grouped launch),
// copied into scalar registers: the first threads of the workgroup load one
// word each into the LDS array `stage` (kJobWords words), and after a
// barrier every wave takes the words from there with readfirstlane.  The
// values then stay in scalar registers (or their spill lanes) through the
// loops that use them: a load from device memory that the compiler knows
// to be uniform and unchanging would instead be repeated inside those
// loops.  Only the first `bytes` bytes are copied.  Every thread of the
// workgroup calls it; `stage` must not be written again before the next
// barrier of all threads.
constexpr int kJobWords = 96;
template <typename T>
__device__ __forceinline__ T stage_uniform(const T *src, uint32_t *stage,
                                           size_t bytes = sizeof(T)) {
    static_assert(sizeof(T) % 4 == 0 && sizeof(T) <= 4 * kJobWords, "whole words, fits the stage");
    const int words = (int)(bytes / 4);
    if ((int)threadIdx.x < words)
        stage[threadIdx.x] = reinterpret_cast<const uint32_t *>(src)[threadIdx.x];
    __syncthreads();
    T out{};
    char *d = reinterpret_cast<char *>(&out);
#pragma unroll
    for (int w = 0; w < (int)(sizeof(T) / 4); w++) {
        if (w >= words) break;
        const uint32_t v = __builtin_amdgcn_readfirstlane(stage[w]);
        __builtin_memcpy(d + 4 * w, &v, 4);
    }
    return out;
}

// End of a launch of persistent workgroups that take their work items from
// the counter ctr[0]: each workgroup counts itself finished in ctr[1] after
// its last take (fenced), so the last one to finish knows that no take is
// left and returns both counters to zero for the next launch.
__device__ __forceinline__ void group_done(int *ctr) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&ctr[0], 0);
            atomicExch(&ctr[1], 0);
        }
    }
}

}  // namespace ffpic

namespace ffpic {

// Cell of an FP64 position by comparison against the node tables (so the
// cell is a function of (r, theta) alone, whatever the rounding of the first
// guess), plus the in-cell offsets in log r / dlog and theta / dtheta, in
// [0, 1].  The starting guess is taken in single precision: the comparisons
// settle the cell, and only the offset needs the FP64 logarithm.
__device__ __forceinline__ void locate64(int nr, int nth, double rmin, double dlog, double dth,
                                         const double *rn, const double *thn, double r,
                                         double th, int &ci, int &cj, double &a, double &b) {
    const float gi = __logf((float)(r / rmin)) * (float)(1.0 / dlog);
    int i = gi > 0.f ? (gi < (float)(nr - 1) ? (int)gi : nr - 1) : 0;
    const float gj = (float)th * (float)(1.0 / dth);
    int j = gj > 0.f ? (gj < (float)(nth - 1) ? (int)gj : nth - 1) : 0;
    // the guessed cells' bounding nodes are read together; the walks below
    // keep the pair of the current cell (a guess is off by one at most, as
    // a rule, so they rarely read more)
    double rlo = rn[i], rhi = rn[i + 1], tlo = thn[j], thi = thn[j + 1];
    while (i > 0 && r < rlo) { i--; rhi = rlo; rlo = rn[i]; }
    while (i < nr - 1 && r >= rhi) { i++; rlo = rhi; rhi = rn[i + 1]; }
    double aa = log(r / rlo) / dlog;
    if (aa < 0.0) aa = 0.0;
    if (aa > 1.0) aa = 1.0;
    while (j > 0 && th < tlo) { j--; thi = tlo; tlo = thn[j]; }
    while (j < nth - 1 && th >= thi) { j++; tlo = thi; thi = thn[j + 1]; }
    double bb = (th - tlo) / dth;
    if (bb < 0.0) bb = 0.0;
    if (bb > 1.0) bb = 1.0;
    ci = i; cj = j; a = aa; b = bb;
}

}  // namespace ffpic
