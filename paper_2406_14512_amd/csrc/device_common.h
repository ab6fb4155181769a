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
    while (i > 0 && r < rn[i]) i--;
    while (i < nr - 1 && r >= rn[i + 1]) i++;
    double aa = log(r / rn[i]) / dlog;
    if (aa < 0.0) aa = 0.0;
    if (aa > 1.0) aa = 1.0;
    const float gj = (float)th * (float)(1.0 / dth);
    int j = gj > 0.f ? (gj < (float)(nth - 1) ? (int)gj : nth - 1) : 0;
    while (j > 0 && th < thn[j]) j--;
    while (j < nth - 1 && th >= thn[j + 1]) j++;
    double bb = (th - thn[j]) / dth;
    if (bb < 0.0) bb = 0.0;
    if (bb > 1.0) bb = 1.0;
    ci = i; cj = j; a = aa; b = bb;
}

}  // namespace ffpic
