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
// cell is a function of (r, theta) alone, whatever the rounding of log),
// plus the in-cell offsets in log r / dlog and theta / dtheta, in [0, 1].
__device__ __forceinline__ void locate64(int nr, int nth, double rmin, double dlog, double dth,
                                         const double *rn, const double *thn, double r,
                                         double th, int &ci, int &cj, double &a, double &b) {
    int i = (int)floor(log(r / rmin) / dlog);
    if (i < 0) i = 0;
    if (i > nr - 1) i = nr - 1;
    while (i > 0 && r < rn[i]) i--;
    while (i < nr - 1 && r >= rn[i + 1]) i++;
    double aa = log(r / rn[i]) / dlog;
    if (aa < 0.0) aa = 0.0;
    if (aa > 1.0) aa = 1.0;
    int j = (int)floor(th / dth);
    if (j < 0) j = 0;
    if (j > nth - 1) j = nth - 1;
    while (j > 0 && th < thn[j]) j--;
    while (j < nth - 1 && th >= thn[j + 1]) j++;
    double bb = (th - thn[j]) / dth;
    if (bb < 0.0) bb = 0.0;
    if (bb > 1.0) bb = 1.0;
    ci = i; cj = j; a = aa; b = bb;
}

}  // namespace ffpic
