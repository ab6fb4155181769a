// Staggered bilinear gather of the six field components at a particle, in
// FP64 arithmetic on fields of element type T (double, or float for the
// FP32-mixed fields): the interpolation of the FP64 push, shared by the
// diagnostics that need the field at the particles.
//
// Positions in logical coordinates: cell (i, j) and offsets (a, b) in
// log r / dlog and theta / dtheta.  Components on half rows or half columns
// use the half-cell weights; the polar half-columns beyond the axes take the
// ghost value of the first / last column times the component's axis parity
// (-1 for E_theta and B_phi).  Radial half rows are clamped to the grid.
#pragma once

#include "device_common.h"

namespace ffpic {

struct Lin {
    int lo;
    double w;
};

__device__ __forceinline__ Lin half_r(int i, double a, int nr) {
    Lin l;
    if (a >= 0.5) { l.lo = i; l.w = a - 0.5; } else { l.lo = i - 1; l.w = a + 0.5; }
    if (l.lo < 0) { l.lo = 0; l.w = 0.0; }
    if (l.lo > nr - 2) { l.lo = nr - 2; l.w = 1.0; }
    return l;
}
__device__ __forceinline__ Lin half_t(int j, double b) {
    Lin l;
    if (b >= 0.5) { l.lo = j; l.w = b - 0.5; } else { l.lo = j - 1; l.w = b + 0.5; }
    return l;
}

template <typename T>
__device__ __forceinline__ double hv(const T *F, int ld, int nth, int i, int k, double par) {
    if (k < 0) return par * (double)F[ix(ld, i, 0)];
    if (k >= nth) return par * (double)F[ix(ld, i, nth - 1)];
    return (double)F[ix(ld, i, k)];
}

template <typename T>
__device__ __forceinline__ double bil(const T *F, int ld, int nth, Lin lr, Lin lt, bool thalf,
                                      double par) {
    double v00, v10, v01, v11;
    if (thalf) {
        v00 = hv(F, ld, nth, lr.lo, lt.lo, par);
        v10 = hv(F, ld, nth, lr.lo + 1, lt.lo, par);
        v01 = hv(F, ld, nth, lr.lo, lt.lo + 1, par);
        v11 = hv(F, ld, nth, lr.lo + 1, lt.lo + 1, par);
    } else {
        v00 = (double)F[ix(ld, lr.lo, lt.lo)];
        v10 = (double)F[ix(ld, lr.lo + 1, lt.lo)];
        v01 = (double)F[ix(ld, lr.lo, lt.lo + 1)];
        v11 = (double)F[ix(ld, lr.lo + 1, lt.lo + 1)];
    }
    return (1.0 - lr.w) * (1.0 - lt.w) * v00 + lr.w * (1.0 - lt.w) * v10 +
           (1.0 - lr.w) * lt.w * v01 + lr.w * lt.w * v11;
}

// spherical components (r, theta, phi) of E and B at offsets (a, b) of cell (i, j)
template <typename T>
__device__ __forceinline__ void gather_eb(const T *Er, const T *Et, const T *Ep, const T *Br,
                                          const T *Bt, const T *Bp, int nr, int nth, int ld,
                                          int i, int j, double a, double b, double Es[3],
                                          double Bs[3]) {
    Lin rn = {i, a}, rh = half_r(i, a, nr), tn = {j, b}, thh = half_t(j, b);
    Es[0] = bil(Er, ld, nth, rh, tn, false, 1.0);
    Es[1] = bil(Et, ld, nth, rn, thh, true, -1.0);
    Es[2] = bil(Ep, ld, nth, rn, tn, false, 1.0);
    Bs[0] = bil(Br, ld, nth, rn, thh, true, 1.0);
    Bs[1] = bil(Bt, ld, nth, rh, tn, false, 1.0);
    Bs[2] = bil(Bp, ld, nth, rh, thh, true, -1.0);
}

}  // namespace ffpic
