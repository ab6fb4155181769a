// FP64 particle push and charge-conserving deposit (plain FP64 GPU path).
//
// One thread per particle slot.  State per particle: r, theta, u_r,
// u_theta, u_phi (FP64 SoA); a dead slot has r = -1 until the next sort.
// The arithmetic follows the plain FP64 definition step by step and this
// file is compiled without FP contraction, so the path rounds every
// operation as written; currents are accumulated with FP64 atomics.
//
// Push (Sect. 3): eq. (motion) integrated with the Boris rotation; the
// Landau-Lifshitz force g with the effective field of eq. (bperp) is added
// explicitly with the time-centred velocity.  The particle is moved in the
// local Cartesian frame at azimuth 0 and rotated back to the meridional
// plane.  Deposit: zigzag (relay-point) split of the move in logical
// coordinates (log r / dlog, theta / dtheta), charge fluxes through the dual
// faces (exact discrete charge conservation), azimuthal current from v_phi
// at the mid-point.
#include "device_common.h"

namespace ffpic {

struct P64 {
    int nr, nth, ld;
    double rmin, r_abs, dlog, dth, dt;
    const double *rn, *thn;
    double Q, wq, rr;
};

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

__device__ __forceinline__ double hv(const double *F, int ld, int nth, int i, int k, double par) {
    if (k < 0) return par * F[ix(ld, i, 0)];
    if (k >= nth) return par * F[ix(ld, i, nth - 1)];
    return F[ix(ld, i, k)];
}

__device__ __forceinline__ double bil(const double *F, int ld, int nth, Lin lr, Lin lt,
                                      bool thalf, double par) {
    double v00, v10, v01, v11;
    if (thalf) {
        v00 = hv(F, ld, nth, lr.lo, lt.lo, par);
        v10 = hv(F, ld, nth, lr.lo + 1, lt.lo, par);
        v01 = hv(F, ld, nth, lr.lo, lt.lo + 1, par);
        v11 = hv(F, ld, nth, lr.lo + 1, lt.lo + 1, par);
    } else {
        v00 = F[ix(ld, lr.lo, lt.lo)];
        v10 = F[ix(ld, lr.lo + 1, lt.lo)];
        v01 = F[ix(ld, lr.lo, lt.lo + 1)];
        v11 = F[ix(ld, lr.lo + 1, lt.lo + 1)];
    }
    return (1.0 - lr.w) * (1.0 - lt.w) * v00 + lr.w * (1.0 - lt.w) * v10 +
           (1.0 - lr.w) * lt.w * v01 + lr.w * lt.w * v11;
}

__device__ __forceinline__ void boris_rr(double u[3], const double E[3], const double B[3],
                                         double dt, double wq, double rr) {
    double h = 0.5 * dt * wq;
    double um[3], t[3], sv[3], up[3], uL[3];
    for (int k = 0; k < 3; k++) um[k] = u[k] + h * E[k];
    double gm = sqrt(1.0 + (um[0] * um[0] + um[1] * um[1] + um[2] * um[2]));
    for (int k = 0; k < 3; k++) t[k] = h * B[k] / gm;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int k = 0; k < 3; k++) sv[k] = 2.0 * t[k] / (1.0 + t2);
    double c0 = um[1] * t[2] - um[2] * t[1];
    double c1 = um[2] * t[0] - um[0] * t[2];
    double c2 = um[0] * t[1] - um[1] * t[0];
    up[0] = um[0] + c0; up[1] = um[1] + c1; up[2] = um[2] + c2;
    c0 = up[1] * sv[2] - up[2] * sv[1];
    c1 = up[2] * sv[0] - up[0] * sv[2];
    c2 = up[0] * sv[1] - up[1] * sv[0];
    uL[0] = um[0] + c0 + h * E[0];
    uL[1] = um[1] + c1 + h * E[1];
    uL[2] = um[2] + c2 + h * E[2];
    if (rr != 0.0) {
        double ub[3], beta[3], Fv[3];
        for (int k = 0; k < 3; k++) ub[k] = 0.5 * (u[k] + uL[k]);
        double gb = sqrt(1.0 + (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]));
        for (int k = 0; k < 3; k++) beta[k] = ub[k] / gb;
        Fv[0] = E[0] + (beta[1] * B[2] - beta[2] * B[1]);
        Fv[1] = E[1] + (beta[2] * B[0] - beta[0] * B[2]);
        Fv[2] = E[2] + (beta[0] * B[1] - beta[1] * B[0]);
        double be = beta[0] * E[0] + beta[1] * E[1] + beta[2] * E[2];
        double bp2 = (Fv[0] * Fv[0] + Fv[1] * Fv[1] + Fv[2] * Fv[2]) - be * be;
        if (bp2 < 0.0) bp2 = 0.0;
        double x0 = Fv[1] * B[2] - Fv[2] * B[1];
        double x1 = Fv[2] * B[0] - Fv[0] * B[2];
        double x2 = Fv[0] * B[1] - Fv[1] * B[0];
        uL[0] = uL[0] + dt * rr * (x0 + be * E[0] - gb * gb * bp2 * beta[0]);
        uL[1] = uL[1] + dt * rr * (x1 + be * E[1] - gb * gb * bp2 * beta[1]);
        uL[2] = uL[2] + dt * rr * (x2 + be * E[2] - gb * gb * bp2 * beta[2]);
    }
    u[0] = uL[0]; u[1] = uL[1]; u[2] = uL[2];
}

__global__ void __launch_bounds__(256) k_push64(
    P64 p, int nub, const int32_t *__restrict__ nslots, const uint8_t *__restrict__ kill,
    const double *__restrict__ Er, const double *__restrict__ Et, const double *__restrict__ Ep,
    const double *__restrict__ Br, const double *__restrict__ Bt, const double *__restrict__ Bp,
    double *__restrict__ R, double *__restrict__ TH, double *__restrict__ UR,
    double *__restrict__ UT, double *__restrict__ UP, double *__restrict__ Jr,
    double *__restrict__ Jt, double *__restrict__ Jp, unsigned long long *__restrict__ removed,
    uint32_t *__restrict__ err) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    bool live = q < nub && q < nslots[0];
    double r = live ? R[q] : -1.0;
    live = live && r > 0.0;
    bool killed = false, star = false, absb = false;
    if (live) {
        double th = TH[q];
        int i, j;
        double a, b;
        locate64(p.nr, p.nth, p.rmin, p.dlog, p.dth, p.rn, p.thn, r, th, i, j, a, b);
        if (kill[(size_t)i * p.nth + j]) {
            killed = true;
            R[q] = -1.0;
        } else {
            const int ld = p.ld, nth = p.nth;
            Lin rn = {i, a}, rh = half_r(i, a, p.nr), tn = {j, b}, thh = half_t(j, b);
            double Es[3], Bs[3];
            Es[0] = bil(Er, ld, nth, rh, tn, false, 1.0);
            Es[1] = bil(Et, ld, nth, rn, thh, true, -1.0);
            Es[2] = bil(Ep, ld, nth, rn, tn, false, 1.0);
            Bs[0] = bil(Br, ld, nth, rn, thh, true, 1.0);
            Bs[1] = bil(Bt, ld, nth, rh, tn, false, 1.0);
            Bs[2] = bil(Bp, ld, nth, rh, thh, true, -1.0);
            double st = sin(th), ct = cos(th);
            double E[3] = {Es[0] * st + Es[1] * ct, Es[2], Es[0] * ct - Es[1] * st};
            double B[3] = {Bs[0] * st + Bs[1] * ct, Bs[2], Bs[0] * ct - Bs[1] * st};
            double ur = UR[q], ut = UT[q], up = UP[q];
            double u[3] = {ur * st + ut * ct, up, ur * ct - ut * st};
            boris_rr(u, E, B, p.dt, p.wq, p.rr);
            double g = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
            if (!isfinite(g)) atomicOr(err, FFPIC_ERR_NONFINITE);
            double v0 = u[0] / g, v1 = u[1] / g, v2 = u[2] / g;
            double x = r * st + p.dt * v0, y = p.dt * v1, z = r * ct + p.dt * v2;
            double w = sqrt(x * x + y * y);
            double cp = w > 0.0 ? x / w : 1.0, sp = w > 0.0 ? y / w : 0.0;
            double ux = cp * u[0] + sp * u[1], uy = -sp * u[0] + cp * u[1], uz = u[2];
            double r2 = sqrt(w * w + z * z);
            double th2 = atan2(w, z);
            if (!(r2 >= p.rmin)) {
                star = true;
                R[q] = -1.0;
            } else if (r2 >= p.r_abs) {
                absb = true;
                R[q] = -1.0;
            } else {
                double st2 = w / r2, ct2 = z / r2;
                int i2, j2;
                double a2, b2;
                locate64(p.nr, p.nth, p.rmin, p.dlog, p.dth, p.rn, p.thn, r2, th2, i2, j2, a2, b2);
                int di = i2 - i, dj = j2 - j;
                if (di > 1 || di < -1 || dj > 1 || dj < -1) atomicOr(err, FFPIC_ERR_CFL);
                // zigzag deposit in coordinates relative to the start cell
                double x1 = a, y1 = b, x2 = di + a2, y2 = dj + b2;
                double xr = fmin((di < 0 ? di : 0) + 1.0, fmax((double)(di > 0 ? di : 0), 0.5 * (x1 + x2)));
                double yr = fmin((dj < 0 ? dj : 0) + 1.0, fmax((double)(dj > 0 ? dj : 0), 0.5 * (y1 + y2)));
                double Q = p.Q;
                double fx1 = Q * (xr - x1), fy1 = Q * (yr - y1);
                double fx2 = Q * (x2 - xr), fy2 = Q * (y2 - yr);
                double wx1 = 0.5 * (x1 + xr), wy1 = 0.5 * (y1 + yr);
                double wx2 = 0.5 * (xr + x2) - di, wy2 = 0.5 * (yr + y2) - dj;
                gadd(&Jr[ix(ld, i, j)], fx1 * (1.0 - wy1));
                gadd(&Jr[ix(ld, i, j + 1)], fx1 * wy1);
                gadd(&Jt[ix(ld, i, j)], fy1 * (1.0 - wx1));
                gadd(&Jt[ix(ld, i + 1, j)], fy1 * wx1);
                gadd(&Jr[ix(ld, i2, j2)], fx2 * (1.0 - wy2));
                gadd(&Jr[ix(ld, i2, j2 + 1)], fx2 * wy2);
                gadd(&Jt[ix(ld, i2, j2)], fy2 * (1.0 - wx2));
                gadd(&Jt[ix(ld, i2 + 1, j2)], fy2 * wx2);
                double xm = 0.5 * (x1 + x2), ym = 0.5 * (y1 + y2);
                int im = (int)floor(xm), jm = (int)floor(ym);
                if (i + im > p.nr - 1) im = p.nr - 1 - i;
                if (j + jm > p.nth - 1) jm = p.nth - 1 - j;
                double wx = xm - im, wy = ym - jm;
                double qv = Q * v1;
                gadd(&Jp[ix(ld, i + im, j + jm)], qv * (1.0 - wx) * (1.0 - wy));
                gadd(&Jp[ix(ld, i + im + 1, j + jm)], qv * wx * (1.0 - wy));
                gadd(&Jp[ix(ld, i + im, j + jm + 1)], qv * (1.0 - wx) * wy);
                gadd(&Jp[ix(ld, i + im + 1, j + jm + 1)], qv * wx * wy);
                R[q] = r2;
                TH[q] = th2;
                UR[q] = ux * st2 + uz * ct2;
                UT[q] = ux * ct2 - uz * st2;
                UP[q] = uy;
            }
        }
    }
    count_wave(&removed[1], killed);
    count_wave(&removed[2], star);
    count_wave(&removed[3], absb);
}

void push64(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    if (S.nub == 0) return;
    P64 p;
    p.nr = c->nr; p.nth = c->nth; p.ld = c->ld;
    p.rmin = c->d.rmin; p.r_abs = c->d.r_abs; p.dlog = c->dlog; p.dth = c->dth; p.dt = c->dt;
    p.rn = c->dtab64[T_RN];
    p.thn = c->dtab64[T_THN];
    double qm = S.qm;
    p.Q = (qm > 0 ? 1.0 : -1.0) * S.weight;
    p.wq = c->d.omega_b * qm;
    p.rr = c->d.rr_coef * fabs(qm) * fabs(qm) * fabs(qm);
    double **E = (double **)c->E, **B = (double **)c->B, **J = (double **)c->J;
    double **a = (double **)S.cur;
    int nb = (int)((S.nub + 255) / 256);
    hipLaunchKernelGGL(k_push64, dim3(nb), dim3(256), 0, c->stream, p, (int)S.nub,
                       c->nslots + s, c->kill, E[0], E[1], E[2], B[0], B[1], B[2], a[0], a[1],
                       a[2], a[3], a[4], J[0], J[1], J[2], c->removed + 4 * s, c->err);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
