// FP64 particle push and charge-conserving deposit (plain FP64 GPU path).
//
// One thread per particle slot.  State per particle: r, theta, u_r,
// u_theta, u_phi (FP64 SoA); a dead slot has r = -1 until the next sort.
// The per-particle arithmetic follows the plain FP64 definition step by step
// and this file is compiled without FP contraction, so every operation is
// rounded as written; only the order in which currents are summed differs.
//
// Push (Sect. 3): eq. (motion) integrated with the Boris rotation; the
// Landau-Lifshitz force g with the effective field of eq. (bperp) is added
// explicitly with the time-centred velocity (its strength scaled by the
// ramp of Sect. 5); inside the shell around the star only the momentum
// along B is kept.  The particle is moved in the
// local Cartesian frame at azimuth 0 and rotated back to the meridional
// plane.  Deposit: zigzag (relay-point) split of the move in logical
// coordinates (log r / dlog, theta / dtheta), charge fluxes through the dual
// faces (exact discrete charge conservation), azimuthal current from v_phi
// at the mid-point.  Accumulation as in the FP32 path: an LDS patch per
// workgroup over the bounding box of its (cell-sorted) particles, in-cell
// moves summed across each 16-lane row first (DPP, one cell per row and
// pass), one global FP64 atomic per non-zero patch entry.
#include "gather.h"

namespace ffpic {

constexpr int kTile64 = 1024;   // LDS patch entries per component (FP64)

struct P64 {
    int nr, nth, ld;
    double rmin, r_abs, dlog, dth, dt;
    const double *rn, *thn;
    double Q, wq, rr;
    double shell_r;        // r below this: only the momentum along B is kept
};

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

// a DPP lane permutation of a double (both 32-bit halves moved the same way)
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sums eight per-lane values over each 16-lane row, halving the number of
// values at every stage (exchange with lane^1, lane^2, a rotation by four
// lanes, a rotation by eight).  Lane l then holds the row sum of value
// 4*bit0(l) + 2*bit1(l) + bit2(l); keep[] are the four values a lane sums in
// the first stage (values 4..7 on lanes with bit 0 set, 0..3 otherwise),
// pass[] the four its neighbour sums.
__device__ __forceinline__ double row_sum8_64(const double keep[4], const double pass[4], bool b1,
                                              bool b2) {
    double y[4];
#pragma unroll
    for (int m = 0; m < 4; m++) y[m] = keep[m] + dpp64<0xB1>(pass[m]);
    const double z0 = (b1 ? y[2] : y[0]) + dpp64<0x4E>(b1 ? y[0] : y[2]);
    const double z1 = (b1 ? y[3] : y[1]) + dpp64<0x4E>(b1 ? y[1] : y[3]);
    const double w = (b2 ? z1 : z0) + dpp64<0x124>(b2 ? z0 : z1);
    return w + dpp64<0x128>(w);
}

struct Acc64 {
    double *tile;    // nullptr: global mode
    int ti0, tj0, TJ;
    double *g[3];
    int ld;
    __device__ __forceinline__ void add(int comp, int i, int j, double v) const {
        if (tile) atomicAdd(&tile[comp * kTile64 + (i - ti0) * TJ + (j - tj0)], v);
        else gadd(&g[comp][ix(ld, i, j)], v);
    }
};

// five waves per SIMD fit without spills (94 VGPRs); the default allocation
// takes 98 and leaves four
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) k_push64(
    P64 p, int nub, const int32_t *__restrict__ nslots, const uint8_t *__restrict__ kill,
    const double *__restrict__ Er, const double *__restrict__ Et, const double *__restrict__ Ep,
    const double *__restrict__ Br, const double *__restrict__ Bt, const double *__restrict__ Bp,
    double *__restrict__ R, double *__restrict__ TH, double *__restrict__ UR,
    double *__restrict__ UT, double *__restrict__ UP, double *__restrict__ Jr,
    double *__restrict__ Jt, double *__restrict__ Jp, unsigned long long *__restrict__ removed,
    uint32_t *__restrict__ err) {
    __shared__ double tile[3 * kTile64];
    __shared__ int box[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int q = blockIdx.x * blockDim.x + tid;
    // the slot's whole state is loaded at once (a thread past the last slot
    // loads the last one and ignores it; nub >= 1): loaded where first used,
    // behind the branches, each load waited for the one before
    const int qs = min(q, nub - 1);
    const double r0 = R[qs], th0 = TH[qs], ur0 = UR[qs], ut0 = UT[qs], up0 = UP[qs];
    bool live = q < nub && q < nslots[0];
    const double r = live ? r0 : -1.0;
    live = live && r > 0.0;
    double th = 0.0;
    int i = 0, j = 0;
    double a = 0.0, b = 0.0;
    if (live) {
        th = th0;
        locate64(p.nr, p.nth, p.rmin, p.dlog, p.dth, p.rn, p.thn, r, th, i, j, a, b);
    }
    // bounding box of the block's cells
    int imin = live ? i : 1 << 30, imax = live ? i : -1;
    int jmin = live ? j : 1 << 30, jmax = live ? j : -1;
    if (tid == 0) { box[0] = 1 << 30; box[1] = -1; box[2] = 1 << 30; box[3] = -1; }
    __syncthreads();
    for (int o = 32; o >= 1; o >>= 1) {
        imin = min(imin, __shfl_xor(imin, o, 64));
        imax = max(imax, __shfl_xor(imax, o, 64));
        jmin = min(jmin, __shfl_xor(jmin, o, 64));
        jmax = max(jmax, __shfl_xor(jmax, o, 64));
    }
    if (lane == 0 && imax >= 0) {
        atomicMin(&box[0], imin); atomicMax(&box[1], imax);
        atomicMin(&box[2], jmin); atomicMax(&box[3], jmax);
    }
    __syncthreads();
    if (box[1] < 0) return;   // uniform: no live particle in the block
    const int ti0 = box[0] - 1, tj0 = box[2] - 1;
    const int TI = box[1] - box[0] + 4, TJ = box[3] - box[2] + 4;
    const bool use_lds = TI * TJ <= kTile64;
    Acc64 acc{use_lds ? tile : nullptr, ti0, tj0, TJ, {Jr, Jt, Jp}, p.ld};
    // the deposit value this lane adds after the row reduction: component,
    // radial and polar node offsets from the cell (values 0..7 of s[] below)
    const int rl = lane & 15;
    const bool b0 = rl & 1, b1 = rl & 2, b2 = rl & 4;
    const int kq = (b0 ? 4 : 0) + (b1 ? 2 : 0) + (b2 ? 1 : 0);
    const int kcomp = kq < 2 ? 0 : (kq < 4 ? 1 : 2);
    const int kdi = (kq == 3 || kq == 5 || kq == 7) ? 1 : 0;
    const int kdj = (kq == 1 || kq == 6 || kq == 7) ? 1 : 0;
    double *kg = kcomp == 0 ? Jr : (kcomp == 1 ? Jt : Jp);   // global mode
    if (use_lds) {
        for (int e = tid; e < TI * TJ; e += 256) {
            tile[e] = 0.0; tile[kTile64 + e] = 0.0; tile[2 * kTile64 + e] = 0.0;
        }
        __syncthreads();
    }

    bool killed = false, star = false, absb = false;
    bool simple = false, cross = false;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i2 = 0, j2 = 0, di = 0, dj = 0;
    double x1 = 0, y1 = 0, x2 = 0, y2 = 0, v1 = 0;
    if (live && kill[(size_t)i * p.nth + j]) {
        killed = true;
        R[q] = -1.0;
        live = false;
    }
    if (live) {
        double Es[3], Bs[3];
        gather_eb(Er, Et, Ep, Br, Bt, Bp, p.nr, p.nth, p.ld, i, j, a, b, Es, Bs);
        double st, ct;
        sincos(th, &st, &ct);           // one argument reduction for both
        double E[3] = {Es[0] * st + Es[1] * ct, Es[2], Es[0] * ct - Es[1] * st};
        double B[3] = {Bs[0] * st + Bs[1] * ct, Bs[2], Bs[0] * ct - Bs[1] * st};
        const double ur = ur0, ut = ut0, up = up0;
        double u[3] = {ur * st + ut * ct, up, ur * ct - ut * st};
        boris_rr(u, E, B, p.dt, p.wq, p.rr);
        if (r < p.shell_r) {
            // shell around the star (Sect. 5): drop the momentum across B
            const double b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
            if (b2 > 0.0) {
                const double ub = (u[0] * B[0] + u[1] * B[1] + u[2] * B[2]) / b2;
                u[0] = ub * B[0]; u[1] = ub * B[1]; u[2] = ub * B[2];
            }
        }
        double g = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
        if (!isfinite(g)) atomicOr(err, FFPIC_ERR_NONFINITE);
        double v0 = u[0] / g, vv2 = u[2] / g;
        v1 = u[1] / g;
        double x = r * st + p.dt * v0, y = p.dt * v1, z = r * ct + p.dt * vv2;
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
            double a2, b2;
            locate64(p.nr, p.nth, p.rmin, p.dlog, p.dth, p.rn, p.thn, r2, th2, i2, j2, a2, b2);
            di = i2 - i;
            dj = j2 - j;
            bool cfl = di > 1 || di < -1 || dj > 1 || dj < -1;
            if (cfl) atomicOr(err, FFPIC_ERR_CFL);
            x1 = a; y1 = b; x2 = di + a2; y2 = dj + b2;
            R[q] = r2;
            TH[q] = th2;
            UR[q] = ux * st2 + uz * ct2;
            UT[q] = ux * ct2 - uz * st2;
            UP[q] = uy;
            if (di == 0 && dj == 0) {
                // zigzag with both ends in the cell: the two segments share
                // the four faces of the cell, mid-point cell = the cell
                double xr = fmin(1.0, fmax(0.0, 0.5 * (x1 + x2)));
                double yr = fmin(1.0, fmax(0.0, 0.5 * (y1 + y2)));
                double Q = p.Q;
                double fx1 = Q * (xr - x1), fy1 = Q * (yr - y1);
                double fx2 = Q * (x2 - xr), fy2 = Q * (y2 - yr);
                double wx1 = 0.5 * (x1 + xr), wy1 = 0.5 * (y1 + yr);
                double wx2 = 0.5 * (xr + x2), wy2 = 0.5 * (yr + y2);
                s[0] = fx1 * (1.0 - wy1) + fx2 * (1.0 - wy2);
                s[1] = fx1 * wy1 + fx2 * wy2;
                s[2] = fy1 * (1.0 - wx1) + fy2 * (1.0 - wx2);
                s[3] = fy1 * wx1 + fy2 * wx2;
                double xm = 0.5 * (x1 + x2), ym = 0.5 * (y1 + y2);
                int im = (int)floor(xm), jm = (int)floor(ym);
                if (i + im > p.nr - 1) im = p.nr - 1 - i;
                if (j + jm > p.nth - 1) jm = p.nth - 1 - j;
                if (im == 0 && jm == 0) {
                    double wx = xm, wy = ym, qv = Q * v1;
                    s[4] = qv * (1.0 - wx) * (1.0 - wy);
                    s[5] = qv * wx * (1.0 - wy);
                    s[6] = qv * (1.0 - wx) * wy;
                    s[7] = qv * wx * wy;
                    simple = true;
                } else {
                    cross = true;
                }
            } else if (!cfl) {
                cross = true;
            } else {
                cross = true;     // flagged; deposit anyway (indices stay in range)
            }
        }
    }
    // ---- in-cell moves, one cell per 16-lane row and pass: the lanes of a
    // row whose cell is that of the row's first pending lane sum their eight
    // values over the row, and lanes 0..7 of the row add one sum each.  Every
    // pass retires at least the first pending lane of each row, so the loop
    // ends within 16 passes with every in-cell move deposited.
    bool pend = simple;
    const int c = (i << 16) | j;
    double rk[4], rp[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        rk[e] = b0 ? s[4 + e] : s[e];
        rp[e] = b0 ? s[e] : s[4 + e];
    }
#pragma unroll 1
    while (true) {
        const unsigned long long m = __ballot(pend);
        if (m == 0ull) break;
        const unsigned rowm = (unsigned)(m >> (lane & 48)) & 0xffffu;
        const int src = rowm ? (lane & 48) + __builtin_ctz(rowm) : lane;
        const int lc = __shfl(c, src, 64);
        const bool part = pend && c == lc;
        const unsigned long long pm = __ballot(part);
        double pk[4], pp[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            pk[e] = part ? rk[e] : 0.0;
            pp[e] = part ? rp[e] : 0.0;
        }
        const double v = row_sum8_64(pk, pp, b1, b2);
        if ((lane & 8) == 0 && ((pm >> (lane & 48)) & 0xffffull) != 0ull) {
            const int li = (lc >> 16) + kdi, lj = (lc & 0xffff) + kdj;
            if (acc.tile) atomicAdd(&tile[kcomp * kTile64 + (li - ti0) * TJ + (lj - tj0)], v);
            else gadd(&kg[ix(p.ld, li, lj)], v);
        }
        pend = pend && !part;
    }
    if (cross) {
        // general zigzag in coordinates relative to the start cell
        Acc64 gacc = acc;
        if (di > 1 || di < -1 || dj > 1 || dj < -1) gacc.tile = nullptr;   // outside the patch
        double xr = fmin((di < 0 ? di : 0) + 1.0, fmax((double)(di > 0 ? di : 0), 0.5 * (x1 + x2)));
        double yr = fmin((dj < 0 ? dj : 0) + 1.0, fmax((double)(dj > 0 ? dj : 0), 0.5 * (y1 + y2)));
        double Q = p.Q;
        double fx1 = Q * (xr - x1), fy1 = Q * (yr - y1);
        double fx2 = Q * (x2 - xr), fy2 = Q * (y2 - yr);
        double wx1 = 0.5 * (x1 + xr), wy1 = 0.5 * (y1 + yr);
        double wx2 = 0.5 * (xr + x2) - di, wy2 = 0.5 * (yr + y2) - dj;
        gacc.add(0, i, j, fx1 * (1.0 - wy1));
        gacc.add(0, i, j + 1, fx1 * wy1);
        gacc.add(1, i, j, fy1 * (1.0 - wx1));
        gacc.add(1, i + 1, j, fy1 * wx1);
        gacc.add(0, i2, j2, fx2 * (1.0 - wy2));
        gacc.add(0, i2, j2 + 1, fx2 * wy2);
        gacc.add(1, i2, j2, fy2 * (1.0 - wx2));
        gacc.add(1, i2 + 1, j2, fy2 * wx2);
        double xm = 0.5 * (x1 + x2), ym = 0.5 * (y1 + y2);
        int im = (int)floor(xm), jm = (int)floor(ym);
        if (i + im > p.nr - 1) im = p.nr - 1 - i;
        if (j + jm > p.nth - 1) jm = p.nth - 1 - j;
        double wx = xm - im, wy = ym - jm;
        double qv = Q * v1;
        gacc.add(2, i + im, j + jm, qv * (1.0 - wx) * (1.0 - wy));
        gacc.add(2, i + im + 1, j + jm, qv * wx * (1.0 - wy));
        gacc.add(2, i + im, j + jm + 1, qv * (1.0 - wx) * wy);
        gacc.add(2, i + im + 1, j + jm + 1, qv * wx * wy);
    }
    count_wave(&removed[1], killed);
    count_wave(&removed[2], star);
    count_wave(&removed[3], absb);
    if (use_lds) {
        __syncthreads();
        for (int e = tid; e < TI * TJ; e += 256) {
            int ti = e / TJ, tj = e - ti * TJ;
            int gi = ti0 + ti, gj = tj0 + tj;
            if (gi < 0 || gi > p.nr || gj < 0 || gj > p.nth) continue;
            size_t gk = ix(p.ld, gi, gj);
            double w0 = tile[e], w1 = tile[kTile64 + e], w2 = tile[2 * kTile64 + e];
            if (w0 != 0.0) gadd(&Jr[gk], w0);
            if (w1 != 0.0) gadd(&Jt[gk], w1);
            if (w2 != 0.0) gadd(&Jp[gk], w2);
        }
    }
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
    p.rr = c->d.rr_coef * rr_factor(c) * fabs(qm) * fabs(qm) * fabs(qm);
    p.shell_r = c->d.shell_r;
    double **E = (double **)c->E, **B = (double **)c->B, **J = (double **)c->J;
    double **a = (double **)S.cur;
    int nb = (int)((S.nub + 255) / 256);
    hipLaunchKernelGGL(k_push64, dim3(nb), dim3(256), 0, c->stream, p, (int)S.nub,
                       c->nslots + s, c->kill, E[0], E[1], E[2], B[0], B[1], B[2], a[0], a[1],
                       a[2], a[3], a[4], J[0], J[1], J[2], c->removed + 4 * s, c->err);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
