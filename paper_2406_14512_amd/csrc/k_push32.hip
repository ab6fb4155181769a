// FP32-mixed particle push and charge-conserving deposit.
//
// Particle state (SoA, 24 B): cell = (i << 16) | j (int32, -1 = dead slot),
// a = in-cell offset in log r / dlog, b = in-cell offset in theta / dtheta
// (FP32, in [0, 1)), u_r, u_theta, u_phi (FP32).  Splitting the position
// into an integer cell and a small FP32 offset keeps 2^-24 of a cell of
// resolution anywhere on the grid, where an absolute FP32 coordinate would
// lose several digits at r ~ 100.
//
// Physics as in the FP64 path (Sect. 3, eq. motion with the
// radiation-reaction force g and eq. bperp; Boris rotation; zigzag
// charge-conserving deposit), but the move is evaluated in the particle's
// local frame: the radial and polar displacements are formed from the
// small step itself (log1p for the radial one, the arctangent of a small
// ratio for the polar one), so that no difference of two large FP32
// coordinates is ever taken.
//
// Deposit: each workgroup takes a contiguous chunk of the (cell-sorted)
// particle array, holds the chunk's state in registers, finds the bounding
// box of its cells and accumulates the currents in an LDS patch covering the
// box (plus the one-cell reach of a step); the patch is then flushed to the
// FP32 current arrays in HBM with one global atomic per touched entry.
// Within a wavefront, particles that stay in their cell and share it with
// the wave's leader are summed across lanes first (cross-lane reduction), so
// a sorted wave issues 8 LDS adds instead of 8 x 64.  Chunks whose box is
// too large for the patch (sparse regions) add straight to HBM.
#include "device_common.h"

namespace ffpic {

constexpr int kWG = 256;
constexpr int kPPT = 4;                  // particles per thread per chunk
constexpr int kChunk = kWG * kPPT;
constexpr int kTile = 2048;              // LDS patch entries per component

struct P32 {
    int nr, nth, ld;
    float dlog, dth, dt, inv_dlog, inv_dth;
    int iabs;                            // r_abs lies in radial cell iabs ...
    float aabs;                          // ... at offset aabs
    const float *rn, *sn, *cn;
    float Q, wq, rr;
};

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct Acc {
    float *lds;      // nullptr: global mode
    int ti0, tj0, TI, TJ;
    float *gr, *gt, *gp;
    int ld;
    __device__ __forceinline__ void add(int comp, int i, int j, float v) {
        if (lds) {
            int ti = i - ti0, tj = j - tj0;
            if (ti >= 0 && ti < TI && tj >= 0 && tj < TJ) {
                atomicAdd(&lds[comp * kTile + ti * TJ + tj], v);
                return;
            }
        }
        {
            float *g = comp == 0 ? gr : comp == 1 ? gt : gp;
            gadd(&g[ix(ld, i, j)], v);
        }
    }
};

// staggered bilinear gather (logical coordinates, axis parity ghosts,
// constant beyond the radial ends)
__device__ __forceinline__ float bil32(const float *__restrict__ F, int ld, int nth, int ilo,
                                       float wr, int jlo, float wt, bool thalf, float par) {
    int j0 = jlo, j1 = jlo + 1;
    float s0 = 1.f, s1 = 1.f;
    if (thalf) {
        if (j0 < 0) { j0 = 0; s0 = par; }
        if (j1 >= nth) { j1 = nth - 1; s1 = par; }
    }
    size_t r0 = (size_t)ilo * ld, r1 = r0 + ld;
    float v00 = s0 * F[r0 + j0], v01 = s1 * F[r0 + j1];
    float v10 = s0 * F[r1 + j0], v11 = s1 * F[r1 + j1];
    float lo = v00 + wt * (v01 - v00);
    float hi = v10 + wt * (v11 - v10);
    return lo + wr * (hi - lo);
}

__global__ void __launch_bounds__(kWG) k_push32(
    P32 p, int nub, const int32_t *__restrict__ nslots, const uint8_t *__restrict__ kill,
    const float *__restrict__ Er, const float *__restrict__ Et, const float *__restrict__ Ep,
    const float *__restrict__ Br, const float *__restrict__ Bt, const float *__restrict__ Bp,
    int32_t *__restrict__ CELL, float *__restrict__ A, float *__restrict__ Bo,
    float *__restrict__ UR, float *__restrict__ UT, float *__restrict__ UP,
    float *__restrict__ Jr, float *__restrict__ Jt, float *__restrict__ Jp,
    unsigned long long *__restrict__ removed, uint32_t *__restrict__ err) {
    __shared__ float tile[3 * kTile];
    __shared__ int box[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int n = min(nub, nslots[0]);
    const int base = blockIdx.x * kChunk;

    int cell[kPPT];
    int imin = 1 << 30, imax = -1, jmin = 1 << 30, jmax = -1;
#pragma unroll
    for (int k = 0; k < kPPT; k++) {
        int q = base + k * kWG + tid;
        cell[k] = q < n ? CELL[q] : -1;
        if (cell[k] >= 0) {
            int i = cell[k] >> 16, j = cell[k] & 0xffff;
            if (kill[(size_t)i * p.nth + j]) continue;
            imin = min(imin, i); imax = max(imax, i);
            jmin = min(jmin, j); jmax = max(jmax, j);
        }
    }
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
    Acc acc;
    acc.gr = Jr; acc.gt = Jt; acc.gp = Jp; acc.ld = p.ld;
    acc.ti0 = box[0] - 1;
    acc.tj0 = box[2] - 1;
    acc.TI = box[1] - box[0] + 4;
    acc.TJ = box[3] - box[2] + 4;
    const bool any = box[1] >= 0;
    const bool use_lds = any && acc.TI * acc.TJ <= kTile;
    acc.lds = use_lds ? tile : nullptr;
    if (use_lds) {
        int m = acc.TI * acc.TJ;
        for (int e = tid; e < m; e += kWG) {
            tile[e] = 0.f; tile[kTile + e] = 0.f; tile[2 * kTile + e] = 0.f;
        }
    }
    __syncthreads();

    int nkill = 0, nstar = 0, nabs = 0;
    if (any) {
#pragma unroll 1
        for (int k = 0; k < kPPT; k++) {
            int q = base + k * kWG + tid;
            int c = cell[k];
            bool live = c >= 0;
            int i = c >> 16, j = c & 0xffff;
            if (live && kill[(size_t)i * p.nth + j]) {
                live = false;
                CELL[q] = -1;
                nkill++;
            }
            // contributions of this particle
            bool simple = false;     // stays in its cell: 8 adds at fixed offsets
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f, s6 = 0.f, s7 = 0.f;
            int i2 = i, j2 = j;
            float x1 = 0.f, y1 = 0.f, x2 = 0.f, y2 = 0.f, qv = 0.f;
            bool dep = false;
            if (live) {
                float a = A[q], b = Bo[q];
                float ur = UR[q], ut = UT[q], up = UP[q];
                // gather
                int hr = a >= 0.5f ? i : i - 1;
                float whr = a >= 0.5f ? a - 0.5f : a + 0.5f;
                if (hr < 0) { hr = 0; whr = 0.f; }
                if (hr > p.nr - 2) { hr = p.nr - 2; whr = 1.f; }
                int ht = b >= 0.5f ? j : j - 1;
                float wht = b >= 0.5f ? b - 0.5f : b + 0.5f;
                const int ld = p.ld, nth = p.nth;
                float esr = bil32(Er, ld, nth, hr, whr, j, b, false, 1.f);
                float est = bil32(Et, ld, nth, i, a, ht, wht, true, -1.f);
                float esp = bil32(Ep, ld, nth, i, a, j, b, false, 1.f);
                float bsr = bil32(Br, ld, nth, i, a, ht, wht, true, 1.f);
                float bst = bil32(Bt, ld, nth, hr, whr, j, b, false, 1.f);
                float bsp = bil32(Bp, ld, nth, hr, whr, ht, wht, true, -1.f);
                // theta = theta_j + d, small-angle sine/cosine of d
                float d = b * p.dth, d2 = d * d;
                float sd = d * (1.f - d2 * (1.f / 6.f) * (1.f - d2 * (1.f / 20.f)));
                float cd = 1.f - 0.5f * d2 * (1.f - d2 * (1.f / 12.f));
                float snj = p.sn[j], cnj = p.cn[j];
                float st = snj * cd + cnj * sd;
                float ct = cnj * cd - snj * sd;
                // r = r_i exp(a dlog)
                float xl = a * p.dlog;
                float r = p.rn[i] * (1.f + xl * (1.f + xl * (0.5f + xl * (1.f / 6.f + xl * (1.f / 24.f)))));
                // local Cartesian frame at azimuth 0
                float Ex = esr * st + est * ct, Ey = esp, Ez = esr * ct - est * st;
                float Bx = bsr * st + bst * ct, By = bsp, Bz = bsr * ct - bst * st;
                float ux = ur * st + ut * ct, uy = up, uz = ur * ct - ut * st;
                // Boris rotation
                float h = 0.5f * p.dt * p.wq;
                float mx = ux + h * Ex, my = uy + h * Ey, mz = uz + h * Ez;
                float gm = sqrtf(1.f + mx * mx + my * my + mz * mz);
                float ig = h / gm;
                float tx = Bx * ig, ty = By * ig, tz = Bz * ig;
                float sf = 2.f / (1.f + tx * tx + ty * ty + tz * tz);
                float px = mx + (my * tz - mz * ty);
                float py = my + (mz * tx - mx * tz);
                float pz = mz + (mx * ty - my * tx);
                float sx = tx * sf, sy = ty * sf, sz = tz * sf;
                float nx = mx + (py * sz - pz * sy) + h * Ex;
                float ny = my + (pz * sx - px * sz) + h * Ey;
                float nz = mz + (px * sy - py * sx) + h * Ez;
                // radiation reaction (explicit, time-centred velocity)
                if (p.rr != 0.f) {
                    float bx = 0.5f * (ux + nx), by = 0.5f * (uy + ny), bz = 0.5f * (uz + nz);
                    float gb = sqrtf(1.f + bx * bx + by * by + bz * bz);
                    float igb = 1.f / gb;
                    bx *= igb; by *= igb; bz *= igb;
                    float Fx = Ex + (by * Bz - bz * By);
                    float Fy = Ey + (bz * Bx - bx * Bz);
                    float Fz = Ez + (bx * By - by * Bx);
                    float be = bx * Ex + by * Ey + bz * Ez;
                    float bp2 = fmaxf(Fx * Fx + Fy * Fy + Fz * Fz - be * be, 0.f);
                    float gg = gb * gb * bp2;
                    float kk = p.dt * p.rr;
                    nx += kk * ((Fy * Bz - Fz * By) + be * Ex - gg * bx);
                    ny += kk * ((Fz * Bx - Fx * Bz) + be * Ey - gg * by);
                    nz += kk * ((Fx * By - Fy * Bx) + be * Ez - gg * bz);
                }
                float g = sqrtf(1.f + nx * nx + ny * ny + nz * nz);
                if (!isfinite(g)) atomicOr(err, FFPIC_ERR_NONFINITE);
                float ivg = p.dt / g;
                float dx = nx * ivg, dy = ny * ivg, dz = nz * ivg;
                // move in the local frame
                float w = r * st;
                float xx = w + dx;
                float w2 = sqrtf(xx * xx + dy * dy);
                float den = w2 + w;
                float dw = den > 0.f ? (2.f * w * dx + dx * dx + dy * dy) / den : 0.f;
                float drr = dw * st + dz * ct;
                float dtt = dw * ct - dz * st;
                float ir = 1.f / r;
                float yv = drr * ir;
                float zv = dtt * ir;
                float arg = 2.f * yv + yv * yv + zv * zv;
                float dxi = 0.5f * log1pf(arg) * p.inv_dlog;
                float tq = dtt / (r + drr);
                float tq2 = tq * tq;
                float dth = tq * (1.f - tq2 * (1.f / 3.f - tq2 * (1.f / 5.f)));
                float cp = w2 > 0.f ? xx / w2 : 1.f;
                float sp = w2 > 0.f ? dy / w2 : 0.f;
                float rx = cp * nx + sp * ny, ry = -sp * nx + cp * ny, rz = nz;
                float dd2 = dth * dth;
                float sdd = dth * (1.f - dd2 * (1.f / 6.f));
                float cdd = 1.f - 0.5f * dd2;
                float st2 = st * cdd + ct * sdd, ct2 = ct * cdd - st * sdd;
                // new cell and offsets (carry)
                float na = a + dxi, nb = b + dth * p.inv_dth;
                int di = (int)floorf(na), dj = (int)floorf(nb);
                na -= (float)di;
                nb -= (float)dj;
                if (na >= 1.f) { na -= 1.f; di++; }
                if (nb >= 1.f) { nb -= 1.f; dj++; }
                i2 = i + di;
                j2 = j + dj;
                if (j2 < 0) { j2 = 0; nb = 0.f; dj = -j; }
                if (j2 > p.nth - 1) { j2 = p.nth - 1; nb = 0.99999994f; dj = j2 - j; }
                bool cfl = di > 1 || di < -1 || dj > 1 || dj < -1;
                if (cfl) atomicOr(err, FFPIC_ERR_CFL);
                bool finite = isfinite(g) && isfinite(na) && isfinite(nb) && isfinite(rx) &&
                              isfinite(ry) && isfinite(rz);
                if (!finite) {
                    // flagged in the error word; never deposited
                    atomicOr(err, FFPIC_ERR_NONFINITE);
                    CELL[q] = -1;
                } else if (i2 < 0) {
                    CELL[q] = -1;
                    nstar++;
                } else if (i2 > p.iabs || (i2 == p.iabs && na >= p.aabs)) {
                    CELL[q] = -1;
                    nabs++;
                } else {
                    CELL[q] = (i2 << 16) | j2;
                    A[q] = na;
                    Bo[q] = nb;
                    UR[q] = rx * st2 + rz * ct2;
                    UT[q] = rx * ct2 - rz * st2;
                    UP[q] = ry;
                    dep = !cfl;
                    x1 = a; y1 = b;
                    x2 = (float)di + na;
                    y2 = (float)dj + nb;
                    qv = ny * (1.f / g);
                    if (dep && di == 0 && dj == 0) {
                        simple = true;
                        float ddx = x2 - x1, ddy = y2 - y1;
                        float xm = 0.5f * (x1 + x2), ym = 0.5f * (y1 + y2);
                        s0 = ddx * (1.f - ym);
                        s1 = ddx * ym;
                        s2 = ddy * (1.f - xm);
                        s3 = ddy * xm;
                        s4 = qv * (1.f - xm) * (1.f - ym);
                        s5 = qv * xm * (1.f - ym);
                        s6 = qv * (1.f - xm) * ym;
                        s7 = qv * xm * ym;
                    }
                }
            }
            // cross-lane pre-reduction of same-cell, in-cell moves
            bool pend = simple;
#pragma unroll 1
            for (int it = 0; it < 2; it++) {
                unsigned long long m = __ballot(pend);
                if (m == 0ull) break;
                int leader = __ffsll((long long)m) - 1;
                int lc = __shfl(c, leader, 64);
                bool part = pend && c == lc;
                float v0 = wave_sum(part ? s0 : 0.f);
                float v1 = wave_sum(part ? s1 : 0.f);
                float v2 = wave_sum(part ? s2 : 0.f);
                float v3 = wave_sum(part ? s3 : 0.f);
                float v4 = wave_sum(part ? s4 : 0.f);
                float v5 = wave_sum(part ? s5 : 0.f);
                float v6 = wave_sum(part ? s6 : 0.f);
                float v7 = wave_sum(part ? s7 : 0.f);
                if (lane == leader) {
                    int li = lc >> 16, lj = lc & 0xffff;
                    float Q = p.Q;
                    acc.add(0, li, lj, Q * v0);
                    acc.add(0, li, lj + 1, Q * v1);
                    acc.add(1, li, lj, Q * v2);
                    acc.add(1, li + 1, lj, Q * v3);
                    acc.add(2, li, lj, Q * v4);
                    acc.add(2, li + 1, lj, Q * v5);
                    acc.add(2, li, lj + 1, Q * v6);
                    acc.add(2, li + 1, lj + 1, Q * v7);
                }
                pend = pend && !part;
            }
            if (pend) {
                float Q = p.Q;
                acc.add(0, i, j, Q * s0);
                acc.add(0, i, j + 1, Q * s1);
                acc.add(1, i, j, Q * s2);
                acc.add(1, i + 1, j, Q * s3);
                acc.add(2, i, j, Q * s4);
                acc.add(2, i + 1, j, Q * s5);
                acc.add(2, i, j + 1, Q * s6);
                acc.add(2, i + 1, j + 1, Q * s7);
            }
            if (dep && !simple) {
                // general zigzag (the particle leaves its cell)
                int di = i2 - i, dj = j2 - j;
                float xr = fminf((float)min(di, 0) + 1.f, fmaxf((float)max(di, 0), 0.5f * (x1 + x2)));
                float yr = fminf((float)min(dj, 0) + 1.f, fmaxf((float)max(dj, 0), 0.5f * (y1 + y2)));
                float Q = p.Q;
                float fx1 = Q * (xr - x1), fy1 = Q * (yr - y1);
                float fx2 = Q * (x2 - xr), fy2 = Q * (y2 - yr);
                float wx1 = 0.5f * (x1 + xr), wy1 = 0.5f * (y1 + yr);
                float wx2 = 0.5f * (xr + x2) - (float)di, wy2 = 0.5f * (yr + y2) - (float)dj;
                acc.add(0, i, j, fx1 * (1.f - wy1));
                acc.add(0, i, j + 1, fx1 * wy1);
                acc.add(1, i, j, fy1 * (1.f - wx1));
                acc.add(1, i + 1, j, fy1 * wx1);
                acc.add(0, i2, j2, fx2 * (1.f - wy2));
                acc.add(0, i2, j2 + 1, fx2 * wy2);
                acc.add(1, i2, j2, fy2 * (1.f - wx2));
                acc.add(1, i2 + 1, j2, fy2 * wx2);
                float xm = 0.5f * (x1 + x2), ym = 0.5f * (y1 + y2);
                int im = (int)floorf(xm), jm = (int)floorf(ym);
                if (i + im > p.nr - 1) im = p.nr - 1 - i;
                if (j + jm > p.nth - 1) jm = p.nth - 1 - j;
                float wx = xm - (float)im, wy = ym - (float)jm;
                float qq = Q * qv;
                acc.add(2, i + im, j + jm, qq * (1.f - wx) * (1.f - wy));
                acc.add(2, i + im + 1, j + jm, qq * wx * (1.f - wy));
                acc.add(2, i + im, j + jm + 1, qq * (1.f - wx) * wy);
                acc.add(2, i + im + 1, j + jm + 1, qq * wx * wy);
            }
        }
    }
    {
        int tk = nkill, ts = nstar, ta = nabs;
        for (int o = 32; o >= 1; o >>= 1) {
            tk += __shfl_xor(tk, o, 64);
            ts += __shfl_xor(ts, o, 64);
            ta += __shfl_xor(ta, o, 64);
        }
        if (lane == 0) {
            if (tk) atomicAdd(&removed[1], (unsigned long long)tk);
            if (ts) atomicAdd(&removed[2], (unsigned long long)ts);
            if (ta) atomicAdd(&removed[3], (unsigned long long)ta);
        }
    }
    if (use_lds) {
        __syncthreads();
        int m = acc.TI * acc.TJ;
        for (int e = tid; e < m; e += kWG) {
            int ti = e / acc.TJ, tj = e - ti * acc.TJ;
            int gi = acc.ti0 + ti, gj = acc.tj0 + tj;
            if (gi < 0 || gi > p.nr || gj < 0 || gj > p.nth) continue;
            size_t g = ix(p.ld, gi, gj);
            float v0 = tile[e], v1 = tile[kTile + e], v2 = tile[2 * kTile + e];
            if (v0 != 0.f) gadd(&Jr[g], v0);
            if (v1 != 0.f) gadd(&Jt[g], v1);
            if (v2 != 0.f) gadd(&Jp[g], v2);
        }
    }
}

void push32(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    if (S.nub == 0) return;
    P32 p;
    p.nr = c->nr; p.nth = c->nth; p.ld = c->ld;
    p.dlog = (float)c->dlog; p.dth = (float)c->dth; p.dt = (float)c->dt;
    p.inv_dlog = (float)(1.0 / c->dlog);
    p.inv_dth = (float)(1.0 / c->dth);
    double xa = log(c->d.r_abs / c->d.rmin) / c->dlog;
    p.iabs = (int)floor(xa);
    p.aabs = (float)(xa - floor(xa));
    p.rn = (const float *)c->dtab[T_RN];
    p.sn = (const float *)c->dtab[T_SN];
    p.cn = (const float *)c->dtab[T_CN];
    double qm = S.qm;
    p.Q = (float)((qm > 0 ? 1.0 : -1.0) * S.weight);
    p.wq = (float)(c->d.omega_b * qm);
    p.rr = (float)(c->d.rr_coef * fabs(qm) * fabs(qm) * fabs(qm));
    float **E = (float **)c->E, **B = (float **)c->B, **J = (float **)c->J;
    int nb = (int)((S.nub + kChunk - 1) / kChunk);
    hipLaunchKernelGGL(k_push32, dim3(nb), dim3(kWG), 0, c->stream, p, (int)S.nub,
                       c->nslots + s, c->kill, E[0], E[1], E[2], B[0], B[1], B[2],
                       (int32_t *)S.cur[0], (float *)S.cur[1], (float *)S.cur[2],
                       (float *)S.cur[3], (float *)S.cur[4], (float *)S.cur[5], J[0], J[1], J[2],
                       c->removed + 4 * s, c->err);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
