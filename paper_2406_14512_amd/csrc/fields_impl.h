// Flux function, mask and field step kernels, templated on the working
// precision R.  Included by k_fields64.hip (compiled without FP
// contraction, so the FP64 path rounds every product and sum as written)
// and by k_fields32.hip.
//
// Field arrays are node-shaped, theta fastest (see include/ffpic.h).  One
// thread per (i, j) entry; blocks of 256 along theta, one grid row per i.
#pragma once

#include "device_common.h"

namespace ffpic {

// ---------------------------------------------------------------------------
// eq. (psi): Psi(i, 0) = 0, Psi(i, j+1) = Psi(i, j) + B_r(i, j+1/2) A_r(i, j)
// with A_r = r_i^2 (cos theta_j - cos theta_{j+1}); FP64, sequential in j so
// that the rounding is fixed.  A workgroup owns kPsiRows radial rows and
// walks them in tiles of kPsiCols columns: all 256 threads load a tile with
// coalesced reads along theta and form its terms B_r A_r in parallel (each
// product rounded as in the serial form) into LDS, then one lane per row
// runs the serial sum over the tile while the next tile's loads are in
// flight, and the tile of partial sums is written back coalesced.
constexpr int kPsiRows = 16;
constexpr int kPsiCols = 256;

// workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for the thread's global loads and stores, so the next
// tile's loads and the write-back stay in flight across it
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename R>
__global__ void __launch_bounds__(kPsiCols) k_psi(Geo<double> g, const R *__restrict__ br,
                                                  double *__restrict__ psi) {
    __shared__ double tile[kPsiRows][kPsiCols + 1];
    const int t = threadIdx.x;
    const int i0 = blockIdx.x * kPsiRows;
    const int ld = g.ld, nr = g.nr, nth = g.nth;
    const int rows = min(kPsiRows, nr + 1 - i0);
    double r2[kPsiRows];
#pragma unroll
    for (int rr = 0; rr < kPsiRows; rr++) r2[rr] = rr < rows ? g.rn2[i0 + rr] : 0.0;
    double acc = 0.0;
    if (t < rows) psi[ix(ld, i0 + t, 0)] = 0.0;
    // The tile's B_r and column areas are loaded one tile ahead.
    R nxt[kPsiRows];
    double arn;
    auto load = [&](int jt) {
        arn = jt + t < nth ? g.dcn[jt + t] : 0.0;
#pragma unroll
        for (int rr = 0; rr < kPsiRows; rr++)
            nxt[rr] = (rr < rows && jt + t < nth) ? br[ix(ld, i0 + rr, jt + t)] : (R)0;
    };
    // the tile's terms B_r A_r, each product rounded as in the serial form
    auto terms = [&]() {
#pragma unroll
        for (int rr = 0; rr < kPsiRows; rr++) {
#pragma clang fp contract(off)
            tile[rr][t] = (double)nxt[rr] * (r2[rr] * arn);
        }
    };
    load(0);
    terms();
    for (int j0 = 0; j0 < nth; j0 += kPsiCols) {
        const int w = min(kPsiCols, nth - j0);
        lds_barrier();
        const int jn = j0 + kPsiCols;
        if (jn < nth) load(jn);
        if (t < rows) {
#pragma unroll 16
            for (int k = 0; k < w; k++) {
#pragma clang fp contract(off)
                acc = acc + tile[t][k];
                tile[t][k] = acc;
            }
        }
        lds_barrier();
        // every lane stores every row: a lane past the last column or row
        // writes the last one instead (that entry's own value again), so
        // that with no branch around the stores the compiler can count those
        // still in flight, and the wait for the next tile's loads does not
        // also wait for this write-back
        const int tc = min(t, w - 1);
#pragma unroll
        for (int rr = 0; rr < kPsiRows; rr++) {
            const int rc = min(rr, rows - 1);
            psi[ix(ld, i0 + rc, j0 + 1 + tc)] = tile[rc][tc];
        }
        lds_barrier();
        if (jn < nth) terms();
    }
}

// blending function f at nodes (eq. transition, four thresholds) and the
// kill flag of each cell (all four corners at f = 1)
template <typename R>
__global__ void k_mask(int nr, int nth, int ld, int ff, double t0, double t1, double t2,
                       double t3, const double *__restrict__ psi, R *__restrict__ f,
                       uint8_t *__restrict__ kill) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (j > nth) return;
    double fv = ff ? blend(psi[ix(ld, i, j)], t0, t1, t2, t3) : 0.0;
    f[ix(ld, i, j)] = (R)fv;
    if (i < nr && j < nth) {
        bool k = false;
        if (ff && fv == 1.0)
            k = blend(psi[ix(ld, i + 1, j)], t0, t1, t2, t3) == 1.0 &&
                blend(psi[ix(ld, i, j + 1)], t0, t1, t2, t3) == 1.0 &&
                blend(psi[ix(ld, i + 1, j + 1)], t0, t1, t2, t3) == 1.0;
        kill[(size_t)i * nth + j] = k ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// eq. (faraday) in Stokes form on the primal faces: B -= h curl E
template <typename R>
__global__ void k_faraday(Geo<R> g, const R *__restrict__ er, const R *__restrict__ et,
                          const R *__restrict__ ep, R *__restrict__ br, R *__restrict__ bt,
                          R *__restrict__ bp, R h) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    size_t k = ix(ld, i, j);
    if (j < nth) {
        R circ = g.rn[i] * (g.sn[j + 1] * ep[k + 1] - g.sn[j] * ep[k]);
        br[k] -= h * circ / (g.rn2[i] * g.dcn[j]);
    }
    if (i < nr) {
        if (j > 0 && j < nth) {
            R circ = g.sn[j] * (g.rn[i + 1] * ep[k + ld] - g.rn[i] * ep[k]);
            bt[k] += h * circ / (g.sn[j] * g.dr2n[i]);
        } else {
            bt[k] = (R)0;
        }
        if (j < nth) {
            R circ = g.dth * (g.rn[i + 1] * et[k + ld] - g.rn[i] * et[k]) -
                     g.drn[i] * (er[k + 1] - er[k]);
            bp[k] -= h * circ / (g.dth * g.dr2n[i]);
        }
    }
}

// node collocation by arithmetic averages (Sect. 3): one-sided at the radial
// ends, parity across the axis
template <typename R>
__device__ __forceinline__ void node_e(const Geo<R> &g, const R *er, const R *et, const R *ep,
                                       int i, int j, R e[3]) {
    size_t k = ix(g.ld, i, j);
    e[0] = i == 0 ? er[k] : i == g.nr ? er[k - g.ld] : (R)0.5 * (er[k - g.ld] + er[k]);
    e[1] = (j == 0 || j == g.nth) ? (R)0 : (R)0.5 * (et[k - 1] + et[k]);
    e[2] = ep[k];
}

template <typename R>
__device__ __forceinline__ void node_b(const Geo<R> &g, const R *br, const R *bt, const R *bp,
                                       int i, int j, R b[3]) {
    const int ld = g.ld, nr = g.nr, nth = g.nth;
    size_t k = ix(ld, i, j);
    b[0] = j == 0 ? br[k] : j == nth ? br[k - 1] : (R)0.5 * (br[k - 1] + br[k]);
    b[1] = i == 0 ? bt[k] : i == nr ? bt[k - ld] : (R)0.5 * (bt[k - ld] + bt[k]);
    if (j == 0 || j == nth) {
        b[2] = (R)0;
    } else if (i == 0) {
        b[2] = (R)0.5 * (bp[k - 1] + bp[k]);
    } else if (i == nr) {
        b[2] = (R)0.5 * (bp[k - ld - 1] + bp[k - ld]);
    } else {
        b[2] = (R)0.25 * (bp[k - ld - 1] + bp[k - ld] + bp[k - 1] + bp[k]);
    }
}

// div E over the dual cell of node (i, j), 1 <= i <= nr - 1
template <typename R>
__device__ __forceinline__ R div_e(const Geo<R> &g, const R *er, const R *et, int i, int j) {
    size_t k = ix(g.ld, i, j);
    R flux = g.rh2[i] * g.dcd[j] * er[k] - g.rh2[i - 1] * g.dcd[j] * er[k - g.ld];
    if (j < g.nth) flux += g.sh[j] * g.dr2h[i] * et[k];
    if (j > 0) flux -= g.sh[j - 1] * g.dr2h[i] * et[k - 1];
    return flux / (g.dr3h[i] * g.dcd[j]);
}

// force-free current at nodes: the drift part of eq. (JFFE),
// J = rho (E x B) / B^2, rho = div E / 4 pi, with E^n and B^{n+1/2}
template <typename R>
__global__ void k_jffe(Geo<R> g, const R *__restrict__ er, const R *__restrict__ et,
                       const R *__restrict__ ep, const R *__restrict__ br,
                       const R *__restrict__ bt, const R *__restrict__ bp,
                       R *__restrict__ j0, R *__restrict__ j1, R *__restrict__ j2) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (j > g.nth) return;
    const R fourpi = (R)(4.0 * kPi);
    int ii = i == 0 ? 1 : i;
    R rho = i == g.nr ? (R)0 : div_e(g, er, et, ii, j) / fourpi;
    R e[3], b[3];
    node_e(g, er, et, ep, i, j, e);
    node_b(g, br, bt, bp, i, j, b);
    R b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    R x0 = e[1] * b[2] - e[2] * b[1];
    R x1 = e[2] * b[0] - e[0] * b[2];
    R x2 = e[0] * b[1] - e[1] * b[0];
    size_t k = ix(g.ld, i, j);
    bool ok = b2 > (R)0;
    j0[k] = ok ? rho * x0 / b2 : (R)0;
    j1[k] = ok ? rho * x1 / b2 : (R)0;
    j2[k] = ok ? rho * x2 / b2 : (R)0;
}

// eq. (ampere) on the dual faces with the blended current of eq. (blending)
template <typename R>
__global__ void k_ampere(Geo<R> g, R *__restrict__ er, R *__restrict__ et, R *__restrict__ ep,
                         const R *__restrict__ br, const R *__restrict__ bt,
                         const R *__restrict__ bp, R *__restrict__ jr_, R *__restrict__ jt_,
                         R *__restrict__ jp_, const R *__restrict__ f, const R *__restrict__ n0,
                         const R *__restrict__ n1, const R *__restrict__ n2, int ff) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    const R fourpi = (R)(4.0 * kPi);
    const R dt = g.dt;
    size_t k = ix(ld, i, j);
    // the deposit accumulators are consumed here and cleared for the next push
    const R jrk = jr_[k], jtk = jt_[k], jpk = jp_[k];
    jr_[k] = (R)0;
    jt_[k] = (R)0;
    jp_[k] = (R)0;
    if (i < nr) {
        R A = g.rh2[i] * g.dcd[j];
        R circ = (j < nth ? g.rh[i] * g.sh[j] * bp[k] : (R)0) -
                 (j > 0 ? g.rh[i] * g.sh[j - 1] * bp[k - 1] : (R)0);
        R J;
        if (ff) {
            R fs = (R)0.5 * (f[k] + f[k + ld]);
            J = ((R)1 - fs) * jrk / (dt * A) + fs * (R)0.5 * (n0[k] + n0[k + ld]);
        } else {
            J = jrk / (dt * A);
        }
        er[k] += dt * circ / A - fourpi * dt * J;
    }
    if (i >= 1 && i < nr) {
        if (j < nth) {
            R A = g.sh[j] * g.dr2h[i];
            R circ = -(g.rh[i] * g.sh[j] * bp[k] - g.rh[i - 1] * g.sh[j] * bp[k - ld]);
            R J;
            if (ff) {
                R fs = (R)0.5 * (f[k] + f[k + 1]);
                J = ((R)1 - fs) * jtk / (dt * A) + fs * (R)0.5 * (n1[k] + n1[k + 1]);
            } else {
                J = jtk / (dt * A);
            }
            et[k] += dt * circ / A - fourpi * dt * J;
        }
        if (j >= 1 && j < nth) {
            R A = g.dthd[j] * g.dr2h[i];
            R circ = g.dth * (g.rh[i] * bt[k] - g.rh[i - 1] * bt[k - ld]) -
                     g.drh[i] * (br[k] - br[k - 1]);
            R J;
            if (ff) {
                R fs = f[k];
                J = ((R)1 - fs) * jpk / (g.dr3h[i] * g.dcd[j]) + fs * n2[k];
            } else {
                J = jpk / (g.dr3h[i] * g.dcd[j]);
            }
            ep[k] += dt * circ / A - fourpi * dt * J;
        }
    }
}

// force-free correction at a node: E.B projection then the |E| <= |B| cap
// (Sect. 3); B = 0 gives E = 0
template <typename R>
__device__ __forceinline__ void ff_node(const R e[3], const R b[3], R o[3]) {
    R b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (!(b2 > (R)0)) {
        o[0] = o[1] = o[2] = (R)0;
        return;
    }
    R eb = e[0] * b[0] + e[1] * b[1] + e[2] * b[2];
    for (int c = 0; c < 3; c++) o[c] = e[c] - eb * b[c] / b2;
    R e2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    if (e2 >= b2 && e2 > (R)0) {
        R s = sqrt(b2 / e2);
        for (int c = 0; c < 3; c++) o[c] = s * o[c];
    }
}

// node corrections delta = f (E* - E) from E^{n+1} and B^{n+1/2}
template <typename R>
__global__ void k_ffdelta(Geo<R> g, const R *__restrict__ er, const R *__restrict__ et,
                          const R *__restrict__ ep, const R *__restrict__ br,
                          const R *__restrict__ bt, const R *__restrict__ bp,
                          const R *__restrict__ f, R *__restrict__ d0, R *__restrict__ d1,
                          R *__restrict__ d2) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (j > g.nth) return;
    size_t k = ix(g.ld, i, j);
    R fv = f[k];
    R o[3] = {(R)0, (R)0, (R)0};
    if (fv > (R)0) {
        R e[3], b[3], s[3];
        node_e(g, er, et, ep, i, j, e);
        node_b(g, br, bt, bp, i, j, b);
        ff_node(e, b, s);
        for (int c = 0; c < 3; c++) o[c] = fv * (s[c] - e[c]);
    }
    d0[k] = o[0];
    d1[k] = o[1];
    d2[k] = o[2];
}

// corrections averaged back onto the staggered E (boundary values kept)
template <typename R>
__global__ void k_ffapply(Geo<R> g, R *__restrict__ er, R *__restrict__ et, R *__restrict__ ep,
                          const R *__restrict__ d0, const R *__restrict__ d1,
                          const R *__restrict__ d2) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    size_t k = ix(ld, i, j);
    if (i < nr) er[k] += (R)0.5 * (d0[k] + d0[k + ld]);
    if (i >= 1 && i < nr) {
        if (j < nth) et[k] += (R)0.5 * (d1[k] + d1[k + 1]);
        if (j >= 1 && j < nth) ep[k] += d2[k];
    }
}

// absorbing layer beyond r_abs (damp E, relax B to its initial value) and
// zeroing of the deposit accumulators for the next step
// absorbing layer (rows from i0 on, where the damping factor is below 1):
// E is damped, B relaxes to its initial value
template <typename R>
__global__ void k_absorb(Geo<R> g, int i0, R *__restrict__ er, R *__restrict__ et,
                         R *__restrict__ ep, R *__restrict__ br, R *__restrict__ bt,
                         R *__restrict__ bp, const R *__restrict__ b0r, const R *__restrict__ b0t,
                         const R *__restrict__ b0p) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = i0 + blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    size_t k = ix(ld, i, j);
    R ln = g.lamn[i];
    R lh = i < nr ? g.lamh[i] : (R)1;
    if (ln == (R)1 && lh == (R)1) return;
    if (i < nr) {
        er[k] *= lh;
        bt[k] = b0t[k] + lh * (bt[k] - b0t[k]);
        if (j < nth) bp[k] = b0p[k] + lh * (bp[k] - b0p[k]);
    }
    ep[k] *= ln;
    if (j < nth) {
        et[k] *= ln;
        br[k] = b0r[k] + ln * (br[k] - b0r[k]);
    }
}

// ---------------------------------------------------------------------------
// launchers

template <typename R>
static void run_field_step(ffpic_ctx *c) {
    Geo<R> g = geo<R>(c);
    dim3 blk(256), grd((c->nth + 1 + 255) / 256, c->nr + 1);
    R **E = (R **)c->E, **B = (R **)c->B, **B0 = (R **)c->B0, **J = (R **)c->J;
    R **S = (R **)c->scr;
    R *f = (R *)c->f;
    int ff = c->d.ff_enable ? 1 : 0;
    R h = (R)(0.5 * c->dt);
    hipLaunchKernelGGL(k_faraday<R>, grd, blk, 0, c->stream, g, E[0], E[1], E[2], B[0], B[1],
                       B[2], h);
    if (ff)
        hipLaunchKernelGGL(k_jffe<R>, grd, blk, 0, c->stream, g, E[0], E[1], E[2], B[0], B[1],
                           B[2], S[0], S[1], S[2]);
    hipLaunchKernelGGL(k_ampere<R>, grd, blk, 0, c->stream, g, E[0], E[1], E[2], B[0], B[1],
                       B[2], J[0], J[1], J[2], f, S[0], S[1], S[2], ff);
    if (ff) {
        hipLaunchKernelGGL(k_ffdelta<R>, grd, blk, 0, c->stream, g, E[0], E[1], E[2], B[0],
                           B[1], B[2], f, S[3], S[4], S[5]);
        hipLaunchKernelGGL(k_ffapply<R>, grd, blk, 0, c->stream, g, E[0], E[1], E[2], S[3],
                           S[4], S[5]);
    }
    hipLaunchKernelGGL(k_faraday<R>, grd, blk, 0, c->stream, g, E[0], E[1], E[2], B[0], B[1],
                       B[2], h);
    if (c->absorb_row0 <= c->nr)
        hipLaunchKernelGGL(k_absorb<R>, dim3(grd.x, c->nr + 1 - c->absorb_row0), blk, 0,
                           c->stream, g, c->absorb_row0, E[0], E[1], E[2], B[0], B[1], B[2],
                           B0[0], B0[1], B0[2]);
    FFPIC_LAUNCH_CHECK();
}

template <typename R>
static void run_psi_mask(ffpic_ctx *c) {
    Geo<double> g = geo<double>(c);
    hipLaunchKernelGGL(k_psi<R>, dim3((c->nr + 1 + kPsiRows - 1) / kPsiRows), dim3(kPsiCols), 0,
                       c->stream, g, (const R *)c->B[0], c->psi);
    dim3 blk(256), grd((c->nth + 1 + 255) / 256, c->nr + 1);
    const double *t = c->d.psi_thr;
    hipLaunchKernelGGL(k_mask<R>, grd, blk, 0, c->stream, c->nr, c->nth, c->ld,
                       c->d.ff_enable ? 1 : 0, t[0], t[1], t[2], t[3], c->psi, (R *)c->f,
                       c->kill);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
