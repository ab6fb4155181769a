// Flux function and mask kernels, and the force-free node correction,
// templated on the working precision R.  Included (through fields_fused.h)
// by k_fields64.hip (compiled without FP contraction, so the FP64 path
// rounds every product and sum as written) and by k_fields32.hip.
//
// Field arrays are node-shaped, theta fastest (see include/ffpic.h).
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
