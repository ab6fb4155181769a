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
constexpr int kPsiRun = 32;     // terms a lane sums between LDS reads

// workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for the thread's global loads and stores, so the next
// tile's loads and the write-back stay in flight across it
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// the arguments of one system's flux function
template <typename R>
struct PsiJob {
    int nr, nth, ld;
    int blocks;                // workgroups of kPsiRows rows
    const double *rn2, *dcn;   // r_i^2, cos theta_j - cos theta_{j+1}
    const R *br;
    double *psi;
};

// rows [bx * kPsiRows, ...) of one system; every thread of the workgroup
// calls it and returns from it together
template <typename R>
__device__ __forceinline__ void psi_block(const PsiJob<R> &P, int bx,
                                          double (*tile)[kPsiCols + 1]) {
    const int t = threadIdx.x;
    const int i0 = bx * kPsiRows;
    const int ld = P.ld, nr = P.nr, nth = P.nth;
    const R *__restrict__ br = P.br;
    double *__restrict__ psi = P.psi;
    const int rows = min(kPsiRows, nr + 1 - i0);
    double r2[kPsiRows];
#pragma unroll
    for (int rr = 0; rr < kPsiRows; rr++) r2[rr] = rr < rows ? P.rn2[i0 + rr] : 0.0;
    double acc = 0.0;
    if (t < rows) psi[ix(ld, i0 + t, 0)] = 0.0;
    // The tile's B_r and column areas are loaded one tile ahead.
    R nxt[kPsiRows];
    double arn;
    auto load = [&](int jt) {
        arn = jt + t < nth ? P.dcn[jt + t] : 0.0;
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
            // in blocks of kPsiRun terms: all reads, then the serial sums in
            // registers, then all writes, so that the chain of additions
            // waits for LDS once per block rather than every few terms
            double *__restrict__ row = tile[t];
            int k = 0;
            for (; k + kPsiRun <= w; k += kPsiRun) {
                double v[kPsiRun];
#pragma unroll
                for (int u = 0; u < kPsiRun; u++) v[u] = row[k + u];
#pragma unroll
                for (int u = 0; u < kPsiRun; u++) {
#pragma clang fp contract(off)
                    acc = acc + v[u];
                    v[u] = acc;
                }
#pragma unroll
                for (int u = 0; u < kPsiRun; u++) row[k + u] = v[u];
            }
            for (; k < w; k++) {
#pragma clang fp contract(off)
                acc = acc + row[k];
                row[k] = acc;
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

template <typename R>
__global__ void __launch_bounds__(kPsiCols) k_psi(const PsiJob<R> P) {
    __shared__ double tile[kPsiRows][kPsiCols + 1];
    psi_block<R>(P, (int)blockIdx.x, tile);
}

// the arguments of one system's mask
template <typename R>
struct MaskJob {
    int nr, nth, ld, ff;
    int cblocks;               // workgroups of 256 columns per row
    double t0, t1, t2, t3;
    const double *psi;
    R *f;
    uint8_t *kill;
};

// blending function f at nodes (eq. transition, four thresholds) and the
// kill flag of each cell (all four corners at f = 1): columns from bx * 256
// of row i
template <typename R>
__device__ __forceinline__ void mask_row(const MaskJob<R> &M, int bx, int i) {
    const int j = bx * 256 + (int)threadIdx.x;
    const int nr = M.nr, nth = M.nth, ld = M.ld;
    if (j > nth) return;
    const double t0 = M.t0, t1 = M.t1, t2 = M.t2, t3 = M.t3;
    const double *__restrict__ psi = M.psi;
    // the node and its three neighbours towards the cell's far corner are
    // loaded together (the last row and column read their own node again):
    // behind a branch each, the compiler would wait for one after the other
    const bool cell = i < nr && j < nth;
    const int i1 = cell ? i + 1 : i, j1 = cell ? j + 1 : j;
    const double p00 = psi[ix(ld, i, j)], p10 = psi[ix(ld, i1, j)];
    const double p01 = psi[ix(ld, i, j1)], p11 = psi[ix(ld, i1, j1)];
    const double fv = M.ff ? blend(p00, t0, t1, t2, t3) : 0.0;
    M.f[ix(ld, i, j)] = (R)fv;
    if (cell) {
        const bool k = M.ff && fv == 1.0 && blend(p10, t0, t1, t2, t3) == 1.0 &&
                       blend(p01, t0, t1, t2, t3) == 1.0 && blend(p11, t0, t1, t2, t3) == 1.0;
        M.kill[(size_t)i * nth + j] = k ? 1 : 0;
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_mask(const MaskJob<R> M) {
    mask_row<R>(M, (int)blockIdx.x, (int)blockIdx.y);
}

// The flux functions of many systems in one launch of persistent
// workgroups taking row blocks from a counter (job k owns items
// [starts[k], starts[k + 1])), and their masks in a second launch whose
// workgroups stride over (system, row) items: a mask row is a few kB of
// streaming, too little to be worth a counter.
template <typename R>
__global__ void __launch_bounds__(kPsiCols) k_psi_group(const PsiJob<R> *__restrict__ jobs,
                                                        const int *__restrict__ starts,
                                                        int njobs, int *__restrict__ ctr) {
    __shared__ double tile[kPsiRows][kPsiCols + 1];
    __shared__ int next, job;
    __shared__ uint32_t stage[kJobWords];
    const int total = starts[njobs];
    if (threadIdx.x == 0) next = atomicAdd(&ctr[0], 1);
    __syncthreads();
    int item = __builtin_amdgcn_readfirstlane(next);
    while (item < total) {
        find_job(starts, njobs, item, &job);
        int nx = 0;                    // the next item, taken during this one
        if (threadIdx.x == 0) nx = atomicAdd(&ctr[0], 1);
        __syncthreads();
        const int lo = __builtin_amdgcn_readfirstlane(job);
        psi_block<R>(stage_uniform(jobs + lo, stage), item - starts[lo], tile);
        if (threadIdx.x == 0) next = nx;
        __syncthreads();
        item = __builtin_amdgcn_readfirstlane(next);
    }
    group_done(ctr);
}

template <typename R>
__global__ void __launch_bounds__(256) k_mask_group(const MaskJob<R> *__restrict__ jobs,
                                                    const int *__restrict__ starts, int njobs) {
    __shared__ int job;
    const int total = starts[njobs];
    for (int item = (int)blockIdx.x; item < total; item += (int)gridDim.x) {
        find_job(starts, njobs, item, &job);
        __syncthreads();
        const int lo = __builtin_amdgcn_readfirstlane(job);
        const MaskJob<R> &M = jobs[lo];
        const int i = item - starts[lo];
        for (int bx = 0; bx < M.cblocks; bx++) mask_row<R>(M, bx, i);
        __syncthreads();               // job is rewritten for the next item
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
PsiJob<R> psi_job(const ffpic_ctx *c) {
    PsiJob<R> P;
    P.nr = c->nr; P.nth = c->nth; P.ld = c->ld;
    P.blocks = (c->nr + 1 + kPsiRows - 1) / kPsiRows;
    P.rn2 = c->dtab64[T_RN2];
    P.dcn = c->dtab64[T_DCN];
    P.br = (const R *)c->B[0];
    P.psi = c->psi;
    return P;
}

template <typename R>
MaskJob<R> mask_job(const ffpic_ctx *c) {
    MaskJob<R> M;
    M.nr = c->nr; M.nth = c->nth; M.ld = c->ld;
    M.ff = c->d.ff_enable ? 1 : 0;
    M.cblocks = (c->nth + 1 + 255) / 256;
    const double *t = c->d.psi_thr;
    M.t0 = t[0]; M.t1 = t[1]; M.t2 = t[2]; M.t3 = t[3];
    M.psi = c->psi;
    M.f = (R *)c->f;
    M.kill = c->kill;
    return M;
}

template <typename R>
static void run_psi_mask(ffpic_ctx *c) {
    const PsiJob<R> P = psi_job<R>(c);
    hipLaunchKernelGGL(k_psi<R>, dim3(P.blocks), dim3(kPsiCols), 0, c->stream, P);
    const MaskJob<R> M = mask_job<R>(c);
    hipLaunchKernelGGL(k_mask<R>, dim3(M.cblocks, c->nr + 1), dim3(256), 0, c->stream, M);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
