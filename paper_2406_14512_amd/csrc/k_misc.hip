// Particle load / export conversions, precision conversions and the FP64
// diagnostics (moments, Gauss-law residual, div B, Poynting flux, field
// energy).  Reductions are two-pass (per-block partials, then one block in
// a fixed order), so every diagnostic is deterministic.
#include "device_common.h"

namespace ffpic {

constexpr double kNear1f = 0.99999994039535522;   // largest float below 1

__device__ __forceinline__ bool valid_particle(double r, double th, double ur, double ut,
                                               double up, double rmin, double r_abs) {
    return isfinite(r) && isfinite(th) && isfinite(ur) && isfinite(ut) && isfinite(up) &&
           r >= rmin && r < r_abs && th >= 0.0 && th <= kPi;
}

__global__ void k_load64(int n, int off, double rmin, double r_abs, const double *r,
                         const double *th, const double *ur, const double *ut, const double *up,
                         double *R, double *TH, double *UR, double *UT, double *UP,
                         unsigned long long *removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (q < n) {
        bool ok = valid_particle(r[q], th[q], ur[q], ut[q], up[q], rmin, r_abs);
        R[off + q] = ok ? r[q] : -1.0;
        TH[off + q] = th[q];
        UR[off + q] = ur[q];
        UT[off + q] = ut[q];
        UP[off + q] = up[q];
        bad = !ok;
    }
    count_wave(&removed[0], bad);
}

__global__ void k_load32(int n, int off, int nr, int nth, double rmin, double r_abs, double dlog,
                         double dth, const double *rn, const double *thn, const double *r,
                         const double *th, const double *ur, const double *ut, const double *up,
                         int32_t *CELL, float *A, float *Bo, float *UR, float *UT, float *UP,
                         unsigned long long *removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (q < n) {
        bool ok = valid_particle(r[q], th[q], ur[q], ut[q], up[q], rmin, r_abs);
        int cell = -1;
        float af = 0.f, bf = 0.f;
        if (ok) {
            int i, j;
            double a, b;
            locate64(nr, nth, rmin, dlog, dth, rn, thn, r[q], th[q], i, j, a, b);
            af = (float)a;
            bf = (float)b;
            // an offset that rounds up to 1 moves to the next cell
            if (af >= 1.f) {
                if (i < nr - 1) { i++; af = 0.f; } else { af = (float)kNear1f; }
            }
            if (bf >= 1.f) {
                if (j < nth - 1) { j++; bf = 0.f; } else { bf = (float)kNear1f; }
            }
            cell = (i << 16) | j;
        }
        CELL[off + q] = cell;
        A[off + q] = af;
        Bo[off + q] = bf;
        UR[off + q] = (float)ur[q];
        UT[off + q] = (float)ut[q];
        UP[off + q] = (float)up[q];
        bad = !ok;
    }
    count_wave(&removed[0], bad);
}

void convert_loaded(ffpic_ctx *c, int s, int64_t off, int64_t n, const double *r,
                    const double *th, const double *ur, const double *uth, const double *uph) {
    ffpic::Species &S = c->sp[s];
    int nb = (int)((n + 255) / 256);
    if (c->fp64) {
        double **a = (double **)S.cur;
        hipLaunchKernelGGL(k_load64, dim3(nb), dim3(256), 0, c->stream, (int)n, (int)off,
                           c->d.rmin, c->d.r_abs, r, th, ur, uth, uph, a[0], a[1], a[2], a[3],
                           a[4], c->removed + 4 * s);
    } else {
        hipLaunchKernelGGL(k_load32, dim3(nb), dim3(256), 0, c->stream, (int)n, (int)off, c->nr,
                           c->nth, c->d.rmin, c->d.r_abs, c->dlog, c->dth, c->dtab64[T_RN],
                           c->dtab64[T_THN], r, th, ur, uth, uph, (int32_t *)S.cur[0],
                           (float *)S.cur[1], (float *)S.cur[2], (float *)S.cur[3],
                           (float *)S.cur[4], (float *)S.cur[5], c->removed + 4 * s);
    }
    FFPIC_LAUNCH_CHECK();
}

__global__ void k_export64(int n, int nr, int nth, double rmin, double dlog, double dth,
                           const double *rn, const double *thn, const double *R, const double *TH,
                           const double *UR, const double *UT, const double *UP, double *r,
                           double *th, double *ur, double *ut, double *up, int32_t *cell) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double rr = R[q];
    r[q] = rr; th[q] = TH[q]; ur[q] = UR[q]; ut[q] = UT[q]; up[q] = UP[q];
    int cc = -1;
    if (rr > 0.0) {
        int i, j;
        double a, b;
        locate64(nr, nth, rmin, dlog, dth, rn, thn, rr, TH[q], i, j, a, b);
        cc = i * nth + j;
    }
    cell[q] = cc;
}

__global__ void k_export32(int n, int nth, double dlog, double dth, const double *rn,
                           const double *thn, const int32_t *CELL, const float *A,
                           const float *Bo, const float *UR, const float *UT, const float *UP,
                           double *r, double *th, double *ur, double *ut, double *up,
                           int32_t *cell) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int c = CELL[q];
    if (c < 0) {
        r[q] = -1.0; th[q] = 0.0; cell[q] = -1;
    } else {
        int i = c >> 16, j = c & 0xffff;
        r[q] = rn[i] * exp((double)A[q] * dlog);
        th[q] = thn[j] + (double)Bo[q] * dth;
        cell[q] = i * nth + j;
    }
    ur[q] = UR[q]; ut[q] = UT[q]; up[q] = UP[q];
}

void export_particles(ffpic_ctx *c, int s, int64_t first, int64_t n, double *r, double *th,
                      double *ur, double *uth, double *uph, int32_t *cell) {
    ffpic::Species &S = c->sp[s];
    if (n == 0) return;
    int nb = (int)((n + 255) / 256);
    if (c->fp64) {
        const double *a[5];
        for (int k = 0; k < 5; k++) a[k] = (const double *)S.cur[k] + first;
        hipLaunchKernelGGL(k_export64, dim3(nb), dim3(256), 0, c->stream, (int)n, c->nr, c->nth,
                           c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN], c->dtab64[T_THN], a[0],
                           a[1], a[2], a[3], a[4], r, th, ur, uth, uph, cell);
    } else {
        hipLaunchKernelGGL(k_export32, dim3(nb), dim3(256), 0, c->stream, (int)n, c->nth,
                           c->dlog, c->dth, c->dtab64[T_RN], c->dtab64[T_THN],
                           (const int32_t *)S.cur[0] + first, (const float *)S.cur[1] + first,
                           (const float *)S.cur[2] + first, (const float *)S.cur[3] + first,
                           (const float *)S.cur[4] + first, (const float *)S.cur[5] + first, r,
                           th, ur, uth, uph, cell);
    }
    FFPIC_LAUNCH_CHECK();
}

template <typename R>
__global__ void k_to64(const R *src, double *dst, size_t n) {
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = (double)src[q];
}
template <typename R>
__global__ void k_from64(const double *src, R *dst, size_t n) {
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = (R)src[q];
}

void to_f64(ffpic_ctx *c, const void *src, double *dst, size_t n) {
    dim3 g((unsigned)((n + 255) / 256));
    if (c->fp64) hipLaunchKernelGGL(k_to64<double>, g, dim3(256), 0, c->stream, (const double *)src, dst, n);
    else hipLaunchKernelGGL(k_to64<float>, g, dim3(256), 0, c->stream, (const float *)src, dst, n);
    FFPIC_LAUNCH_CHECK();
}
void from_f64(ffpic_ctx *c, const double *src, void *dst, size_t n) {
    dim3 g((unsigned)((n + 255) / 256));
    if (c->fp64) hipLaunchKernelGGL(k_from64<double>, g, dim3(256), 0, c->stream, src, (double *)dst, n);
    else hipLaunchKernelGGL(k_from64<float>, g, dim3(256), 0, c->stream, src, (float *)dst, n);
    FFPIC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// deterministic block reductions

constexpr int kRedBlocks = 512;

template <int K>
__device__ void block_store(double v[K], double *part) {
    __shared__ double sm[K][256];
    for (int k = 0; k < K; k++) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < K; k++) sm[k][threadIdx.x] += sm[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < K; k++) part[(size_t)blockIdx.x * K + k] = sm[k][0];
}

template <int K>
__global__ void k_final(const double *part, int nblk, double *out) {
    __shared__ double sm[K][256];
    double v[K];
    for (int k = 0; k < K; k++) v[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int k = 0; k < K; k++) v[k] += part[(size_t)b * K + k];
    for (int k = 0; k < K; k++) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < K; k++) sm[k][threadIdx.x] += sm[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < K; k++) out[k] = sm[k][0];
}

template <bool F64>
__global__ void k_moments(int nub, const int32_t *nslots, const void *c0, const void *u0, const void *u1, const void *u2,
                          double *part) {
    double v[5] = {0, 0, 0, 0, 0};
    const int n = min(nub, nslots[0]);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        double ur, ut, up;
        bool live;
        if (F64) {
            live = ((const double *)c0)[q] > 0.0;
            ur = ((const double *)u0)[q]; ut = ((const double *)u1)[q]; up = ((const double *)u2)[q];
        } else {
            live = ((const int32_t *)c0)[q] >= 0;
            ur = ((const float *)u0)[q]; ut = ((const float *)u1)[q]; up = ((const float *)u2)[q];
        }
        if (!live) continue;
        v[0] += 1.0;
        v[1] += sqrt(1.0 + ur * ur + ut * ut + up * up);
        v[2] += ur; v[3] += ut; v[4] += up;
    }
    block_store<5>(v, part);
}

void moments(ffpic_ctx *c, int s, double *part, double *out5) {
    ffpic::Species &S = c->sp[s];
    int n = (int)S.nub;
    if (c->fp64)
        hipLaunchKernelGGL(k_moments<true>, dim3(kRedBlocks), dim3(256), 0, c->stream, n, c->nslots + s,
                           S.cur[0], S.cur[2], S.cur[3], S.cur[4], part);
    else
        hipLaunchKernelGGL(k_moments<false>, dim3(kRedBlocks), dim3(256), 0, c->stream, n, c->nslots + s,
                           S.cur[0], S.cur[3], S.cur[4], S.cur[5], part);
    hipLaunchKernelGGL(k_final<5>, dim3(1), dim3(256), 0, c->stream, part, kRedBlocks, out5);
    FFPIC_LAUNCH_CHECK();
}

__global__ void k_fill0(double *p, size_t n) {
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (size_t)gridDim.x * blockDim.x)
        p[q] = 0.0;
}

// node charge sum Q S_xi S_eta (FP64 atomics) into `q`
template <bool F64>
__global__ void k_charge(int n, const int32_t *nslots, int nr, int nth, int ld, double rmin, double dlog, double dth,
                         const double *rn, const double *thn, const void *c0, const void *c1,
                         const void *c2, double Q, double *qn) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n || q >= nslots[0]) return;
    int i, j;
    double a, b;
    if (F64) {
        double r = ((const double *)c0)[q];
        if (!(r > 0.0)) return;
        locate64(nr, nth, rmin, dlog, dth, rn, thn, r, ((const double *)c1)[q], i, j, a, b);
    } else {
        int cc = ((const int32_t *)c0)[q];
        if (cc < 0) return;
        i = cc >> 16; j = cc & 0xffff;
        a = ((const float *)c1)[q];
        b = ((const float *)c2)[q];
    }
    atomicAdd(&qn[ix(ld, i, j)], Q * (1.0 - a) * (1.0 - b));
    atomicAdd(&qn[ix(ld, i + 1, j)], Q * a * (1.0 - b));
    atomicAdd(&qn[ix(ld, i, j + 1)], Q * (1.0 - a) * b);
    atomicAdd(&qn[ix(ld, i + 1, j + 1)], Q * a * b);
}

// block maximum of |x| over the block's threads, written to part[blockIdx.x]
__device__ void block_max(double m, double *part) {
    __shared__ double sm[256];
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// FP64 value of a field entry: the FP64 array itself, or, in FP32-mixed
// mode, the FP64 background plus the FP32 perturbation
template <typename R>
__device__ __forceinline__ double fval(const R *x, const double *x0, size_t k) {
    return x0 ? x0[k] + (double)x[k] : (double)x[k];
}

// Gauss-law residual div E - 4 pi rho over the dual cell of each node
// (zero on the first and last rows), in FP64; written as a map (G) and/or
// folded into per-block maxima of |G| (part)
template <typename R>
__global__ void k_gauss(Geo<double> g, const R *er, const R *et, const double *e0r,
                        const double *e0t, const double *qn, double *G, double *part) {
    const size_t total = (size_t)(g.nr + 1) * g.ld;
    double m = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / g.ld), j = (int)(k % g.ld);
        double v = 0.0;
        if (i > 0 && i < g.nr) {
            double flux = g.rh2[i] * g.dcd[j] * fval(er, e0r, k) -
                          g.rh2[i - 1] * g.dcd[j] * fval(er, e0r, k - g.ld);
            if (j < g.nth) flux += g.sh[j] * g.dr2h[i] * fval(et, e0t, k);
            if (j > 0) flux -= g.sh[j - 1] * g.dr2h[i] * fval(et, e0t, k - 1);
            double vol = g.dr3h[i] * g.dcd[j];
            v = flux / vol - 4.0 * kPi * qn[k] / vol;
        }
        if (G) G[k] = v;
        m = fmax(m, fabs(v));
    }
    if (part) block_max(m, part);
}

void gauss(ffpic_ctx *c, double *qn, double *map, double *part) {
    hipLaunchKernelGGL(k_fill0, dim3(kRedBlocks), dim3(256), 0, c->stream, qn, c->nn);
    for (int s = 0; s < c->d.nspec; s++) {
        ffpic::Species &S = c->sp[s];
        if (S.nub == 0) continue;
        double Q = (S.qm > 0 ? 1.0 : -1.0) * S.weight;
        int nb = (int)((S.nub + 255) / 256);
        if (c->fp64)
            hipLaunchKernelGGL(k_charge<true>, dim3(nb), dim3(256), 0, c->stream, (int)S.nub, c->nslots + s, c->nr,
                               c->nth, c->ld, c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN],
                               c->dtab64[T_THN], S.cur[0], S.cur[1], S.cur[2], Q, qn);
        else
            hipLaunchKernelGGL(k_charge<false>, dim3(nb), dim3(256), 0, c->stream, (int)S.nub, c->nslots + s, c->nr,
                               c->nth, c->ld, c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN],
                               c->dtab64[T_THN], S.cur[0], S.cur[1], S.cur[2], Q, qn);
    }
    Geo<double> g = geo<double>(c);
    if (c->fp64)
        hipLaunchKernelGGL(k_gauss<double>, dim3(kRedBlocks), dim3(256), 0, c->stream, g,
                           (const double *)c->E[0], (const double *)c->E[1], nullptr, nullptr, qn,
                           map, part);
    else
        hipLaunchKernelGGL(k_gauss<float>, dim3(kRedBlocks), dim3(256), 0, c->stream, g,
                           (const float *)c->dE[0], (const float *)c->dE[1], c->E0d[0], c->E0d[1],
                           qn, map, part);
    FFPIC_LAUNCH_CHECK();
}

// div B over each primal cell (zero past the last row and column), in
// FP64 (FP32-mixed: FP64 background plus the perturbation)
template <typename R>
__global__ void k_divb(Geo<double> g, const R *br, const R *bt, const double *b0r,
                       const double *b0t, double *D, double *part) {
    const size_t total = (size_t)(g.nr + 1) * g.ld;
    double m = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / g.ld), j = (int)(k % g.ld);
        double v = 0.0;
        if (i < g.nr && j < g.nth) {
            double flux = g.rn2[i + 1] * g.dcn[j] * fval(br, b0r, k + g.ld) -
                          g.rn2[i] * g.dcn[j] * fval(br, b0r, k) +
                          g.sn[j + 1] * g.dr2n[i] * fval(bt, b0t, k + 1) -
                          g.sn[j] * g.dr2n[i] * fval(bt, b0t, k);
            v = flux / (g.dr3n[i] * g.dcn[j]);
        }
        if (D) D[k] = v;
        m = fmax(m, fabs(v));
    }
    if (part) block_max(m, part);
}

void divb(ffpic_ctx *c, double *map, double *part) {
    Geo<double> g = geo<double>(c);
    if (c->fp64)
        hipLaunchKernelGGL(k_divb<double>, dim3(kRedBlocks), dim3(256), 0, c->stream, g,
                           (const double *)c->B[0], (const double *)c->B[1], nullptr, nullptr, map,
                           part);
    else
        hipLaunchKernelGGL(k_divb<float>, dim3(kRedBlocks), dim3(256), 0, c->stream, g,
                           (const float *)c->dB[0], (const float *)c->dB[1], c->B0d[0], c->B0d[1],
                           map, part);
    FFPIC_LAUNCH_CHECK();
}

// Poynting flux through the sphere r_i: (c / 4 pi) 2 pi
// int (E_th B_ph - E_ph B_th) r^2 sin(theta) dtheta; one block per radius
template <typename R>
__global__ void k_poynting(Geo<double> g, const R *et, const R *ep, const R *bt, const R *bp,
                           double *L) {
    int i = blockIdx.x;
    __shared__ double sm[256];
    double acc = 0.0;
    if (i > 0 && i < g.nr) {
        for (int j = threadIdx.x; j <= g.nth; j += 256) {
            size_t k = ix(g.ld, i, j);
            if (j < g.nth) {
                double bph = 0.5 * ((double)bp[k - g.ld] + (double)bp[k]);
                acc += (double)et[k] * bph * g.dcn[j];
            }
            double bth = 0.5 * ((double)bt[k - g.ld] + (double)bt[k]);
            acc -= (double)ep[k] * bth * g.dcd[j];
        }
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) L[i] = (i > 0 && i < g.nr) ? 0.5 * g.rn2[i] * sm[0] : 0.0;
}

void poynting(ffpic_ctx *c, double *L) {
    Geo<double> g = geo<double>(c);
    if (c->fp64)
        hipLaunchKernelGGL(k_poynting<double>, dim3(c->nr + 1), dim3(256), 0, c->stream, g,
                           (const double *)c->E[1], (const double *)c->E[2],
                           (const double *)c->B[1], (const double *)c->B[2], L);
    else
        hipLaunchKernelGGL(k_poynting<float>, dim3(c->nr + 1), dim3(256), 0, c->stream, g,
                           (const float *)c->E[1], (const float *)c->E[2],
                           (const float *)c->B[1], (const float *)c->B[2], L);
    FFPIC_LAUNCH_CHECK();
}

// field energy: each staggered sample weighted by the volume of the cell it
// stands for (radial x polar extents of its primal or dual interval)
template <typename R>
__global__ void k_energy(Geo<double> g, const R *er, const R *et, const R *ep, const R *br,
                         const R *bt, const R *bp, double *part) {
    double v[2] = {0.0, 0.0};
    size_t total = (size_t)(g.nr + 1) * g.ld;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(k / g.ld), j = (int)(k % g.ld);
        double e = 0.0, b = 0.0, x;
        if (i < g.nr) { x = er[k]; e += x * x * g.dr3n[i] * g.dcd[j]; }
        if (j < g.nth) { x = et[k]; e += x * x * g.dr3h[i] * g.dcn[j]; }
        x = ep[k]; e += x * x * g.dr3h[i] * g.dcd[j];
        if (j < g.nth) { x = br[k]; b += x * x * g.dr3h[i] * g.dcn[j]; }
        if (i < g.nr) { x = bt[k]; b += x * x * g.dr3n[i] * g.dcd[j]; }
        if (i < g.nr && j < g.nth) { x = bp[k]; b += x * x * g.dr3n[i] * g.dcn[j]; }
        v[0] += e / (8.0 * kPi);
        v[1] += b / (8.0 * kPi);
    }
    block_store<2>(v, part);
}

void energies(ffpic_ctx *c, double *part, double *out2) {
    Geo<double> g = geo<double>(c);
    if (c->fp64)
        hipLaunchKernelGGL(k_energy<double>, dim3(kRedBlocks), dim3(256), 0, c->stream, g,
                           (const double *)c->E[0], (const double *)c->E[1], (const double *)c->E[2],
                           (const double *)c->B[0], (const double *)c->B[1], (const double *)c->B[2],
                           part);
    else
        hipLaunchKernelGGL(k_energy<float>, dim3(kRedBlocks), dim3(256), 0, c->stream, g,
                           (const float *)c->E[0], (const float *)c->E[1], (const float *)c->E[2],
                           (const float *)c->B[0], (const float *)c->B[1], (const float *)c->B[2],
                           part);
    hipLaunchKernelGGL(k_final<2>, dim3(1), dim3(256), 0, c->stream, part, kRedBlocks, out2);
    FFPIC_LAUNCH_CHECK();
}

int diag_partials() { return kRedBlocks; }

}  // namespace ffpic
