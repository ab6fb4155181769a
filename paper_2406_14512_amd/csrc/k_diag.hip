// Species spectra over a region of the meridional plane (the observables of
// Sect. 5): the Lorentz-factor histogram, the leading power of the
// radiation-reaction force, P = K gamma^2 Bperp^2 (eq. bperp), and the
// synchrotron spectral energy distribution, each particle emitting the
// single-particle synchrotron spectrum normalised to its P:
//   nu dP/dnu = P x F(x) 9 sqrt(3) / (8 pi),  x = nu / nu_c,
//   nu_c = 3/(4 pi) gamma^2 omega_b |qm| Bperp,
// F(x) = x int_x^inf K_{5/3} the synchrotron function.
//
// One workgroup takes 1024 slots.  Each thread decodes its particles,
// bins gamma into an LDS histogram, gathers E and B at the particle (the
// interpolation of the FP64 push, in FP64 also for the FP32 fields) and
// leaves P and nu_c in LDS; then each thread takes one frequency and sums
// the block's particles for it (LDS broadcast reads, no atomics), and the
// block adds its partial sums to the output with one global atomic per bin.
//
// F comes from a table of ln F on a uniform grid in ln x over
// [1e-8, 100], built once on the host by quadrature of
//   F(x) = x int_0^inf exp(-x cosh t) cosh(5t/3) / cosh t dt
// (the representation K_nu(s) = int_0^inf exp(-s cosh t) cosh(nu t) dt
// integrated over s), and interpolated linearly in (ln x, ln F); below the
// table F follows its x^(1/3) law, above it F < 1e-40 is taken as 0.
#include <cmath>

#include "gather.h"

namespace ffpic {

namespace {

constexpr int kSpecWG = 256;
constexpr int kSpecPPT = 4;
constexpr int kSpecChunk = kSpecWG * kSpecPPT;
constexpr int kSyncN = 8192;
constexpr double kSyncX0 = 1e-8, kSyncX1 = 100.0;

struct SpecArgs {
    int nr, nth, ld, ngamma, nnu;
    double rmin, dlog, dth;
    const double *rn, *thn;
    double r0, r1, t0, t1;          // region
    double gmin, dlg;               // gamma bins
    const double *edge;             // ngamma + 1 edges
    const double *nu;               // nnu frequencies
    double w, K, wb;                // weight, radiation-reaction coefficient, omega_b |qm|
    const double *lnF;              // table of ln F
    double lx0, ihx;                // ln of its first abscissa, 1 / spacing
};

// x F(x) 9 sqrt(3) / (8 pi)
__device__ __forceinline__ double sync_kernel(const SpecArgs &A, double x) {
    const double lx = log(x);
    const double s = (lx - A.lx0) * A.ihx;
    double F;
    if (s < 0.0) {
        F = exp(A.lnF[0] + (lx - A.lx0) * (1.0 / 3.0));
    } else if (s >= (double)(kSyncN - 1)) {
        return 0.0;
    } else {
        const int k = (int)s;
        const double fr = s - (double)k;
        F = exp(A.lnF[k] + fr * (A.lnF[k + 1] - A.lnF[k]));
    }
    return x * F * (9.0 * 1.7320508075688772 / (8.0 * 3.14159265358979323846));
}

template <bool FP64, typename T>
__global__ void __launch_bounds__(kSpecWG)
    k_spectra(SpecArgs A, int nub, const int32_t *__restrict__ nslots, const void *s0,
              const void *s1, const void *s2, const void *s3, const void *s4, const void *s5,
              const T *__restrict__ Er, const T *__restrict__ Et, const T *__restrict__ Ep,
              const T *__restrict__ Br, const T *__restrict__ Bt, const T *__restrict__ Bp,
              double *__restrict__ out) {
    __shared__ double hist[FFPIC_SPEC_MAX];
    __shared__ double sP[kSpecChunk], sNu[kSpecChunk];
    __shared__ double wred[kSpecWG / 64];
    const int tid = threadIdx.x;
    const int n = min(nub, nslots[0]);
    const int base = blockIdx.x * kSpecChunk;
    for (int m = tid; m < A.ngamma; m += kSpecWG) hist[m] = 0.0;
    __syncthreads();
    double psum = 0.0;
    for (int k = 0; k < kSpecPPT; k++) {
        const int q = base + k * kSpecWG + tid;
        double P = 0.0, nuc = 0.0;
        bool in = false;
        int i = 0, j = 0;
        double a = 0.0, b = 0.0, r = 0.0, th = 0.0, u0 = 0.0, u1 = 0.0, u2 = 0.0;
        if (q < n) {
            if (FP64) {
                r = ((const double *)s0)[q];
                if (r > 0.0) {
                    th = ((const double *)s1)[q];
                    in = r >= A.r0 && r < A.r1 && th >= A.t0 && th < A.t1;
                    if (in) {
                        locate64(A.nr, A.nth, A.rmin, A.dlog, A.dth, A.rn, A.thn, r, th, i, j,
                                 a, b);
                        u0 = ((const double *)s2)[q];
                        u1 = ((const double *)s3)[q];
                        u2 = ((const double *)s4)[q];
                    }
                }
            } else {
                const int c = ((const int32_t *)s0)[q];
                if (c >= 0) {
                    i = c >> 16;
                    j = c & 0xffff;
                    a = (double)((const float *)s1)[q];
                    b = (double)((const float *)s2)[q];
                    r = A.rn[i] * exp(a * A.dlog);
                    th = A.thn[j] + b * A.dth;
                    in = r >= A.r0 && r < A.r1 && th >= A.t0 && th < A.t1;
                    if (in) {
                        u0 = (double)((const float *)s3)[q];
                        u1 = (double)((const float *)s4)[q];
                        u2 = (double)((const float *)s5)[q];
                    }
                }
            }
        }
        if (in) {
            const double g = sqrt(1.0 + u0 * u0 + u1 * u1 + u2 * u2);
            // log bin, settled against the edge table
            int m = (int)floor(log(g / A.gmin) / A.dlg);
            if (m < 0) m = 0;
            if (m > A.ngamma - 1) m = A.ngamma - 1;
            while (m > 0 && g < A.edge[m]) m--;
            while (m < A.ngamma - 1 && g >= A.edge[m + 1]) m++;
            if (g >= A.edge[m] && g < A.edge[m + 1]) atomicAdd(&hist[m], A.w);
            double E[3], B[3];
            gather_eb(Er, Et, Ep, Br, Bt, Bp, A.nr, A.nth, A.ld, i, j, a, b, E, B);
            const double be0 = u0 / g, be1 = u1 / g, be2 = u2 / g;
            const double F0 = E[0] + (be1 * B[2] - be2 * B[1]);
            const double F1 = E[1] + (be2 * B[0] - be0 * B[2]);
            const double F2 = E[2] + (be0 * B[1] - be1 * B[0]);
            const double be = be0 * E[0] + be1 * E[1] + be2 * E[2];
            double bp2 = F0 * F0 + F1 * F1 + F2 * F2 - be * be;
            if (bp2 < 0.0) bp2 = 0.0;
            P = A.K * g * g * bp2;
            nuc = 3.0 / (4.0 * 3.14159265358979323846) * g * g * A.wb * sqrt(bp2);
            psum += A.w * P;
        }
        sP[k * kSpecWG + tid] = P;
        sNu[k * kSpecWG + tid] = nuc;
    }
    __syncthreads();
    for (int f = tid; f < A.nnu; f += kSpecWG) {
        const double nu = A.nu[f];
        double acc = 0.0;
        for (int e = 0; e < kSpecChunk; e++) {
            const double P = sP[e], nuc = sNu[e];
            if (P > 0.0 && nuc > 0.0) acc += P * sync_kernel(A, nu / nuc);
        }
        if (acc != 0.0) gadd(&out[A.ngamma + f], A.w * acc);
    }
    for (int m = tid; m < A.ngamma; m += kSpecWG)
        if (hist[m] != 0.0) gadd(&out[m], hist[m]);
    for (int o = 32; o >= 1; o >>= 1) psum += __shfl_xor(psum, o, 64);
    if ((tid & 63) == 0) wred[tid >> 6] = psum;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kSpecWG / 64; w++) t += wred[w];
        if (t != 0.0) gadd(&out[A.ngamma + A.nnu], t);
    }
}

// F(x) = x int_0^inf exp(-x cosh t) cosh(5t/3) / cosh t dt, trapezoidal rule
// in t (geometric convergence for this even analytic integrand)
double synchrotron_F_host(double x) {
    const double h = 1.0 / 64.0;
    double sum = 0.0;
    for (int k = 0;; k++) {
        const double t = k * h;
        const double ch = std::cosh(t);
        if (x * ch > 745.0) break;
        sum += (k == 0 ? 0.5 : 1.0) * std::exp(-x * ch) * std::cosh(t * (5.0 / 3.0)) / ch;
    }
    return x * h * sum;
}

void *dev_alloc(size_t bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    return p;
}

}  // namespace

void spectra(ffpic_ctx *c, int s, const ffpic_spectra_req *rq, double *dev_out) {
#pragma clang fp contract(off)
    const int ng = rq->ngamma, nn = rq->nnu;
    if (!c->spec_tab) {
        std::vector<double> t(kSyncN);
        const double l0 = std::log(kSyncX0), l1 = std::log(kSyncX1);
        for (int k = 0; k < kSyncN; k++)
            t[k] = std::log(synchrotron_F_host(std::exp(l0 + (l1 - l0) * k / (kSyncN - 1))));
        c->spec_tab = (double *)dev_alloc(kSyncN * sizeof(double));
        c->spec_edge = (double *)dev_alloc((FFPIC_SPEC_MAX + 1) * sizeof(double));
        c->spec_nu = (double *)dev_alloc(FFPIC_SPEC_MAX * sizeof(double));
        if (hipMemcpy(c->spec_tab, t.data(), kSyncN * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess)
            throw std::runtime_error("upload of the synchrotron table failed");
    }
    // bin edges and frequencies in FP64 on the host
    std::vector<double> edge(ng + 1), nu(nn);
    const double dlg = std::log(rq->gmax / rq->gmin) / ng;
    for (int m = 0; m <= ng; m++) edge[m] = rq->gmin * std::exp(m * dlg);
    for (int m = 0; m < nn; m++)
        nu[m] = nn > 1 ? rq->numin * std::exp(m * std::log(rq->numax / rq->numin) / (nn - 1))
                       : rq->numin;
    if (hipMemcpyAsync(c->spec_edge, edge.data(), (ng + 1) * sizeof(double),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->spec_nu, nu.data(), nn * sizeof(double), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipMemsetAsync(dev_out, 0, (ng + nn + 1) * sizeof(double), c->stream) != hipSuccess)
        throw std::runtime_error("spectra set-up copy failed");
    // the host vectors must outlive the asynchronous copies
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        throw std::runtime_error("stream synchronisation failed");
    const ffpic::Species &S = c->sp[s];
    if (S.nub == 0) return;
    SpecArgs A{};
    A.nr = c->nr; A.nth = c->nth; A.ld = c->ld; A.ngamma = ng; A.nnu = nn;
    A.rmin = c->d.rmin; A.dlog = c->dlog; A.dth = c->dth;
    A.rn = c->dtab64[T_RN]; A.thn = c->dtab64[T_THN];
    A.r0 = rq->rmin; A.r1 = rq->rmax; A.t0 = rq->thmin; A.t1 = rq->thmax;
    A.gmin = rq->gmin; A.dlg = dlg; A.edge = c->spec_edge; A.nu = c->spec_nu;
    const double qm = S.qm;
    A.w = S.weight;
    A.K = c->d.rr_coef * rr_factor(c) * std::fabs(qm) * std::fabs(qm) * std::fabs(qm);
    A.wb = c->d.omega_b * std::fabs(qm);
    A.lnF = c->spec_tab;
    A.lx0 = std::log(kSyncX0);
    A.ihx = (kSyncN - 1) / (std::log(kSyncX1) - std::log(kSyncX0));
    const int nb = (int)((S.nub + kSpecChunk - 1) / kSpecChunk);
    void *const *a = S.cur;
    if (c->fp64) {
        double *const *E = (double *const *)c->E, *const *B = (double *const *)c->B;
        hipLaunchKernelGGL((k_spectra<true, double>), dim3(nb), dim3(kSpecWG), 0, c->stream, A,
                           (int)S.nub, c->nslots + s, a[0], a[1], a[2], a[3], a[4], a[4], E[0],
                           E[1], E[2], B[0], B[1], B[2], dev_out);
    } else {
        float *const *E = (float *const *)c->E, *const *B = (float *const *)c->B;
        hipLaunchKernelGGL((k_spectra<false, float>), dim3(nb), dim3(kSpecWG), 0, c->stream, A,
                           (int)S.nub, c->nslots + s, a[0], a[1], a[2], a[3], a[4], a[5], E[0],
                           E[1], E[2], B[0], B[1], B[2], dev_out);
    }
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
