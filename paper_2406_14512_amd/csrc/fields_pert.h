// FP32 field step in perturbation form.
//
// In FP32 the static magnetosphere itself is the problem: the corotation E
// and the dipole B are discretely curl-free (or nearly so) in exact
// arithmetic, but once each component is rounded to FP32 their discrete
// curls are O(1e-7 |F| / cell) noise, which the Yee update integrates into
// B_phi and E_phi every step.  So the FP32 state is kept as a perturbation
// dF = F - F0 about an FP64 background F0 (the initial fields), whose
// discrete curls (the background rates) and charge density are evaluated
// once in FP64 on the host:
//   dB <- dB - h curl(dE) + h rateB0        (rateB0 = -curl E0)
//   dE <- dE + dt (curl(dB) + rateE0) - 4 pi dt J
//   rho = div(dE) / 4 pi + rho0
// Rounding then acts on the small perturbation, not on the background.  The
// totals F = F0 + dF are rewritten after every update for the particle
// gather and the force-free correction, which use totals.
#pragma once

#include "fields_impl.h"

namespace ffpic {

// force-free correction at a node in FP32 (Sect. 3: E.B projection, then
// |E| <= |B|), with the hardware reciprocal and square roots (about 1 ulp)
// in place of the divisions; B = 0 gives E = 0
__device__ __forceinline__ void ff_node_f(const float e[3], const float b[3], float o[3]) {
    const float b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (!(b2 > 0.f)) { o[0] = o[1] = o[2] = 0.f; return; }
    const float ib2 = __builtin_amdgcn_rcpf(b2);
    const float eb = (e[0] * b[0] + e[1] * b[1] + e[2] * b[2]) * ib2;
    for (int c = 0; c < 3; c++) o[c] = e[c] - eb * b[c];
    const float e2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    if (e2 >= b2 && e2 > 0.f) {
        const float s = __builtin_amdgcn_sqrtf(b2) * __builtin_amdgcn_rsqf(e2);
        for (int c = 0; c < 3; c++) o[c] = s * o[c];
    }
}

struct PertArrays {
    float *dE[3], *dB[3];
    const float *E0[3], *B0[3];
    const float *rE0[3];   // Ampere background rate curl(B0) at E positions
    const float *rB0[3];   // Faraday background rate -curl(E0) at B positions
    const float *rho0;     // div(E0) / 4 pi at nodes
};

__global__ void k_faraday_p(Geo<float> g, PertArrays P, float *__restrict__ br,
                            float *__restrict__ bt, float *__restrict__ bp, float h) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    size_t k = ix(ld, i, j);
    const float *er = P.dE[0], *et = P.dE[1], *ep = P.dE[2];
    if (j < nth) {
        float circ = g.rn[i] * (g.sn[j + 1] * ep[k + 1] - g.sn[j] * ep[k]);
        float v = P.dB[0][k] - h * circ / (g.rn2[i] * g.dcn[j]) + h * P.rB0[0][k];
        P.dB[0][k] = v;
        br[k] = P.B0[0][k] + v;
    }
    if (i < nr) {
        if (j > 0 && j < nth) {
            float circ = g.sn[j] * (g.rn[i + 1] * ep[k + ld] - g.rn[i] * ep[k]);
            float v = P.dB[1][k] + h * circ / (g.sn[j] * g.dr2n[i]) + h * P.rB0[1][k];
            P.dB[1][k] = v;
            bt[k] = P.B0[1][k] + v;
        } else {
            P.dB[1][k] = 0.f;
            bt[k] = 0.f;
        }
        if (j < nth) {
            float circ = g.dth * (g.rn[i + 1] * et[k + ld] - g.rn[i] * et[k]) -
                         g.drn[i] * (er[k + 1] - er[k]);
            float v = P.dB[2][k] - h * circ / (g.dth * g.dr2n[i]) + h * P.rB0[2][k];
            P.dB[2][k] = v;
            bp[k] = P.B0[2][k] + v;
        }
    }
}

__global__ void k_jffe_p(Geo<float> g, PertArrays P, const float *__restrict__ er,
                         const float *__restrict__ et, const float *__restrict__ ep,
                         const float *__restrict__ br, const float *__restrict__ bt,
                         const float *__restrict__ bp, float *__restrict__ j0,
                         float *__restrict__ j1, float *__restrict__ j2) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (j > g.nth) return;
    const float fourpi = (float)(4.0 * kPi);
    size_t k = ix(g.ld, i, j);
    int ii = i == 0 ? 1 : i;
    float rho = i == g.nr ? 0.f : div_e(g, P.dE[0], P.dE[1], ii, j) / fourpi + P.rho0[k];
    float e[3], b[3];
    node_e(g, er, et, ep, i, j, e);
    node_b(g, br, bt, bp, i, j, b);
    float b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    float x0 = e[1] * b[2] - e[2] * b[1];
    float x1 = e[2] * b[0] - e[0] * b[2];
    float x2 = e[0] * b[1] - e[1] * b[0];
    // at a magnetic null the drift current is undefined: zero (as for B = 0)
    bool ok = b2 > 1e-30f;
    const float rb = ok ? rho * __builtin_amdgcn_rcpf(b2) : 0.f;
    j0[k] = rb * x0;
    j1[k] = rb * x1;
    j2[k] = rb * x2;
}

__global__ void k_ampere_p(Geo<float> g, PertArrays P, float *__restrict__ er,
                           float *__restrict__ et, float *__restrict__ ep,
                           float *__restrict__ jr_, float *__restrict__ jt_,
                           float *__restrict__ jp_, const float *__restrict__ f,
                           const float *__restrict__ n0, const float *__restrict__ n1,
                           const float *__restrict__ n2, int ff) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    const float fourpi = (float)(4.0 * kPi);
    const float dt = g.dt;
    size_t k = ix(ld, i, j);
    // the deposit accumulators are consumed here and cleared for the next push
    const float jrk = jr_[k], jtk = jt_[k], jpk = jp_[k];
    jr_[k] = 0.f;
    jt_[k] = 0.f;
    jp_[k] = 0.f;
    const float *br = P.dB[0], *bt = P.dB[1], *bp = P.dB[2];
    if (i < nr) {
        float A = g.rh2[i] * g.dcd[j];
        float circ = (j < nth ? g.rh[i] * g.sh[j] * bp[k] : 0.f) -
                     (j > 0 ? g.rh[i] * g.sh[j - 1] * bp[k - 1] : 0.f);
        float J = jrk / (dt * A);
        if (ff) {
            float fs = 0.5f * (f[k] + f[k + ld]);
            if (fs > 0.f) J = (1.f - fs) * J + fs * 0.5f * (n0[k] + n0[k + ld]);
        }
        float v = P.dE[0][k] + dt * (circ / A + P.rE0[0][k]) - fourpi * dt * J;
        P.dE[0][k] = v;
        er[k] = P.E0[0][k] + v;
    }
    if (i >= 1 && i < nr) {
        if (j < nth) {
            float A = g.sh[j] * g.dr2h[i];
            float circ = -(g.rh[i] * g.sh[j] * bp[k] - g.rh[i - 1] * g.sh[j] * bp[k - ld]);
            float J = jtk / (dt * A);
            if (ff) {
                float fs = 0.5f * (f[k] + f[k + 1]);
                if (fs > 0.f) J = (1.f - fs) * J + fs * 0.5f * (n1[k] + n1[k + 1]);
            }
            float v = P.dE[1][k] + dt * (circ / A + P.rE0[1][k]) - fourpi * dt * J;
            P.dE[1][k] = v;
            et[k] = P.E0[1][k] + v;
        }
        if (j >= 1 && j < nth) {
            float A = g.dthd[j] * g.dr2h[i];
            float circ = g.dth * (g.rh[i] * bt[k] - g.rh[i - 1] * bt[k - ld]) -
                         g.drh[i] * (br[k] - br[k - 1]);
            float J = jpk / (g.dr3h[i] * g.dcd[j]);
            if (ff) {
                float fs = f[k];
                if (fs > 0.f) J = (1.f - fs) * J + fs * n2[k];
            }
            float v = P.dE[2][k] + dt * (circ / A + P.rE0[2][k]) - fourpi * dt * J;
            P.dE[2][k] = v;
            ep[k] = P.E0[2][k] + v;
        }
    }
}

__global__ void k_ffapply_p(Geo<float> g, PertArrays P, float *__restrict__ er,
                            float *__restrict__ et, float *__restrict__ ep,
                            const float *__restrict__ d0, const float *__restrict__ d1,
                            const float *__restrict__ d2) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    size_t k = ix(ld, i, j);
    if (i < nr) {
        float v = P.dE[0][k] + 0.5f * (d0[k] + d0[k + ld]);
        P.dE[0][k] = v;
        er[k] = P.E0[0][k] + v;
    }
    if (i >= 1 && i < nr) {
        if (j < nth) {
            float v = P.dE[1][k] + 0.5f * (d1[k] + d1[k + 1]);
            P.dE[1][k] = v;
            et[k] = P.E0[1][k] + v;
        }
        if (j >= 1 && j < nth) {
            float v = P.dE[2][k] + d2[k];
            P.dE[2][k] = v;
            ep[k] = P.E0[2][k] + v;
        }
    }
}

// absorbing layer in perturbation form (rows from i0 on)
__global__ void k_absorb_p(Geo<float> g, int i0, PertArrays P, float *__restrict__ er,
                           float *__restrict__ et, float *__restrict__ ep, float *__restrict__ br,
                           float *__restrict__ bt, float *__restrict__ bp) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = i0 + blockIdx.y;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    if (j > nth) return;
    size_t k = ix(ld, i, j);
    float ln = g.lamn[i];
    float lh = i < nr ? g.lamh[i] : 1.f;
    if (ln == 1.f && lh == 1.f) return;
    auto damp_e = [&](int c, float lam) {
        float tot = lam * (P.E0[c][k] + P.dE[c][k]);
        P.dE[c][k] = tot - P.E0[c][k];
        return tot;
    };
    auto damp_b = [&](int c, float lam) {
        float v = lam * P.dB[c][k];
        P.dB[c][k] = v;
        return P.B0[c][k] + v;
    };
    if (i < nr) {
        er[k] = damp_e(0, lh);
        bt[k] = damp_b(1, lh);
        if (j < nth) bp[k] = damp_b(2, lh);
    }
    ep[k] = damp_e(2, ln);
    if (j < nth) {
        et[k] = damp_e(1, ln);
        br[k] = damp_b(0, ln);
    }
}


// node corrections delta = f (E* - E) from E^{n+1} and B^{n+1/2} (FP32)
__global__ void k_ffdelta_f(Geo<float> g, const float *__restrict__ er, const float *__restrict__ et,
                            const float *__restrict__ ep, const float *__restrict__ br,
                            const float *__restrict__ bt, const float *__restrict__ bp,
                            const float *__restrict__ f, float *__restrict__ d0,
                            float *__restrict__ d1, float *__restrict__ d2) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (j > g.nth) return;
    size_t k = ix(g.ld, i, j);
    float fv = f[k];
    float o[3] = {0.f, 0.f, 0.f};
    if (fv > 0.f) {
        float e[3], b[3], s[3];
        node_e(g, er, et, ep, i, j, e);
        node_b(g, br, bt, bp, i, j, b);
        ff_node_f(e, b, s);
        for (int c = 0; c < 3; c++) o[c] = fv * (s[c] - e[c]);
    }
    d0[k] = o[0];
    d1[k] = o[1];
    d2[k] = o[2];
}

static void run_field_step_pert(ffpic_ctx *c) {
    Geo<float> g = geo<float>(c);
    dim3 blk(256), grd((c->nth + 1 + 255) / 256, c->nr + 1);
    float **E = (float **)c->E, **B = (float **)c->B, **J = (float **)c->J;
    float **S = (float **)c->scr;
    float *f = (float *)c->f;
    PertArrays P;
    for (int k = 0; k < 3; k++) {
        P.dE[k] = (float *)c->dE[k];
        P.dB[k] = (float *)c->dB[k];
        P.E0[k] = (const float *)c->E0[k];
        P.B0[k] = (const float *)c->B0[k];
        P.rE0[k] = (const float *)c->rE0[k];
        P.rB0[k] = (const float *)c->rB0[k];
    }
    P.rho0 = (const float *)c->rho0;
    int ff = c->d.ff_enable ? 1 : 0;
    float h = (float)(0.5 * c->dt);
    hipLaunchKernelGGL(k_faraday_p, grd, blk, 0, c->stream, g, P, B[0], B[1], B[2], h);
    if (ff)
        hipLaunchKernelGGL(k_jffe_p, grd, blk, 0, c->stream, g, P, E[0], E[1], E[2], B[0], B[1],
                           B[2], S[0], S[1], S[2]);
    hipLaunchKernelGGL(k_ampere_p, grd, blk, 0, c->stream, g, P, E[0], E[1], E[2], J[0], J[1],
                       J[2], f, S[0], S[1], S[2], ff);
    if (ff) {
        hipLaunchKernelGGL(k_ffdelta_f, grd, blk, 0, c->stream, g, E[0], E[1], E[2], B[0],
                           B[1], B[2], f, S[3], S[4], S[5]);
        hipLaunchKernelGGL(k_ffapply_p, grd, blk, 0, c->stream, g, P, E[0], E[1], E[2], S[3],
                           S[4], S[5]);
    }
    hipLaunchKernelGGL(k_faraday_p, grd, blk, 0, c->stream, g, P, B[0], B[1], B[2], h);
    if (c->absorb_row0 <= c->nr)
        hipLaunchKernelGGL(k_absorb_p, dim3(grd.x, c->nr + 1 - c->absorb_row0), blk, 0,
                           c->stream, g, c->absorb_row0, P, E[0], E[1], E[2], B[0], B[1], B[2]);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
