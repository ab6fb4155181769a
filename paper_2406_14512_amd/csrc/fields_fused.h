// The whole field step of Sect. 3 in one kernel: Faraday half step
// (eq. faraday, Stokes form on the primal faces), the force-free drift
// current at nodes (eq. JFFE: rho E x B / B^2 with rho = div E / 4 pi, from
// E^n and B^{n+1/2}), the blend of eq. (blending) at the staggered points
// (f averaged from the adjacent nodes) inside Ampere's law (eq. ampere, on
// the dual faces), the force-free E correction at nodes (E.B projected out,
// |E| capped at |B|, weighted by f) averaged back to the staggered points,
// the second Faraday half step, the absorbing layer of Sect. 4, and the
// totals the particle gather reads.  Corotation on the star: E_th and E_ph
// of row 0 are never updated; axis: E_ph = B_th = 0 on j = 0, nth.
//
// This file's kernel is the FP64 step, which evolves E and B.  The FP32
// step (fields_fused32.h, same stages and tiling) is a perturbation form.  In FP32 the
// static magnetosphere itself is the problem: the corotation E and the
// dipole B are discretely curl-free (or nearly so) in exact arithmetic, but
// once each component is rounded to FP32 their discrete curls are
// O(1e-7 |F| / cell) noise, which the Yee update would integrate into B_phi
// and E_phi every step.  So the FP32 state is dF = F - F0 about an FP64
// background F0 (the initial fields), whose discrete curls (the background
// rates) and charge density are evaluated once in FP64 on the host:
//   dB <- dB - h curl(dE) + h rateB0        (rateB0 = -curl E0)
//   dE <- dE + dt (curl(dB) + rateE0) - 4 pi dt J
//   rho = div(dE) / 4 pi + rho0
// Rounding then acts on the small perturbation, not on the background; the
// node quantities (J_FFE, the correction) use the totals F0 + dF, which the
// FP32 step also writes for the particle gather.
//
// Tiling.  A workgroup owns a strip of kFzW theta columns (plus kFzL halo
// columns before and kFzR after, one thread per column) and a slab of
// `rows` radial rows, and marches through the slab row by row, keeping the
// recent rows of each stage in registers (its own column) and in small
// LDS rings (the theta neighbours).  At iteration q it loads row q and
// computes
//   Faraday half step B^{n+1/2}    row q-1   (needs E^n rows q-1, q)
//   node J_FFE                     row q-1   (E^n rows q-2, q-1; B^{n+1/2} rows q-2, q-1)
//   Ampere E^{n+1}                 row q-2   (B^{n+1/2} rows q-3, q-2; J_FFE rows q-2, q-1)
//   node correction delta          row q-2   (E rows q-3, q-2; B^{n+1/2} rows q-3, q-2)
//   delta averaged back            row q-3   (delta rows q-3, q-2)
//   Faraday half step B^{n+1},     row q-4   (E rows q-4, q-3)
//   absorber, stores
// so each slab reads 2 rows above and 4 below its own, and every node is
// loaded and stored once.  Three workgroup barriers per row order the LDS
// exchanges.  Neighbouring slabs read each other's rows as halo, so the
// state is double-buffered (read one buffer, write the other), and so are
// the deposit accumulators: this step reads the push's and clears the
// other set for the next push.
#pragma once

#include <algorithm>
#include <utility>

#include "fields_impl.h"

namespace ffpic {

constexpr int kFzT = 256;                 // threads = columns of a strip with its halo
constexpr int kFzL = 2, kFzR = 4;         // halo columns before and after
constexpr int kFzW = kFzT - kFzL - kFzR;  // owned columns per strip

template <typename R>
struct FusedArgs {
    Geo<R> g;
    R h;                       // half time step
    int rows;                  // owned rows per workgroup
    int absorb0;               // first row whose absorber factor is below 1
    const R *sE[3], *sB[3];    // state in: E, B
    R *oE[3], *oB[3];          // state out (the other buffer)
    const R *B0[3];            // initial B (the absorber relaxes B to it)
    const R *J[3];             // this step's deposit accumulators
    R *Jz[3];                  // the other accumulators, cleared here
    const R *f;                // blending function at nodes
};

// force-free correction at a node in FP32 (E.B projection, then
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

template <typename R, bool FF>
__global__ void __launch_bounds__(kFzT) k_field_fused(const FusedArgs<R> A) {
    const Geo<R> &g = A.g;
    const int nr = g.nr, nth = g.nth, ld = g.ld;
    const int t = threadIdx.x;
    const int j = (int)blockIdx.x * kFzW + t - kFzL;
    const bool colok = j >= 0 && j <= nth;
    const int jc = min(max(j, 0), nth);
    const int tl = t > 0 ? t - 1 : t, tr = t < kFzT - 1 ? t + 1 : t;
    const int i0 = (int)blockIdx.y * A.rows;
    const int iL = min(i0 + A.rows - 1, nr);
    const int qs = max(i0 - 2, 0);
    const R dt = g.dt, h = A.h, dth = g.dth;
    const R fourpi = (R)(4.0 * kPi);
    // column geometry (indices clamped; used only where the stage's
    // condition on j holds)
    const bool jlt = j < nth, jgt = j > 0, jin = j > 0 && j < nth;
    const R sn_j = g.sn[jc], sn_j1 = g.sn[min(jc + 1, nth)];
    const R sh_j = g.sh[min(jc, nth - 1)], sh_jm = g.sh[max(jc - 1, 0)];
    const R dcn_j = g.dcn[min(jc, nth - 1)], dcd_j = g.dcd[jc], dthd_j = g.dthd[jc];

    // LDS rings (theta neighbours); a ring slot holds one row of one quantity
    __shared__ R lE[2][3][kFzT];          // E^n: r, phi, theta
    __shared__ R lB[4][2][kFzT];          // B^{n+1/2}: r, phi
    __shared__ R lN[FF ? 2 : 1][kFzT];    // J_FFE theta
    __shared__ R lF[FF ? 3 : 1][kFzT];    // f
    __shared__ R lEa[FF ? 2 : 1][kFzT];   // E after Ampere, theta
    __shared__ R lD[FF ? 2 : 1][kFzT];    // delta theta
    __shared__ R lEf[2][2][kFzT];         // final E: r, phi

    // own-column history (suffix = rows back from the newest loaded row q)
    R sE0[3] = {}, sE1[3] = {}, sE2[3] = {};        // E state rows q, q-1, q-2
    R sB0[3] = {}, sB1[3] = {};                     // B state rows q, q-1
    R f0 = 0, f1 = 0, f2 = 0;                       // f rows q, q-1, q-2
    R J0[3] = {}, J1[3] = {}, J2[3] = {};           // deposit rows q, q-1, q-2
    R Bh1[3] = {}, Bh2[3] = {}, Bh3[3] = {}, Bh4[3] = {};   // B^{n+1/2} rows q-1..q-4
    R n01 = 0, n02 = 0, n11 = 0, n12 = 0, n21 = 0, n22 = 0;   // J_FFE rows q-1, q-2
    R Ea2[3] = {}, Ea3[3] = {};                     // E after Ampere (state) rows q-2, q-3
    R Eat3r = 0;                                    // its E_r, row q-3
    R d02 = 0, d03 = 0, d13 = 0, d23 = 0;           // delta rows q-2, q-3
    R d12 = 0, d22 = 0;
    R Ef3[3] = {}, Ef4[3] = {};                     // final E (state) rows q-3, q-4

    for (int q = qs; q <= iL + 4; q++) {
        // ---- load row q
        if (q <= nr) {
            const bool ok = colok;
            const size_t k = ix(ld, q, jc);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                sE0[c] = ok ? A.sE[c][k] : (R)0;
                sB0[c] = ok ? A.sB[c][k] : (R)0;
                J0[c] = ok ? A.J[c][k] : (R)0;
            }
            if constexpr (FF) f0 = ok ? A.f[k] : (R)0;
            lE[q & 1][0][t] = sE0[0];
            lE[q & 1][1][t] = sE0[2];
            lE[q & 1][2][t] = sE0[1];
            if constexpr (FF) lF[q % 3][t] = f0;
        }

        // ---- Faraday half step, row a = q - 1: B^{n+1/2}
        const int a = q - 1;
        if (a >= qs && a <= nr) {
            const R *nb = lE[a & 1][0];   // row a, E state r at j+1 is nb[tr]
            const R epn = lE[a & 1][1][tr];
            const R ern = nb[tr];
            R v[3];
            // B_r (j < nth)
            {
                R circ = g.rn[a] * (sn_j1 * epn - sn_j * sE1[2]);
                v[0] = sB1[0] - h * circ / (g.rn2[a] * dcn_j);
                if (!jlt) v[0] = sB1[0];
            }
            if (a < nr) {
                if (jin) {
                    R circ = sn_j * (g.rn[a + 1] * sE0[2] - g.rn[a] * sE1[2]);
                    v[1] = sB1[1] + h * circ / (sn_j * g.dr2n[a]);
                } else {
                    v[1] = (R)0;
                }
                if (jlt) {
                    R circ = dth * (g.rn[a + 1] * sE0[1] - g.rn[a] * sE1[1]) -
                             g.drn[a] * (ern - sE1[0]);
                    v[2] = sB1[2] - h * circ / (dth * g.dr2n[a]);
                } else {
                    v[2] = sB1[2];
                }
            } else {
                v[1] = sB1[1];
                v[2] = sB1[2];
            }
#pragma unroll
            for (int c = 0; c < 3; c++) Bh1[c] = v[c];
            lB[a & 3][0][t] = v[0];
            lB[a & 3][1][t] = v[2];
        }
        __syncthreads();

        // ---- node J_FFE, row b = q - 1 (needs B^{n+1/2} rows b-1, b)
        const int b = q - 1;
        if constexpr (FF) {
            if (b >= qs && b <= nr && (b == 0 || b - 1 >= qs)) {
                // rho = div E / 4 pi over the dual cell of node (max(b, 1), j)
                R rho = (R)0;
                if (b < nr) {
                    // rows ii and ii - 1 of the E state (own column), theta at j-1
                    const bool one = b == 0;
                    const int ii = one ? 1 : b;
                    const R er_i = one ? sE0[0] : sE1[0];
                    const R er_m = one ? sE1[0] : sE2[0];
                    const R et_i = one ? sE0[1] : sE1[1];
                    const R et_l = lE[ii & 1][2][tl];
                    R flux = g.rh2[ii] * dcd_j * er_i - g.rh2[ii - 1] * dcd_j * er_m;
                    if (jlt) flux += sh_j * g.dr2h[ii] * et_i;
                    if (jgt) flux -= sh_jm * g.dr2h[ii] * et_l;
                    R dv = flux / (g.dr3h[ii] * dcd_j);
                    rho = dv / fourpi;
                }
                // node E^n (totals) and B^{n+1/2} (totals)
                R e[3], bb[3];
                {
                    R tr_i = sE1[0];
                    R tr_m = sE2[0];
                    e[0] = b == 0 ? tr_i : b == nr ? tr_m : (R)0.5 * (tr_m + tr_i);
                    R tt_j = sE1[1];
                    R tt_l = lE[b & 1][2][tl];
                    e[1] = (j == 0 || j == nth) ? (R)0 : (R)0.5 * (tt_l + tt_j);
                    e[2] = sE1[2];
                }
                {
                    const R br_l = lB[b & 3][0][tl];
                    bb[0] = j == 0 ? Bh1[0] : j == nth ? br_l : (R)0.5 * (br_l + Bh1[0]);
                    bb[1] = b == 0 ? Bh1[1] : b == nr ? Bh2[1] : (R)0.5 * (Bh2[1] + Bh1[1]);
                    const R bp_l = lB[b & 3][1][tl];
                    if (j == 0 || j == nth) {
                        bb[2] = (R)0;
                    } else if (b == 0) {
                        bb[2] = (R)0.5 * (bp_l + Bh1[2]);
                    } else if (b == nr) {
                        bb[2] = (R)0.5 * (lB[(b - 1) & 3][1][tl] + Bh2[2]);
                    } else {
                        bb[2] = (R)0.25 * (lB[(b - 1) & 3][1][tl] + Bh2[2] + bp_l + Bh1[2]);
                    }
                }
                R b2 = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
                R x0 = e[1] * bb[2] - e[2] * bb[1];
                R x1 = e[2] * bb[0] - e[0] * bb[2];
                R x2 = e[0] * bb[1] - e[1] * bb[0];
                {
                    bool ok = b2 > (R)0;
                    n01 = ok ? rho * x0 / b2 : (R)0;
                    n11 = ok ? rho * x1 / b2 : (R)0;
                    n21 = ok ? rho * x2 / b2 : (R)0;
                }
                lN[b & 1][t] = n11;
            }
        }

        // ---- Ampere, row c = q - 2: E after Ampere
        const int c = q - 2;
        if (c >= qs && c <= nr && (c == 0 || c - 1 >= qs)) {
            R v[3] = {sE2[0], sE2[1], sE2[2]};
            const R *bl = lB[c & 3][0];   // row c, B^{n+1/2} state r, j-1 at [tl]
            const R bp_l = lB[c & 3][1][tl];
            const R jrk = J2[0], jtk = J2[1], jpk = J2[2];
            if (c < nr) {
                R Ar = g.rh2[c] * dcd_j;
                R circ = (jlt ? g.rh[c] * sh_j * Bh2[2] : (R)0) -
                         (jgt ? g.rh[c] * sh_jm * bp_l : (R)0);
                R J;
                if constexpr (FF) {
                    R fs = (R)0.5 * (f2 + f1);
                    {
                        J = ((R)1 - fs) * jrk / (dt * Ar) + fs * (R)0.5 * (n02 + n01);
                    }
                } else {
                    J = jrk / (dt * Ar);
                }
                v[0] = sE2[0] + (dt * circ / Ar - fourpi * dt * J);
            }
            if (c >= 1 && c < nr) {
                if (jlt) {
                    R At = sh_j * g.dr2h[c];
                    R circ = -(g.rh[c] * sh_j * Bh2[2] - g.rh[c - 1] * sh_j * Bh3[2]);
                    R J;
                    if constexpr (FF) {
                        R fs = (R)0.5 * (f2 + lF[c % 3][tr]);
                        {
                            J = ((R)1 - fs) * jtk / (dt * At) + fs * (R)0.5 * (n12 + lN[c & 1][tr]);
                        }
                    } else {
                        J = jtk / (dt * At);
                    }
                    v[1] = sE2[1] + (dt * circ / At - fourpi * dt * J);
                }
                if (jin) {
                    R Ap = dthd_j * g.dr2h[c];
                    R circ = dth * (g.rh[c] * Bh2[1] - g.rh[c - 1] * Bh3[1]) -
                             g.drh[c] * (Bh2[0] - bl[tl]);
                    R J;
                    if constexpr (FF) {
                        R fs = f2;
                        {
                            J = ((R)1 - fs) * jpk / (g.dr3h[c] * dcd_j) + fs * n22;
                        }
                    } else {
                        J = jpk / (g.dr3h[c] * dcd_j);
                    }
                    v[2] = sE2[2] + (dt * circ / Ap - fourpi * dt * J);
                }
            }
#pragma unroll
            for (int k = 0; k < 3; k++) Ea2[k] = v[k];
            if constexpr (FF) lEa[c & 1][t] = v[1];
        }
        __syncthreads();

        // ---- force-free correction at nodes, row d = q - 2
        const int d = q - 2;
        if constexpr (FF) {
            if (d >= qs && d <= nr && (qs == 0 || d >= qs + 2)) {
                R o[3] = {(R)0, (R)0, (R)0};
                if (f2 > (R)0) {
                    R e[3], bb[3], s[3];
                    const R tr_i = Ea2[0];
                    e[0] = d == 0 ? tr_i : d == nr ? Eat3r : (R)0.5 * (Eat3r + tr_i);
                    const R tt_j = Ea2[1];
                    e[1] = (j == 0 || j == nth) ? (R)0 : (R)0.5 * (lEa[d & 1][tl] + tt_j);
                    e[2] = Ea2[2];
                    const R br_l = lB[d & 3][0][tl];
                    bb[0] = j == 0 ? Bh2[0] : j == nth ? br_l : (R)0.5 * (br_l + Bh2[0]);
                    bb[1] = d == 0 ? Bh2[1] : d == nr ? Bh3[1] : (R)0.5 * (Bh3[1] + Bh2[1]);
                    const R bp_l = lB[d & 3][1][tl];
                    if (j == 0 || j == nth) {
                        bb[2] = (R)0;
                    } else if (d == 0) {
                        bb[2] = (R)0.5 * (bp_l + Bh2[2]);
                    } else if (d == nr) {
                        bb[2] = (R)0.5 * (lB[(d - 1) & 3][1][tl] + Bh3[2]);
                    } else {
                        bb[2] = (R)0.25 * (lB[(d - 1) & 3][1][tl] + Bh3[2] + bp_l + Bh2[2]);
                    }
                    ff_node<R>(e, bb, s);
#pragma unroll
                    for (int k = 0; k < 3; k++) o[k] = f2 * (s[k] - e[k]);
                }
                d02 = o[0];
                d12 = o[1];
                d22 = o[2];
                lD[d & 1][t] = o[1];
            }
        }

        // ---- corrections averaged back, row e = q - 3: final E
        const int e = q - 3;
        if (e >= i0 && e <= nr) {
            R v[3] = {Ea3[0], Ea3[1], Ea3[2]};
            if constexpr (FF) {
                if (e < nr) v[0] = Ea3[0] + (R)0.5 * (d03 + d02);
                if (e >= 1 && e < nr) {
                    if (jlt) v[1] = Ea3[1] + (R)0.5 * (d13 + lD[e & 1][tr]);
                    if (jin) v[2] = Ea3[2] + d23;
                }
            }
#pragma unroll
            for (int k = 0; k < 3; k++) Ef3[k] = v[k];
            lEf[e & 1][0][t] = v[0];
            lEf[e & 1][1][t] = v[2];
        }

        // ---- Faraday half step, row f = q - 4: B^{n+1}, absorber, stores
        const int fr = q - 4;
        if (fr >= i0 && fr <= iL) {
            const R epn = lEf[fr & 1][1][tr];
            const R ern = lEf[fr & 1][0][tr];
            R vb[3];
            {
                R circ = g.rn[fr] * (sn_j1 * epn - sn_j * Ef4[2]);
                vb[0] = Bh4[0] - h * circ / (g.rn2[fr] * dcn_j);
                if (!jlt) vb[0] = Bh4[0];
            }
            if (fr < nr) {
                if (jin) {
                    R circ = sn_j * (g.rn[fr + 1] * Ef3[2] - g.rn[fr] * Ef4[2]);
                    vb[1] = Bh4[1] + h * circ / (sn_j * g.dr2n[fr]);
                } else {
                    vb[1] = (R)0;
                }
                if (jlt) {
                    R circ = dth * (g.rn[fr + 1] * Ef3[1] - g.rn[fr] * Ef4[1]) -
                             g.drn[fr] * (ern - Ef4[0]);
                    vb[2] = Bh4[2] - h * circ / (dth * g.dr2n[fr]);
                } else {
                    vb[2] = Bh4[2];
                }
            } else {
                vb[1] = Bh4[1];
                vb[2] = Bh4[2];
            }
            R ve[3] = {Ef4[0], Ef4[1], Ef4[2]};
            // absorbing layer: E damped, B relaxed to its initial value
            if (fr >= A.absorb0) {
                const R ln = g.lamn[fr];
                const R lh = fr < nr ? g.lamh[fr] : (R)1;
                if (!(ln == (R)1 && lh == (R)1)) {
                    const size_t k = ix(ld, fr, jc);
                    if (fr < nr) {
                        ve[0] *= lh;
                        const R b0t = A.B0[1][k];
                        vb[1] = b0t + lh * (vb[1] - b0t);
                        if (jlt) {
                            const R b0p = A.B0[2][k];
                            vb[2] = b0p + lh * (vb[2] - b0p);
                        }
                    }
                    ve[2] *= ln;
                    if (jlt) {
                        ve[1] *= ln;
                        const R b0r = A.B0[0][k];
                        vb[0] = b0r + ln * (vb[0] - b0r);
                    }
                }
            }
            if (t >= kFzL && t < kFzL + kFzW && colok) {
                const size_t k = ix(ld, fr, j);
#pragma unroll
                for (int kk = 0; kk < 3; kk++) {
                    A.oE[kk][k] = ve[kk];
                    A.oB[kk][k] = vb[kk];
                    A.Jz[kk][k] = (R)0;
                }
            }
        }
        __syncthreads();

        // ---- shift the own-column histories by one row
        Eat3r = Ea2[0];   // E_r after Ampere, row q-2
#pragma unroll
        for (int k = 0; k < 3; k++) {
            sE2[k] = sE1[k]; sE1[k] = sE0[k];
            sB1[k] = sB0[k];
            J2[k] = J1[k]; J1[k] = J0[k];
            Bh4[k] = Bh3[k]; Bh3[k] = Bh2[k]; Bh2[k] = Bh1[k];
            Ea3[k] = Ea2[k];
            Ef4[k] = Ef3[k];
        }
        if constexpr (FF) {
            f2 = f1; f1 = f0;
            n02 = n01; n12 = n11; n22 = n21;
            d03 = d02; d13 = d12; d23 = d22;
        }
    }
}

// slab height: enough slabs that the grid fills the GPU once, at least 32
// rows each (the halo costs 6 rows per slab)
inline int fused_rows(const ffpic_ctx *c) {
    const int nbx = (c->nth + 1 + kFzW - 1) / kFzW;
    const int slots = c->fused_slots > 0 ? c->fused_slots : 768;
    const int slabs = std::max(1, slots / nbx);
    const int rows = (c->nr + 1 + slabs - 1) / slabs;
    return c->fused_rows > 0 ? c->fused_rows : std::max(32, rows);
}

// FP64 field step (E and B evolved directly)
static void run_field_fused64(ffpic_ctx *c) {
    using R = double;
    FusedArgs<R> A{};
    A.g = geo<R>(c);
    A.h = (R)(0.5 * c->dt);
    A.absorb0 = c->absorb_row0;
    for (int k = 0; k < 3; k++) {
        A.sE[k] = (const R *)c->E[k];  A.sB[k] = (const R *)c->B[k];
        A.oE[k] = (R *)c->stAlt[k];    A.oB[k] = (R *)c->stAlt[3 + k];
        A.B0[k] = (const R *)c->B0[k];
        A.J[k] = (const R *)c->J[k];
        A.Jz[k] = (R *)c->Jalt[k];
    }
    A.f = (const R *)c->f;
    auto kern = c->d.ff_enable ? k_field_fused<R, true> : k_field_fused<R, false>;
    if (c->fused_slots == 0) {   // workgroups resident at once, for the slab height
        int per_cu = 0, cus = 0, dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, kFzT, 0) !=
                hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            per_cu = 3;
            cus = 256;
        }
        c->fused_slots = std::max(1, per_cu * cus);
    }
    A.rows = fused_rows(c);
    dim3 grd((c->nth + 1 + kFzW - 1) / kFzW, (c->nr + 1 + A.rows - 1) / A.rows);
    hipLaunchKernelGGL(kern, grd, dim3(kFzT), 0, c->stream, A);
    FFPIC_LAUNCH_CHECK();
    // the new state and the cleared accumulators become current
    for (int k = 0; k < 3; k++) {
        std::swap(c->E[k], c->stAlt[k]);
        std::swap(c->B[k], c->stAlt[3 + k]);
        std::swap(c->J[k], c->Jalt[k]);
    }
}

}  // namespace ffpic
