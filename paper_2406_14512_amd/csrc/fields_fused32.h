// The FP32 field step (perturbation form, fields_fused.h) with fewer
// instructions per node than the generic kernel there:
//  * every FP32 division of the step is a product with a reciprocal or a
//    ratio of the FP64 geometry, rounded once on the host into per-row and
//    per-column coefficient tables (same quantities, a few ulp of FP32
//    rounding apart from the divided form);
//  * the row loop is unrolled by four, and each row quantity a thread keeps
//    lives in a register ring whose slot is a compile-time constant, so
//    nothing is shifted from register to register as the march advances;
//  * every array is loaded one iteration before it is used, at the row
//    where its first use needs it;
//  * the row coefficients are uniform loads (scalar cache) and the element
//    offsets 32-bit.
// The stages, their rows at iteration q, the LDS exchanges and the three
// barriers per row are those of k_field_fused; so is the result, up to the
// rounding of the coefficients.
#pragma once

#include "fields_fused.h"

namespace ffpic {

// coefficients of radial row i (float4 #k = entries 4k..4k+3):
//  #0: h / r_i,  h / dr2n_i,  r_i,  r_{i+1}
//  #1: drn_i / dth, and for the divergence over the dual cell of node row i
//      (ii = max(i, 1)): rh2_ii / (4 pi dr3h_ii), rh2_{ii-1} / (4 pi dr3h_ii),
//      dr2h_ii / (4 pi dr3h_ii)
//  #2: dt / rh_i,  4 pi / rh2_i,  dt / dr2h_i,  rh_i
//  #3: rh_{i-1},  4 pi / dr2h_i,  drh_i / dth,  dt dth / dr2h_i
//  #4: 4 pi dt / dr3h_i,  lamn_i,  lamh_i (1 on the last row),  0
// (entries that do not exist on a boundary row are 0 and never used)
constexpr int kRowC = 5;
// coefficients of theta column j: #0: sin th_j, sin th_{j+1}, 1 / dcn_j,
// sin th_{j+1/2};  #1: sin th_{j-1/2}, 1 / dcd_j, 1 / sin th_{j+1/2},
// 1 / dthd_j  (0 where the column has no such entry)
constexpr int kColC = 2;

// Each three-component field is one allocation with its components cs
// elements apart; the kernel takes the base (component 0) of each.
struct F32Args {
    int nr, nth, ld, rows, absorb0;
    unsigned cs;                       // elements between components
    unsigned rates;                    // bit k: curl B0 component k is not zero;
                                       // bit 3 + k: -curl E0 component k is not zero
    float h, dt, fpdt;                 // half step, step, 4 pi dt
    const float *sE, *sB;              // perturbation state in
    float *oE, *oB;                    // state out (the other buffer)
    float *tE, *tB;                    // totals E0 + dE, B0 + dB
    const float *E0, *B0, *rE0, *rB0, *J;
    float *Jz;                         // accumulators cleared for the next push
    const float *rho0, *f;
    const float4 *colc;
};

__device__ __forceinline__ float ld32(const float *base, unsigned off) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + (off << 2));
}
__device__ __forceinline__ void st32(float *base, unsigned off, float v) {
    *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + (off << 2)) = v;
}

template <bool FF, int RE, bool RB>
struct F32Kernel {
    const F32Args &A;
    const float4 *__restrict__ rowc;
    int nr, nth, ld, t, j, tl, tr, i0, iL, qs;
    unsigned jc;
    bool jlt, jgt, jin, own;
    float sn_j, sn_j1, cA_j, sh_j, sh_jm, cdcd_j, csh_j, cdthd_j;
    // LDS rings, indexed by absolute row (theta neighbours)
    float (*lE)[4][kFzT];   // [2]: state r, state phi, state theta, total theta
    float (*lB)[4][kFzT];   // [4]: total r, total phi, state r, state phi
    float (*lN)[kFzT];      // [2]: J_FFE theta
    float (*lF)[kFzT];      // [3]: f
    float (*lEa)[kFzT];     // [2]: total theta after Ampere
    float (*lD)[kFzT];      // [2]: delta theta
    float (*lEf)[2][kFzT];  // [2]: final state r, phi
    // register rings, indexed by (row - qs) & (size - 1)
    float sE[4][3], e0[4][3];      // rows q+1 .. q-2
    float sB[2][3], b0[4][3];      // rows q, q-1 (B0: rows q .. q-3)
    float rho[2], fv[4];           // rho0 rows q, q-1; f rows q .. q-3
    float Jr[2][3], rE[2][3] = {};  // rows q-1, q-2
    float Bh[4][3], Bt[4][3];      // B^{n+1/2} state and total, rows q-1 .. q-4
    float n[2][3];                 // J_FFE rows q-1, q-2
    float Ea[2][3], Eatr[2];       // E after Ampere (state), its total E_r: rows q-2, q-3
    float dl[2][3];                // delta rows q-2, q-3
    float Ef[2][3];                // final E state rows q-3, q-4
    float eF[2][3], bF[2][3];      // E0, B0 rows q-3, q-4 (totals, absorber)
    float rbA[4][3], rbF[2][3];    // -curl E0 rows q .. q-3 (Faraday at a) and q-3, q-4 (at fr)

    __device__ __forceinline__ unsigned off(int row) const { return (unsigned)row * (unsigned)ld + jc; }
    __device__ __forceinline__ float4 rc(int row, int k) const { return rowc[row * kRowC + k]; }

    // Every load below is issued on every iteration (rows clamped to the
    // grid), and every stage computes on every iteration, whether or not its
    // row is one the slab needs: the values of rows outside a stage's valid
    // range never reach a stored value, and with no branch around a load the
    // number of loads in flight is the same on every path, so each wait is
    // for exactly the load it needs.  Only LDS writes and stores are guarded.
    template <int P>
    __device__ __forceinline__ void step(int q) {
        constexpr int s4_1 = (P + 1) & 3, s4_0 = P & 3, s4_m1 = (P + 3) & 3, s4_m2 = (P + 2) & 3;
        constexpr int s4_m3 = (P + 1) & 3, s4_m4 = P & 3;
        constexpr int s2_0 = P & 1, s2_m1 = (P + 1) & 1;   // rows q (= q-2), q-1 (= q-3)
        const float h = A.h, dt = A.dt, fpdt = A.fpdt;
        const unsigned cs = A.cs;
        auto clampr = [&](int r) { return min(max(r, 0), nr); };

        // ---- loads for the coming iterations.  E0, B0 (and -curl E0) of row
        // q-3, which the stores of the next iteration need, are taken from
        // the rings that loaded them four rows ago (row q-3 shares its ring
        // slot with row q+1, so before that slot is reloaded), not read again
        {
            const unsigned o1 = off(clampr(q + 1)), o0 = off(clampr(q));
            const unsigned om1 = off(clampr(q - 1));
#pragma unroll
            for (int c = 0; c < 3; c++) {
                eF[s2_m1][c] = e0[s4_1][c];                 // E0, B0 of row q-3 (stores)
                bF[s2_m1][c] = b0[s4_1][c];
                if constexpr (RB) rbF[s2_m1][c] = rbA[s4_1][c];   // row q-3, Faraday at q+1
            }
#pragma unroll
            for (int c = 0; c < 3; c++) {
                sE[s4_1][c] = ld32(A.sE, o1 + c * cs);      // E^n state and E0, row q+1
                e0[s4_1][c] = ld32(A.E0, o1 + c * cs);
                sB[s2_0][c] = ld32(A.sB, o0 + c * cs);      // B state and B0, row q
                b0[s4_0][c] = ld32(A.B0, o0 + c * cs);
                Jr[s2_m1][c] = ld32(A.J, om1 + c * cs);     // deposit, row q-1
            }
            if constexpr (RE & 1) rE[s2_m1][0] = ld32(A.rE0, om1);
            if constexpr (RE & 2) rE[s2_m1][1] = ld32(A.rE0, om1 + cs);
            if constexpr (RE & 4) rE[s2_m1][2] = ld32(A.rE0, om1 + 2 * cs);
            if constexpr (FF) {
                rho[s2_0] = ld32(A.rho0, o0);
                fv[s4_0] = ld32(A.f, o0);
            }
            if constexpr (RB) {
#pragma unroll
                for (int c = 0; c < 3; c++) rbA[s4_0][c] = ld32(A.rB0, o0 + c * cs);   // row q
            }
        }

        // ---- LDS: E^n row q (neighbours of the Faraday and J_FFE stages),
        //      f row q-1 (neighbour of Ampere)
        if (q <= nr) {
            lE[q & 1][0][t] = sE[s4_0][0];
            lE[q & 1][1][t] = sE[s4_0][2];
            lE[q & 1][2][t] = sE[s4_0][1];
            lE[q & 1][3][t] = e0[s4_0][1] + sE[s4_0][1];
        }
        if constexpr (FF) {
            if (q >= 1 && q - 1 <= nr) lF[(q - 1) % 3][t] = fv[s4_m1];
        }

        // ---- Faraday half step, row a = q - 1
        const int a = q - 1;
        {
            const int ar = clampr(a);
            const bool inner = a < nr;
            const float4 c0 = rc(ar, 0), c1 = rc(ar, 1);
            const float *Ea1 = sE[s4_m1], *Ea0 = sE[s4_0];   // rows a, a+1
            const float *sb = sB[s2_m1];
            const float epn = lE[a & 1][1][tr], ern = lE[a & 1][0][tr];
            float v[3];
            v[0] = jlt ? sb[0] - c0.x * cA_j * (sn_j1 * epn - sn_j * Ea1[2]) : sb[0];
            const float v1 = jin ? sb[1] + c0.y * (c0.w * Ea0[2] - c0.z * Ea1[2]) : 0.f;
            const float v2 = jlt ? sb[2] - c0.y * ((c0.w * Ea0[1] - c0.z * Ea1[1]) - c1.x * (ern - Ea1[0]))
                                 : sb[2];
            v[1] = inner ? v1 : sb[1];
            v[2] = inner ? v2 : sb[2];
            if constexpr (RB) {
                const float *rb = rbA[s4_m1];
                v[0] += jlt ? h * rb[0] : 0.f;
                v[1] += (inner && jin) ? h * rb[1] : 0.f;
                v[2] += (inner && jlt) ? h * rb[2] : 0.f;
            }
#pragma unroll
            for (int c = 0; c < 3; c++) {
                Bh[s4_m1][c] = v[c];
                Bt[s4_m1][c] = b0[s4_m1][c] + v[c];
            }
            if (inner && !jin) Bt[s4_m1][1] = 0.f;
            if (a >= 0 && a <= nr) {
                lB[a & 3][0][t] = Bt[s4_m1][0];
                lB[a & 3][1][t] = Bt[s4_m1][2];
                lB[a & 3][2][t] = v[0];
                lB[a & 3][3][t] = v[2];
            }
        }
        __syncthreads();

        // ---- node J_FFE, row b = q - 1
        const int b = q - 1;
        if constexpr (FF) {
            const int br = clampr(b);
            const bool one = b == 0;
            const float4 c1 = rc(br, 1);
            const float er_i = one ? sE[s4_0][0] : sE[s4_m1][0];
            const float er_m = one ? sE[s4_m1][0] : sE[s4_m2][0];
            const float et_i = one ? sE[s4_0][1] : sE[s4_m1][1];
            const float et_l = lE[(one ? 1 : b) & 1][2][tl];
            const float T = (jlt ? sh_j * et_i : 0.f) - (jgt ? sh_jm * et_l : 0.f);
            const float rhov =
                b < nr ? (c1.y * er_i - c1.z * er_m) + c1.w * T * cdcd_j + rho[s2_m1] : 0.f;
            const float tr_i = e0[s4_m1][0] + sE[s4_m1][0];
            const float tr_m = e0[s4_m2][0] + sE[s4_m2][0];
            float e[3], bb[3];
            e[0] = b == 0 ? tr_i : b == nr ? tr_m : 0.5f * (tr_m + tr_i);
            e[1] = (j == 0 || j == nth) ? 0.f
                                        : 0.5f * (lE[b & 1][3][tl] + (e0[s4_m1][1] + sE[s4_m1][1]));
            e[2] = e0[s4_m1][2] + sE[s4_m1][2];
            const float brl = lB[b & 3][0][tl];
            bb[0] = j == 0 ? Bt[s4_m1][0] : j == nth ? brl : 0.5f * (brl + Bt[s4_m1][0]);
            bb[1] = b == 0 ? Bt[s4_m1][1] : b == nr ? Bt[s4_m2][1] : 0.5f * (Bt[s4_m2][1] + Bt[s4_m1][1]);
            const float bpl = lB[b & 3][1][tl], bpml = lB[(b - 1) & 3][1][tl];
            const float bp4 = 0.25f * (bpml + Bt[s4_m2][2] + bpl + Bt[s4_m1][2]);
            const float bp0 = 0.5f * (bpl + Bt[s4_m1][2]);
            const float bpn = 0.5f * (bpml + Bt[s4_m2][2]);
            bb[2] = (j == 0 || j == nth) ? 0.f : b == 0 ? bp0 : b == nr ? bpn : bp4;
            const float b2 = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
            const float rb = b2 > 1e-30f ? rhov * __builtin_amdgcn_rcpf(b2) : 0.f;
            n[s2_m1][0] = rb * (e[1] * bb[2] - e[2] * bb[1]);
            n[s2_m1][1] = rb * (e[2] * bb[0] - e[0] * bb[2]);
            n[s2_m1][2] = rb * (e[0] * bb[1] - e[1] * bb[0]);
            if (b >= 0 && b <= nr) lN[b & 1][t] = n[s2_m1][1];
        }

        // ---- Ampere, row c = q - 2
        const int c = q - 2;
        {
            const int cr = clampr(c);
            const float4 c2 = rc(cr, 2), c3 = rc(cr, 3), c4 = rc(cr, 4);
            const float bpl = lB[c & 3][3][tl], brl = lB[c & 3][2][tl];
            const float *bh = Bh[s4_m2], *bhm = Bh[s4_m3];   // rows c, c-1
            const float *jj = Jr[s2_0], *se = sE[s4_m2];
            float Jr_ = c2.y * jj[0] * cdcd_j, Jt_ = c3.y * jj[1] * csh_j, Jp_ = c4.x * jj[2] * cdcd_j;
            if constexpr (FF) {
                const float fsr = 0.5f * (fv[s4_m2] + fv[s4_m1]);
                const float fst = 0.5f * (fv[s4_m2] + lF[c % 3 < 0 ? 0 : c % 3][tr]);
                const float fsp = fv[s4_m2];
                const float nr_ = fpdt * 0.5f * (n[s2_0][0] + n[s2_m1][0]);
                const float nt_ = fpdt * 0.5f * (n[s2_0][1] + lN[c & 1][tr]);
                const float np_ = fpdt * n[s2_0][2];
                Jr_ = fsr > 0.f ? (1.f - fsr) * Jr_ + fsr * nr_ : Jr_;
                Jt_ = fst > 0.f ? (1.f - fst) * Jt_ + fst * nt_ : Jt_;
                Jp_ = fsp > 0.f ? (1.f - fsp) * Jp_ + fsp * np_ : Jp_;
            }
            const float circr = (jlt ? sh_j * bh[2] : 0.f) - (jgt ? sh_jm * bpl : 0.f);
            const float vr = se[0] + c2.x * circr * cdcd_j + dt * rE[s2_0][0] - Jr_;
            const float vt = se[1] - c2.z * (c2.w * bh[2] - c3.x * bhm[2]) + dt * rE[s2_0][1] - Jt_;
            const float vp = se[2] +
                             cdthd_j * c3.w * ((c2.w * bh[1] - c3.x * bhm[1]) - c3.z * (bh[0] - brl)) +
                             dt * rE[s2_0][2] - Jp_;
            const bool inner = c < nr, mid = c >= 1 && c < nr;
            Ea[s2_0][0] = inner ? vr : se[0];
            Ea[s2_0][1] = (mid && jlt) ? vt : se[1];
            Ea[s2_0][2] = (mid && jin) ? vp : se[2];
            Eatr[s2_0] = e0[s4_m2][0] + Ea[s2_0][0];
            if constexpr (FF) {
                if (c >= 0 && c <= nr) lEa[c & 1][t] = e0[s4_m2][1] + Ea[s2_0][1];
            }
        }
        __syncthreads();

        // ---- node force-free correction, row d = q - 2
        const int d = q - 2;
        if constexpr (FF) {
            float o3[3] = {0.f, 0.f, 0.f};
            const float fd = fv[s4_m2];
            if (fd > 0.f) {
                float e[3], bb[3], s3[3];
                e[0] = d == 0 ? Eatr[s2_0] : d == nr ? Eatr[s2_m1] : 0.5f * (Eatr[s2_m1] + Eatr[s2_0]);
                e[1] = (j == 0 || j == nth) ? 0.f
                                            : 0.5f * (lEa[d & 1][tl] + (e0[s4_m2][1] + Ea[s2_0][1]));
                e[2] = e0[s4_m2][2] + Ea[s2_0][2];
                const float brl = lB[d & 3][0][tl];
                bb[0] = j == 0 ? Bt[s4_m2][0] : j == nth ? brl : 0.5f * (brl + Bt[s4_m2][0]);
                bb[1] = d == 0 ? Bt[s4_m2][1] : d == nr ? Bt[s4_m3][1] : 0.5f * (Bt[s4_m3][1] + Bt[s4_m2][1]);
                const float bpl = lB[d & 3][1][tl], bpml = lB[(d - 1) & 3][1][tl];
                const float bp4 = 0.25f * (bpml + Bt[s4_m3][2] + bpl + Bt[s4_m2][2]);
                const float bp0 = 0.5f * (bpl + Bt[s4_m2][2]);
                const float bpn = 0.5f * (bpml + Bt[s4_m3][2]);
                bb[2] = (j == 0 || j == nth) ? 0.f : d == 0 ? bp0 : d == nr ? bpn : bp4;
                ff_node_f(e, bb, s3);
#pragma unroll
                for (int k = 0; k < 3; k++) o3[k] = fd * (s3[k] - e[k]);
            }
#pragma unroll
            for (int k = 0; k < 3; k++) dl[s2_0][k] = o3[k];
            if (d >= 0 && d <= nr) lD[d & 1][t] = o3[1];
        }

        // ---- corrections averaged back, row e = q - 3
        const int e = q - 3;
        {
            const float *ea = Ea[s2_m1];
            float v[3] = {ea[0], ea[1], ea[2]};
            if constexpr (FF) {
                const bool inner = e < nr, mid = e >= 1 && e < nr;
                v[0] = inner ? ea[0] + 0.5f * (dl[s2_m1][0] + dl[s2_0][0]) : ea[0];
                v[1] = (mid && jlt) ? ea[1] + 0.5f * (dl[s2_m1][1] + lD[e & 1][tr]) : ea[1];
                v[2] = (mid && jin) ? ea[2] + dl[s2_m1][2] : ea[2];
            }
#pragma unroll
            for (int k = 0; k < 3; k++) Ef[s2_m1][k] = v[k];
            if (e >= 0 && e <= nr) {
                lEf[e & 1][0][t] = v[0];
                lEf[e & 1][1][t] = v[2];
            }
        }

        // ---- Faraday half step, absorber, stores: row fr = q - 4
        const int fr = q - 4;
        if (fr >= i0 && fr <= iL) {
            const float4 c0 = rc(fr, 0), c1 = rc(fr, 1), c4 = rc(fr, 4);
            const float *F0 = Ef[s2_0], *F1 = Ef[s2_m1];   // rows fr, fr+1
            const float epn = lEf[fr & 1][1][tr], ern = lEf[fr & 1][0][tr];
            const float *bh = Bh[s4_m4];
            const bool inner = fr < nr;
            float vb[3];
            vb[0] = jlt ? bh[0] - c0.x * cA_j * (sn_j1 * epn - sn_j * F0[2]) : bh[0];
            const float v1 = jin ? bh[1] + c0.y * (c0.w * F1[2] - c0.z * F0[2]) : 0.f;
            const float v2 = jlt ? bh[2] - c0.y * ((c0.w * F1[1] - c0.z * F0[1]) - c1.x * (ern - F0[0]))
                                 : bh[2];
            vb[1] = inner ? v1 : bh[1];
            vb[2] = inner ? v2 : bh[2];
            if constexpr (RB) {
                const float *rb = rbF[s2_0];
                vb[0] += jlt ? h * rb[0] : 0.f;
                vb[1] += (inner && jin) ? h * rb[1] : 0.f;
                vb[2] += (inner && jlt) ? h * rb[2] : 0.f;
            }
            float ve[3] = {F0[0], F0[1], F0[2]};
            const float *E0r = eF[s2_0], *B0r = bF[s2_0];
            float te[3], tb[3];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                te[k] = E0r[k] + ve[k];
                tb[k] = B0r[k] + vb[k];
            }
            if (inner && !jin) tb[1] = 0.f;
            if (fr >= A.absorb0) {
                const float ln = c4.y, lh = c4.z;
                if (!(ln == 1.f && lh == 1.f)) {
                    auto damp_e = [&](int k, float lam) {
                        const float tot = lam * (E0r[k] + ve[k]);
                        ve[k] = tot - E0r[k];
                        te[k] = tot;
                    };
                    auto damp_b = [&](int k, float lam) {
                        vb[k] = lam * vb[k];
                        tb[k] = B0r[k] + vb[k];
                    };
                    if (inner) {
                        damp_e(0, lh);
                        damp_b(1, lh);
                        if (jlt) damp_b(2, lh);
                    }
                    damp_e(2, ln);
                    if (jlt) {
                        damp_e(1, ln);
                        damp_b(0, ln);
                    }
                }
            }
            if (own) {
                const unsigned o = off(fr);
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const unsigned ok = o + k * cs;
                    st32(A.oE, ok, ve[k]);
                    st32(A.oB, ok, vb[k]);
                    st32(A.tE, ok, te[k]);
                    st32(A.tB, ok, tb[k]);
                    st32(A.Jz, ok, 0.f);
                }
            }
        }
        __syncthreads();
    }
};

// LDS of one workgroup of the FP32 field step
template <bool FF>
struct F32Smem {
    float lE[2][4][kFzT];
    float lB[4][4][kFzT];
    float lN[FF ? 2 : 1][kFzT];
    float lF[FF ? 3 : 1][kFzT];
    float lEa[FF ? 2 : 1][kFzT];
    float lD[FF ? 2 : 1][kFzT];
    float lEf[2][2][kFzT];
};

// One strip of columns (bx) over one slab of rows (by).  Every thread of
// the workgroup calls it and returns from it together.
template <bool FF, int RE, bool RB>
__device__ __forceinline__ void field_block(const F32Args &A, const float4 *__restrict__ rowc,
                                            int bx, int by, F32Smem<FF> &L) {
    F32Kernel<FF, RE, RB> K{A, rowc};
    K.nr = A.nr; K.nth = A.nth; K.ld = A.ld;
    K.t = threadIdx.x;
    K.j = bx * kFzW + K.t - kFzL;
    K.jc = (unsigned)min(max(K.j, 0), K.nth);
    K.tl = K.t > 0 ? K.t - 1 : K.t;
    K.tr = K.t < kFzT - 1 ? K.t + 1 : K.t;
    K.i0 = by * A.rows;
    K.iL = min(K.i0 + A.rows - 1, K.nr);
    K.qs = max(K.i0 - 2, 0);
    K.jlt = K.j < K.nth;
    K.jgt = K.j > 0;
    K.jin = K.jgt && K.jlt;
    K.own = K.t >= kFzL && K.t < kFzL + kFzW && K.j >= 0 && K.j <= K.nth;
    const float4 cc0 = A.colc[K.jc * kColC], cc1 = A.colc[K.jc * kColC + 1];
    K.sn_j = cc0.x; K.sn_j1 = cc0.y; K.cA_j = cc0.z; K.sh_j = cc0.w;
    K.sh_jm = cc1.x; K.cdcd_j = cc1.y; K.csh_j = cc1.z; K.cdthd_j = cc1.w;
    K.lE = L.lE; K.lB = L.lB; K.lN = L.lN; K.lF = L.lF; K.lEa = L.lEa; K.lD = L.lD;
    K.lEf = L.lEf;
    // prologue: E^n state and E0 of the first row
    {
        const unsigned o = K.off(K.qs);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            K.sE[0][c] = ld32(A.sE, o + c * A.cs);
            K.e0[0][c] = ld32(A.E0, o + c * A.cs);
        }
    }
    const int qe = K.iL + 4;
    for (int q = K.qs; q <= qe; q += 4) {
        K.template step<0>(q);
        if (q + 1 <= qe) K.template step<1>(q + 1);
        if (q + 2 <= qe) K.template step<2>(q + 2);
        if (q + 3 <= qe) K.template step<3>(q + 3);
    }
}

// RE: bit k set when component k of the background rate curl B0 is
// loaded (the others are zero); RB: the background rate -curl E0 is loaded
template <bool FF, int RE, bool RB>
__global__ void __launch_bounds__(kFzT) k_field_f32(const F32Args A,
                                                    const float4 *__restrict__ rowc) {
    __shared__ F32Smem<FF> L;
    field_block<FF, RE, RB>(A, rowc, (int)blockIdx.x, (int)blockIdx.y, L);
}

// one system's field step in a grouped launch: its arguments, its row
// coefficients and its strips (the slabs are items / strips)
struct F32Job {
    F32Args A;
    const float4 *rowc;
    int strips;
};

// The field steps of many systems in one launch of persistent workgroups,
// which take (system, strip, slab) items from a counter in device memory;
// job k owns items [starts[k], starts[k + 1]).
template <bool FF, int RE, bool RB>
__global__ void __launch_bounds__(kFzT) k_field_f32_group(const F32Job *__restrict__ jobs,
                                                          const int *__restrict__ starts,
                                                          int njobs, int *__restrict__ ctr) {
    __shared__ F32Smem<FF> L;
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
        const F32Job J = stage_uniform(jobs + lo, stage);
        const int local = item - starts[lo];
        const int by = local / J.strips;
        field_block<FF, RE, RB>(J.A, J.rowc, local - by * J.strips, by, L);
        if (threadIdx.x == 0) next = nx;
        __syncthreads();
        item = __builtin_amdgcn_readfirstlane(next);
    }
    group_done(ctr);
}

// row and column coefficient tables of the FP32 step (host, FP64, rounded)
void fused32_tables(const ffpic_ctx *c, std::vector<float> &rowc, std::vector<float> &colc);

using F32Kern = void (*)(const F32Args, const float4 *);
using F32GroupKern = void (*)(const F32Job *, const int *, int, int *);

// kernel instance index: force-free domain on or off; which background
// rates are read (curl B0: only E_phi's, or all three; -curl E0: none or all)
static int f32_key(const ffpic_ctx *c, const F32Args &A) {
    const bool ff = c->d.ff_enable != 0;
    const bool re_all = (A.rates & 3u) != 0, rb = (A.rates >> 3) != 0;
    return (ff ? 4 : 0) + (re_all ? 2 : 0) + (rb ? 1 : 0);
}

static F32Kern f32_kern(int key) {
    switch (key) {
    case 0: return k_field_f32<false, 4, false>;
    case 1: return k_field_f32<false, 4, true>;
    case 2: return k_field_f32<false, 7, false>;
    case 3: return k_field_f32<false, 7, true>;
    case 4: return k_field_f32<true, 4, false>;
    case 5: return k_field_f32<true, 4, true>;
    case 6: return k_field_f32<true, 7, false>;
    default: return k_field_f32<true, 7, true>;
    }
}

static F32GroupKern f32_group_kern(int key) {
    switch (key) {
    case 0: return k_field_f32_group<false, 4, false>;
    case 1: return k_field_f32_group<false, 4, true>;
    case 2: return k_field_f32_group<false, 7, false>;
    case 3: return k_field_f32_group<false, 7, true>;
    case 4: return k_field_f32_group<true, 4, false>;
    case 5: return k_field_f32_group<true, 4, true>;
    case 6: return k_field_f32_group<true, 7, false>;
    default: return k_field_f32_group<true, 7, true>;
    }
}

static int occupancy_slots(const void *kern, int threads, int fallback_per_cu) {
    int per_cu = 0, cus = 0, dev = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = fallback_per_cu;
        cus = 256;
    }
    return std::max(1, per_cu) * std::max(1, cus);
}

// the arguments of a context's FP32 field step, and the buffer swaps that
// follow its launch
static F32Args f32_args(ffpic_ctx *c) {
    F32Args A{};
    A.nr = c->nr; A.nth = c->nth; A.ld = c->ld;
    A.absorb0 = c->absorb_row0;
    A.h = (float)(0.5 * c->dt);
    A.dt = (float)c->dt;
    A.fpdt = (float)(4.0 * kPi * c->dt);
    A.cs = (unsigned)c->cstride;
    A.rates = 0;
    for (int k = 0; k < 3; k++) {
        if (!c->rE0_zero[k]) A.rates |= 1u << k;
        if (!c->rB0_zero[k]) A.rates |= 8u << k;
    }
    A.sE = (const float *)c->dE[0]; A.sB = (const float *)c->dB[0];
    A.oE = (float *)c->stAlt[0];    A.oB = (float *)c->stAlt[3];
    A.tE = (float *)c->E[0];        A.tB = (float *)c->B[0];
    A.E0 = (const float *)c->E0[0]; A.B0 = (const float *)c->B0[0];
    A.rE0 = (const float *)c->rE0[0];
    A.rB0 = (const float *)c->rB0[0];
    A.J = (const float *)c->J[0];
    A.Jz = (float *)c->Jalt[0];
    A.rho0 = (const float *)c->rho0;
    A.f = (const float *)c->f;
    A.colc = (const float4 *)c->fz_colc;
    if (c->fused_slots == 0)
        c->fused_slots = occupancy_slots((const void *)f32_kern(f32_key(c, A)), kFzT, 3);
    A.rows = fused_rows(c);
    return A;
}

static void after_field_f32(ffpic_ctx *c) {
    for (int k = 0; k < 3; k++) {
        std::swap(c->dE[k], c->stAlt[k]);
        std::swap(c->dB[k], c->stAlt[3 + k]);
        std::swap(c->J[k], c->Jalt[k]);
    }
}

static void run_field_f32(ffpic_ctx *c) {
    const F32Args A = f32_args(c);
    dim3 grd((c->nth + 1 + kFzW - 1) / kFzW, (c->nr + 1 + A.rows - 1) / A.rows);
    const float4 *rowc = (const float4 *)c->fz_rowc;
    hipLaunchKernelGGL(f32_kern(f32_key(c, A)), grd, dim3(kFzT), 0, c->stream, A, rowc);
    FFPIC_LAUNCH_CHECK();
    after_field_f32(c);
}

}  // namespace ffpic
