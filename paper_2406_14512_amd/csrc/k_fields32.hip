// FP32 instantiation of the field-step kernels (perturbation form about the
// FP64 background); the flux function is still integrated in FP64 (from the
// FP32 B_r) so the force-free / PIC boundary is set at FP64 accuracy.
#include <cstring>

#include "fields_fused32.h"

namespace ffpic {

void fused32_tables(const ffpic_ctx *c, std::vector<float> &rowc, std::vector<float> &colc) {
    const int nr = c->nr, nth = c->nth;
    const auto &T = c->tab;
    const double h = 0.5 * c->dt, dt = c->dt, dth = c->dth, fp = 4.0 * kPi;
    rowc.assign((size_t)(nr + 1) * kRowC * 4, 0.f);
    for (int i = 0; i <= nr; i++) {
        float *r = &rowc[(size_t)i * kRowC * 4];
        const int ii = i == 0 ? 1 : i;
        r[0] = (float)(h / T[T_RN][i]);
        r[2] = (float)T[T_RN][i];
        if (i < nr) {
            r[1] = (float)(h / T[T_DR2N][i]);
            r[3] = (float)T[T_RN][i + 1];
            r[4] = (float)(T[T_DRN][i] / dth);
            r[8] = (float)(dt / T[T_RH][i]);
            r[9] = (float)(fp / T[T_RH2][i]);
            r[11] = (float)T[T_RH][i];
        }
        if (ii < nr) {
            const double v = fp * T[T_DR3H][ii];
            r[5] = (float)(T[T_RH2][ii] / v);
            r[6] = (float)(T[T_RH2][ii - 1] / v);
            r[7] = (float)(T[T_DR2H][ii] / v);
        }
        if (i >= 1 && i < nr) {
            r[10] = (float)(dt / T[T_DR2H][i]);
            r[12] = (float)T[T_RH][i - 1];
            r[13] = (float)(fp / T[T_DR2H][i]);
            r[14] = (float)(T[T_DRH][i] / dth);
            r[15] = (float)(dt * dth / T[T_DR2H][i]);
            r[16] = (float)(fp * dt / T[T_DR3H][i]);
        }
        r[17] = (float)T[T_LAMN][i];
        r[18] = i < nr ? (float)T[T_LAMH][i] : 1.f;
    }
    colc.assign((size_t)(nth + 1) * kColC * 4, 0.f);
    for (int j = 0; j <= nth; j++) {
        float *q = &colc[(size_t)j * kColC * 4];
        q[0] = (float)T[T_SN][j];
        q[1] = (float)T[T_SN][std::min(j + 1, nth)];
        if (j < nth) {
            q[2] = (float)(1.0 / T[T_DCN][j]);
            q[3] = (float)T[T_SH][j];
            q[6] = (float)(1.0 / T[T_SH][j]);
        }
        if (j > 0) q[4] = (float)T[T_SH][j - 1];
        q[5] = (float)(1.0 / T[T_DCD][j]);
        q[7] = (float)(1.0 / T[T_DTHD][j]);
    }
}

void field_step32(ffpic_ctx *c) { run_field_f32(c); }
void psi_mask32(ffpic_ctx *c) { run_psi_mask<float>(c); }

// ---- grouped launches over several FP32 contexts (batches)

size_t field_job_bytes() { return sizeof(F32Job); }

int field_job(ffpic_ctx *c, void *out, int *key) {
    F32Job J;
    J.A = f32_args(c);
    J.rowc = (const float4 *)c->fz_rowc;
    J.strips = (c->nth + 1 + kFzW - 1) / kFzW;
    const int slabs = (c->nr + 1 + J.A.rows - 1) / J.A.rows;
    *key = f32_key(c, J.A);
    std::memcpy(out, &J, sizeof(J));
    after_field_f32(c);
    return J.strips * slabs;
}

int field_group_slots(int key) {
    return occupancy_slots((const void *)f32_group_kern(key), kFzT, 3);
}

void field_group_launch(hipStream_t st, int key, const void *jobs, const int *starts, int njobs,
                        int grid, int *ctr) {
    hipLaunchKernelGGL(f32_group_kern(key), dim3(grid), dim3(kFzT), 0, st,
                       (const F32Job *)jobs, starts, njobs, ctr);
    FFPIC_LAUNCH_CHECK();
}

size_t psi_job_bytes() { return sizeof(PsiJob<float>); }
size_t mask_job_bytes() { return sizeof(MaskJob<float>); }

int psi_job32(const ffpic_ctx *c, void *out) {
    const PsiJob<float> P = psi_job<float>(c);
    std::memcpy(out, &P, sizeof(P));
    return P.blocks;
}

int mask_job32(const ffpic_ctx *c, void *out) {
    const MaskJob<float> M = mask_job<float>(c);
    std::memcpy(out, &M, sizeof(M));
    return c->nr + 1;
}

int psi_group_slots() { return occupancy_slots((const void *)k_psi_group<float>, kPsiCols, 4); }

void psi_group_launch(hipStream_t st, const void *jobs, const int *starts, int njobs, int grid,
                      int *ctr) {
    hipLaunchKernelGGL(k_psi_group<float>, dim3(grid), dim3(kPsiCols), 0, st,
                       (const PsiJob<float> *)jobs, starts, njobs, ctr);
    FFPIC_LAUNCH_CHECK();
}

void mask_group_launch(hipStream_t st, const void *jobs, const int *starts, int njobs, int grid) {
    hipLaunchKernelGGL(k_mask_group<float>, dim3(grid), dim3(256), 0, st,
                       (const MaskJob<float> *)jobs, starts, njobs);
    FFPIC_LAUNCH_CHECK();
}
}  // namespace ffpic
