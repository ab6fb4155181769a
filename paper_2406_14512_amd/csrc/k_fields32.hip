// FP32 instantiation of the field-step kernels (perturbation form about the
// FP64 background); the flux function is still integrated in FP64 (from the
// FP32 B_r) so the force-free / PIC boundary is set at FP64 accuracy.
#include "fields_fused.h"

namespace ffpic {
void field_step32(ffpic_ctx *c) { run_field_fused<float, true>(c); }
void psi_mask32(ffpic_ctx *c) { run_psi_mask<float>(c); }
}  // namespace ffpic
