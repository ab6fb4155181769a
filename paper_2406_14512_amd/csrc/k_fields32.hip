// FP32 instantiation of the field-step kernels; the flux function is still
// integrated in FP64 (from the FP32 B_r) so the force-free / PIC boundary
// is set at FP64 accuracy.
#include "fields_impl.h"

namespace ffpic {
void field_step32(ffpic_ctx *c) { run_field_step<float>(c); }
void psi_mask32(ffpic_ctx *c) { run_psi_mask<float>(c); }
}  // namespace ffpic
