// FP64 instantiation of the flux-function, mask and field-step kernels.
// Compiled without FP contraction: every product and sum is rounded as
// written, like the plain FP64 definition of the step.
#include "fields_fused.h"

namespace ffpic {
void field_step64(ffpic_ctx *c) { run_field_fused64(c); }
void psi_mask64(ffpic_ctx *c) { run_psi_mask<double>(c); }
}  // namespace ffpic
