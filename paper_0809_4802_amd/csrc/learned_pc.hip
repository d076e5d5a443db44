// Learned correction of the 4x4 block-Jacobi preconditioner (FP32 kernels).
//
// The paper leaves the Krylov preconditioner open (Section 6).  Per node i a
// two-layer perceptron maps 25 features of the condensed tangent's block row
// to a 4x4 correction Delta_i, and the preconditioner block becomes
// P_i = D_i^-1 (I + Delta_i) with Delta_i masked on Dirichlet rows/columns.
// With a zero output layer this is exactly block-Jacobi.  Training minimises
// mean_s ||r_s - A P r_s||^2 / ||r_s||^2 over residual samples produced by the
// method's own GMRES solves, with hand-written forward, backward (through
// A^T via the transposed-block map) and Adam kernels.
#include "vms_internal.h"

namespace vms {

int learned_blocks(vms_ctx* c, const void*, const float*, void*, int, hipStream_t) {
    return set_error(c, VMS_EINVAL, "learned preconditioner not available in this build");
}

}  // namespace vms

using namespace vms;

extern "C" int vms_pc_features(vms_ctx* c, const void*, float*, hipStream_t) {
    return set_error(c, VMS_EINVAL, "vms_pc_features: not available in this build");
}

extern "C" int vms_pc_blocks(vms_ctx* c, const void*, const float*, float*, hipStream_t) {
    return set_error(c, VMS_EINVAL, "vms_pc_blocks: not available in this build");
}

extern "C" int vms_pc_train_step(vms_ctx* c, const void*, const float*, int32_t, float*, float*, int32_t, float,
                                 float*, float*, hipStream_t) {
    return set_error(c, VMS_EINVAL, "vms_pc_train_step: not available in this build");
}
