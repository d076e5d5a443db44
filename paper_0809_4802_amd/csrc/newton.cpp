// One Newton-Schur iteration (Sections 4.2 and 5): condensed tangent and
// residual assembled into the context's matrix, linear solve of the condensed
// system, element-level recovery of the fine scales, update of (vbar, p, v').
#include "vms_internal.h"

using namespace vms;

extern "C" int vms_newton_step(vms_ctx* c, double* u, double* beta, const double* u_prev, double Re, double dt,
                               const double* body, const vms_newton_opts* opts, vms_newton_info* info,
                               hipStream_t s) {
    if (!c) return set_error(nullptr, VMS_EINVAL, "vms_newton_step: NULL ctx");
    if (!u || !beta || !opts) return set_error(c, VMS_EINVAL, "vms_newton_step: NULL argument");
    if (!(Re > 0.0)) return set_error(c, VMS_EINVAL, "vms_newton_step: Re must be > 0");
    if (dt > 0.0 && !u_prev) return set_error(c, VMS_EINVAL, "vms_newton_step: dt > 0 needs u_prev");
    vms_newton_info inf{};
    inf.bad_elem = -1;
    const double nu = 1.0 / Re;
    const double inv_dt = dt > 0.0 ? 1.0 / dt : 0.0;
    const double* up = dt > 0.0 ? u_prev : nullptr;
    const int n = 4 * c->n_nodes;

    int rc = launch_condense(c, u, up, beta, nu, inv_dt, body, c->A, c->rhs, nullptr, s);
    if (rc) return rc;
    if ((rc = launch_norm_finalize(c, c->rnorm, s))) return rc;
    if ((rc = check_hip(c, hipMemcpyAsync(&inf.rnorm_before, c->rnorm, sizeof(double), hipMemcpyDeviceToHost, s),
                        "read rnorm")))
        return rc;
    if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
    // a non-finite state is reported as such (its K_ff also fails the singularity test)
    if (!std::isfinite(inf.rnorm_before)) {
        if (info) *info = inf;
        return set_error(c, VMS_ENONFINITE, "vms_newton_step: non-finite residual");
    }
    if ((rc = check_element_flags(c, s))) {
        if (info) *info = inf;
        return rc;
    }

    if ((rc = launch_fill(c->du, n * sizeof(double), s))) return rc;
    const int lin = gmres_solve(c, c->A, c->rhs, c->du, &opts->lin, &inf.lin, s);
    if (lin != VMS_OK) {
        if (info) *info = inf;
        return lin;
    }
    if ((rc = vms_recover_update(c, u, beta, u_prev, Re, dt, body, c->du, s))) return rc;
    if ((rc = launch_residual(c, u, up, beta, nu, inv_dt, body, nullptr, s))) return rc;
    if ((rc = launch_norm_finalize(c, c->rnorm + 1, s))) return rc;
    if ((rc = check_hip(c, hipMemcpyAsync(&inf.rnorm_after, c->rnorm + 1, sizeof(double), hipMemcpyDeviceToHost, s),
                        "read rnorm")))
        return rc;
    if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
    if ((rc = check_element_flags(c, s))) {
        if (info) *info = inf;
        return rc;
    }
    if (info) *info = inf;
    if (!std::isfinite(inf.rnorm_after)) return set_error(c, VMS_ENONFINITE, "vms_newton_step: non-finite residual");
    return VMS_OK;
}

// One Newton-Raphson iteration on the uncondensed system (Section 4.2, Eq. NewtonUpdate2):
// coarse and fine unknowns in one global system, solved by the same GMRES on the context's
// uncondensed pattern (block-Jacobi), then u and beta updated from the solution.
extern "C" int vms_full_newton_step(vms_ctx* c, double* u, double* beta, const double* u_prev, double Re,
                                    double dt, const double* body, const vms_newton_opts* opts,
                                    vms_newton_info* info, hipStream_t s) {
    if (!c) return set_error(nullptr, VMS_EINVAL, "vms_full_newton_step: NULL ctx");
    if (!u || !beta || !opts) return set_error(c, VMS_EINVAL, "vms_full_newton_step: NULL argument");
    if (!c->full) return set_error(c, VMS_EINVAL, "vms_full_newton_step: context created without full_system");
    if (!(Re > 0.0)) return set_error(c, VMS_EINVAL, "vms_full_newton_step: Re must be > 0");
    if (dt > 0.0 && !u_prev) return set_error(c, VMS_EINVAL, "vms_full_newton_step: dt > 0 needs u_prev");
    vms_newton_info inf{};
    inf.bad_elem = -1;
    const double nu = 1.0 / Re;
    const double inv_dt = dt > 0.0 ? 1.0 / dt : 0.0;
    const double* up = dt > 0.0 ? u_prev : nullptr;
    vms_ctx* f = c->full;
    const int n = 4 * f->n_nodes;

    int rc = launch_full_assemble(c, u, up, beta, nu, inv_dt, body, f->A, f->rhs, s);
    if (rc) return rc;
    if ((rc = launch_norm_finalize(c, c->rnorm, s))) return rc;
    if ((rc = check_hip(c, hipMemcpyAsync(&inf.rnorm_before, c->rnorm, sizeof(double), hipMemcpyDeviceToHost, s),
                        "read rnorm")))
        return rc;
    if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
    if (!std::isfinite(inf.rnorm_before)) {
        if (info) *info = inf;
        return set_error(c, VMS_ENONFINITE, "vms_full_newton_step: non-finite residual");
    }
    if ((rc = check_element_flags(c, s))) {
        if (info) *info = inf;
        return rc;
    }
    if ((rc = launch_fill(f->du, n * sizeof(double), s))) return rc;
    vms_solve_opts lin = opts->lin;
    lin.pc = VMS_PC_BLOCK_JACOBI;           // the learned correction is trained on condensed blocks
    lin.pc_weights = nullptr;
    lin.deflate = 0;                        // deflated restarting is not built for the uncondensed system
    lin.basis_fp64 = 0;                     // nor the FP64 basis of a mixed context
    lin.log_residuals = nullptr;
    lin.log_max = 0;
    const int lrc = gmres_solve(f, f->A, f->rhs, f->du, &lin, &inf.lin, s);   // not phase-timed
    if (lrc != VMS_OK) {
        c->err = f->err;
        if (info) *info = inf;
        return lrc;
    }
    if ((rc = launch_full_update(c, f->du, u, beta, s))) return rc;
    if ((rc = launch_residual(c, u, up, beta, nu, inv_dt, body, nullptr, s))) return rc;
    if ((rc = launch_norm_finalize(c, c->rnorm + 1, s))) return rc;
    if ((rc = check_hip(c, hipMemcpyAsync(&inf.rnorm_after, c->rnorm + 1, sizeof(double), hipMemcpyDeviceToHost, s),
                        "read rnorm")))
        return rc;
    if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
    if ((rc = check_element_flags(c, s))) {
        if (info) *info = inf;
        return rc;
    }
    if (info) *info = inf;
    if (!std::isfinite(inf.rnorm_after))
        return set_error(c, VMS_ENONFINITE, "vms_full_newton_step: non-finite residual");
    return VMS_OK;
}
