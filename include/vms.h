/*
 * vms.h -- C ABI of the MI355X (gfx950) variational multiscale Newton-Schur
 * library (libvms.so).
 *
 * The method (Turner, Nakshatrala & Hjelmstad, "A variational multiscale
 * Newton-Schur approach for the incompressible Navier-Stokes equations"):
 * equal-order linear tetrahedra for velocity and pressure plus one bubble
 * per element for the fine-scale velocity (Section 3.3); element residuals
 * R_c, R_p, R_f (Section 4.1) and their consistent Newton tangent
 * (Section 4.2, the 3x3-block update system); element-level block Gauss
 * elimination of the fine scales, assembly of the condensed 2x2-block system
 * and fine-scale recovery (Section 5); a Krylov solve of the condensed system
 * (Section 6).
 *
 * Conventions shared by every call
 *   - Arrays are DEVICE pointers owned by the caller unless stated; the
 *     library never frees them.  Host-side structs are read during the call.
 *   - Coarse unknowns per node are (vx, vy, vz, p); global coarse dof
 *     4*node + c.  Element dof order: (v0x,v0y,v0z,p0, ..., v3x,v3y,v3z,p3,
 *     beta_x, beta_y, beta_z).
 *   - nu = 1/Re; the viscous term carries 2*nu as written in the paper's
 *     momentum equation and weak form (Sections 2, 3.2).
 *   - dt <= 0 means steady; otherwise backward Euler from u_prev (Section 4.1
 *     Remark): the coarse rows get the consistent-mass term, the fine rows
 *     the bubble-weighted term of the coarse velocity (quasi-static fine scales).
 *   - Newton sign convention: K * Delta = -R.
 *   - Every call enqueues on `stream` (NULL = default stream) and returns an
 *     int status; calls documented as synchronising wait for the stream.
 *   - No call allocates device or pinned host memory except vms_create (the
 *     HIP runtime objects behind the GMRES cycle graphs aside: the capture
 *     stream and the executable graphs that vms_gmres_solve creates on first
 *     use of a restart length and keeps until vms_destroy).
 *   - Errors: negative status; vms_last_error() describes the last one.
 *     Nothing aborts the process (the paper's code aborted on solver
 *     failure, Section 6; this library returns VMS_ENOCONV_* instead).
 */
#ifndef VMS_H
#define VMS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VMS_OK = 0,
    VMS_EINVAL = -1,           /* bad argument (null pointer, size, option)         */
    VMS_EDEGENERATE = -2,      /* an element with det J <= 0 (index in info)        */
    VMS_ESINGULAR_KFF = -3,    /* fine-scale block K_ff numerically singular        */
    VMS_ENOCONV_GMRES = -4,    /* Krylov solve hit max_iters before rtol            */
    VMS_ENOCONV_NEWTON = -5,   /* reserved for drivers                              */
    VMS_ENONFINITE = -6,       /* NaN/Inf in a residual or norm                     */
    VMS_EHIP = -7,             /* HIP runtime error                                 */
    VMS_ENOMEM = -8            /* device allocation failed in vms_create            */
};

typedef struct vms_ctx vms_ctx;

typedef enum { VMS_FP64 = 0, VMS_MIXED = 1 } vms_precision;
typedef enum { VMS_PC_BLOCK_JACOBI = 0, VMS_PC_LEARNED = 1 } vms_pc_kind;
typedef enum { VMS_LIN_NEWTON = 0, VMS_LIN_PICARD = 1 } vms_linearization;

/* Mesh, read once by vms_create (the library keeps its own copies).
 *   xyz   device double [n_nodes][3]
 *   tets  device int32  [n_elems][4], positively oriented linear tets
 *   dirichlet_dofs  device int32 [n_dirichlet], dof = 4*node + c; the
 *         increment of these dofs is zero (their values live in u).       */
typedef struct {
    int32_t n_nodes;
    int32_t n_elems;
    const double* xyz;
    const int32_t* tets;
    int32_t n_dirichlet;
    const int32_t* dirichlet_dofs;
} vms_mesh_desc;

typedef struct {
    vms_precision precision;   /* VMS_FP64: FP64 everywhere.  VMS_MIXED: FP32
                                  tangent blocks, block-CSR values and inner
                                  GMRES; FP64 K_ff^-1, residuals, refinement. */
    int32_t max_restart;       /* Krylov basis allocated (<= 0: 50)          */
    int32_t full_system;       /* 1: also build the uncondensed system used by
                                  vms_full_assemble / vms_full_newton_step   */
    int32_t deterministic;     /* 1: assembly tiles of one wavefront, whose
                                  staged sums are then formed in one fixed
                                  order: every assembly (and every solve on
                                  it) is bitwise reproducible from run to run
                                  on the same device and build, at about 1.3x
                                  the assembly time.  0: tiles of 256
                                  threads, whose LDS additions interleave in
                                  an order that varies from run to run
                                  (results agree to rounding)               */
    int32_t basis_fp64;        /* VMS_MIXED: 1 also allocates an FP64 Krylov
                                  basis ((max_restart + 3) vectors of
                                  4 n_nodes doubles) for solves with
                                  vms_solve_opts.basis_fp64.  Ignored for
                                  VMS_FP64 (its basis is FP64 already)       */
} vms_create_opts;

/* Builds the 4x4 block-CSR pattern of the condensed system (one block per
 * node pair sharing an element), the element-to-block map and every
 * workspace.  Synchronising.  opts may be NULL (FP64, restart 50). */
int vms_create(const vms_mesh_desc* mesh, const vms_create_opts* opts, hipStream_t stream,
               vms_ctx** out);
int vms_destroy(vms_ctx* ctx);
const char* vms_last_error(const vms_ctx* ctx);   /* ctx may be NULL */

/* Read-only device views of the block pattern: rowptr [n_nodes+1],
 * colidx [nb] (sorted per row), diagpos [n_nodes] (block index of (i,i)).
 * Any pointer argument may be NULL. */
int vms_bsr_info(const vms_ctx* ctx, int64_t* nb, const int32_t** rowptr,
                 const int32_t** colidx, const int32_t** diagpos, int32_t* precision);

/* Uncondensed element residual and tangent (Sections 4.1-4.2).
 *   u      double [n_nodes][4];  u_prev double [n_nodes][4] or NULL (steady)
 *   beta   double [n_elems][3] fine-scale coefficients
 *   body   double [n_nodes][3] P1 nodal body force, or NULL
 *   Ke     double [n_elems][19][19] row-major (mixed ctx: computed in FP32
 *          for the tangent blocks, FP64 for K_ff, widened on output)
 *   Rvec   double [n_elems][19]
 * Ke or Rvec may be NULL.  Not synchronising. */
int vms_element_tangents(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                         double Re, double dt, const double* body, double* Ke, double* Rvec,
                         hipStream_t stream);

/* Condensed tangent and residual, assembled (Section 5):
 *   K* = K_cc - K_cf K_ff^-1 K_fc,  R* = R_cp - K_cf K_ff^-1 R_f  per element,
 *   summed into bsr_vals (FP64 ctx: double, mixed ctx: float) [nb][16]
 *   (4x4 blocks row-major) and rhs = -R* (double [n_nodes][4]).
 * Rows and columns of Dirichlet dofs are replaced by the identity and their
 * rhs by 0.  rnorm (device double[1], may be NULL) receives the FP64 Newton
 * residual norm ||[R_c; R_p] (assembled, free dofs), R_f (all elements)||_2
 * at the input state.  Not synchronising, so a singular K_ff is not reported
 * here (the condensed blocks of that element are then meaningless); vms_newton_step reports it
 * (VMS_ESINGULAR_KFF, the first such element in vms_last_error). */
int vms_condense_assemble(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                          double Re, double dt, const double* body, void* bsr_vals, double* rhs,
                          double* rnorm, hipStream_t stream);

/* The same call for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * identical inputs and outputs, but the scratch the call needs (element
 * error flags and the per-tile partial sums of rnorm) lives in a static
 * device array of the library, 1 MiB + 256 B per GPU, held until the process
 * ends, instead of the context's buffers.  Nothing is allocated or freed and
 * no library routine that allocates is called.  Limit: contexts of at most
 * 65,536 assembly tiles (about 18 million block rows' worth of elements);
 * larger ones get VMS_EINVAL.  Every call on one GPU shares that GPU's
 * array (its contents are rewritten by each call): calls that overlap on one
 * GPU, from any stream, thread or context, race and must be serialised by
 * the caller.  Not synchronising. */
int vms_condense_assemble_noalloc(vms_ctx* ctx, const double* u, const double* u_prev,
                                  const double* beta, double Re, double dt, const double* body,
                                  void* bsr_vals, double* rhs, double* rnorm, hipStream_t stream);

/* FP64 Newton residual norm only (same definition as above); rglob
 * (double [n_nodes][4], may be NULL) receives the assembled [R_c; R_p].
 * Not synchronising. */
int vms_residual(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                 double Re, double dt, const double* body, double* rglob, double* rnorm,
                 hipStream_t stream);

/* Fine-scale recovery and Newton update (Section 5; Section 4.2 update):
 *   dbeta_e = K_ff^-1 (-R_f - K_fc du_e)  at the input state, then
 *   beta += dbeta, u += du (du is zeroed on Dirichlet dofs first).
 * du double [n_nodes][4].  u and beta are updated in place.  Not synchronising. */
int vms_recover_update(vms_ctx* ctx, double* u, double* beta, const double* u_prev, double Re,
                       double dt, const double* body, const double* du, hipStream_t stream);

/* y = A x with the context's block pattern.  FP64 ctx: double A, x, y.
 * Mixed ctx: float A, x, y with FP32 accumulation.  Not synchronising. */
int vms_bsr_spmv(vms_ctx* ctx, const void* bsr_vals, const void* x, void* y, hipStream_t stream);

typedef struct {
    int32_t restart;           /* Krylov dimension m (<= max_restart)                    */
    int32_t max_iters;         /* total Arnoldi steps over all cycles and refinements    */
    double rtol;               /* success iff ||b - A x||_2 <= rtol ||b||_2 (true residual) */
    vms_pc_kind pc;
    const float* pc_weights;   /* device, VMS_PC_LEARNED only (layout in vms_pc_*)       */
    int32_t refine_max;        /* mixed ctx with inner_rtol > 0: FP64 iterative-refinement
                                  sweeps (<= 0: 30)                                        */
    double inner_rtol;         /* mixed ctx.  <= 0 (default): every FP32 restart cycle starts
                                  from the FP64 residual b - A x (FP32-stored A, FP64 x and
                                  arithmetic) scaled to unit norm, and its correction is added
                                  to the FP64 x; each cycle is one refinement sweep.
                                  > 0: a sweep runs FP32 cycles, restarted from the FP32
                                  residual of the FP32 correction, until that residual falls
                                  below inner_rtol (relative to the sweep's residual), or a
                                  cycle's own estimate reached it but the recomputed residual
                                  did not (the FP32 rounding floor); then x is refined in FP64 */
    int32_t cgs2;              /* nonzero: every basis vector gets a second classical
                                  Gram-Schmidt pass, delayed into the next Arnoldi step so
                                  that each step needs one reduction; 0: one pass (each
                                  vector's norm is still measured, not estimated)          */
    int32_t coarse_pressure;   /* 1: add the coarse correction on the constant pressure
                                  mode, P v = M v + z (z^T v) / (z^T A z), z = 1 on every
                                  free pressure dof.  With one pinned pressure dof that mode
                                  is nearly singular and restarted GMRES stalls on it.
                                  Without any prescribed pressure dof (open or traction-free
                                  boundaries) the mode does not exist and the option has no
                                  effect.                                                  */
    float* log_residuals;      /* device float [log_max][n_nodes][4] or NULL: the true
                                  residual b - A x at the start of every restart cycle
                                  (refinement sweep in the mixed ctx) is copied here, as
                                  training samples for the learned preconditioner          */
    int32_t log_max;
    int32_t deflate;           /* deflated restarting (GMRES-DR, Morgan 2002): a cycle that
                                  follows a full one keeps the harmonic Ritz vectors of its
                                  predecessor's `deflate` harmonic Ritz values of smallest
                                  modulus (one more to keep a complex pair whole), restarts
                                  from the true residual and adds restart - kept Arnoldi
                                  steps; a cycle after one that stopped early restarts
                                  plainly.  0 = plain restarts.  1 <= deflate <= 32 and
                                  deflate <= restart - 2, else VMS_EINVAL; so is deflate with
                                  inner_rtol > 0 (mixed ctx) or on the uncondensed system.
                                  Turns cgs2 on.  The kept block's eigenproblem is solved on
                                  the host between cycles (O(restart^3) flops).  With an
                                  FP32 basis (mixed ctx without basis_fp64) the kept block
                                  drifts from the stored vectors over many cycles; see
                                  vms_solve_info.deflation_stopped.                         */
    int32_t basis_fp64;        /* mixed ctx: nonzero runs GMRES with an FP64 Krylov basis
                                  and FP64 vector arithmetic on the FP32-stored matrix and
                                  preconditioner, applied one after the other at every step
                                  (so that the Arnoldi operator is exactly the one the FP64
                                  residual sees); every cycle starts from the FP64 residual
                                  (inner_rtol and refine_max are not used).  Needs a ctx
                                  created with vms_create_opts.basis_fp64 (VMS_EINVAL
                                  otherwise).  No effect on an FP64 ctx.                    */
} vms_solve_opts;

typedef struct {
    int32_t iters;             /* Arnoldi steps                                          */
    int32_t restarts;          /* cycles                                                 */
    int32_t refinements;       /* FP64 refinement sweeps (mixed; with inner_rtol <= 0 one
                                  per cycle)                                               */
    int32_t fell_back_to_bj;   /* learned preconditioner rejected: non-finite blocks, or
                                  no convergence within half of max_iters (the solve then
                                  continues from its iterate with plain block-Jacobi)     */
    double true_rel_res;       /* final ||b - A x|| / ||b|| recomputed in FP64           */
    int32_t logged;            /* residuals written to log_residuals                      */
    int32_t singular_blocks;   /* node diagonal blocks found numerically singular by the last
                                  preconditioner setup; each is applied as the identity (the
                                  true residual still decides convergence)                */
    int32_t deflation_stopped; /* deflate > 0: 1 if a deflated cycle raised the true
                                  residual (or made it non-finite); its correction was
                                  undone and the solve went on with plain restarts        */
} vms_solve_info;

/* Right-preconditioned restarted GMRES(m) on A x = b (Section 6 names a
 * Krylov solver with tolerance and iteration cap; the method and the
 * preconditioner are this library's: 4x4 block-Jacobi or its learned
 * correction).  bsr_vals as in vms_condense_assemble; b, x double [n_nodes][4]
 * (x is the initial guess on entry).  Mixed ctx: FP64 iterative refinement
 * around FP32 GMRES.  Synchronising.  Returns VMS_ENOCONV_GMRES when the true
 * residual misses rtol within max_iters (x then holds the best iterate). */
int vms_gmres_solve(vms_ctx* ctx, const void* bsr_vals, const double* b, double* x,
                    const vms_solve_opts* opts, vms_solve_info* info, hipStream_t stream);

typedef struct {
    vms_solve_opts lin;
} vms_newton_opts;

typedef struct {
    double rnorm_before;       /* FP64 residual norm at the input state                  */
    double rnorm_after;        /* FP64 residual norm after the update                    */
    vms_solve_info lin;
    int32_t bad_elem;          /* first degenerate element, or -1                         */
} vms_newton_info;

/* One Newton-Schur iteration (Sections 4.2 and 5): condense and assemble
 * into the context's own matrix, set up the preconditioner, solve, recover
 * the fine scales, update u and beta in place, evaluate the new residual.
 * Synchronising. */
int vms_newton_step(vms_ctx* ctx, double* u, double* beta, const double* u_prev, double Re,
                    double dt, const double* body, const vms_newton_opts* opts,
                    vms_newton_info* info, hipStream_t stream);

/* ---- uncondensed Newton-Raphson (the baseline the paper compares against) --
 * Section 4.2 states the full Newton system over the coarse and fine unknowns
 * together (Eq. NewtonUpdate2); Section 5 condenses it.  These calls solve it
 * without condensation.  The system is a 4x4 block-CSR system over
 * n_nodes + n_elems block rows: block row i < n_nodes holds the dofs
 * (vx, vy, vz, p) of node i; block row n_nodes + e holds the three fine dofs
 * (beta_x, beta_y, beta_z) of element e and one unused slot (identity row and
 * column, zero rhs).  Blocks: node-node (K_cc summed over elements),
 * node-element (K_cf, fourth column 0), element-node (K_fc, fourth row 0) and
 * the element diagonal (K_ff, unit fourth diagonal).  Dirichlet rows and
 * columns are replaced by the identity.  Needs vms_create_opts.full_system. */

/* Read-only device views of the uncondensed pattern (see vms_bsr_info). */
int vms_full_info(const vms_ctx* ctx, int64_t* nb, int32_t* n_rows, const int32_t** rowptr,
                  const int32_t** colidx);

/* Uncondensed tangent into bsr_vals (FP64 ctx: double, mixed ctx: float)
 * [nb][16], rhs = -R (double [n_nodes + n_elems][4]), rnorm as in
 * vms_condense_assemble.  Not synchronising. */
int vms_full_assemble(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                      double Re, double dt, const double* body, void* bsr_vals, double* rhs,
                      double* rnorm, hipStream_t stream);

/* One Newton-Raphson iteration on the uncondensed system: assemble, solve with
 * the context's GMRES, update u and beta in place, evaluate the new residual.
 * Preconditioner: block-diagonal on the block rows above, the inverse of the
 * Schur complement's diagonal block K_cc(i,i) - sum_e K_cf(i,e) K_ff(e)^-1 K_fc(e,i)
 * on node rows (the plain node block has a zero pressure diagonal) and K_ff^-1
 * on element rows, plus the constant-pressure coarse correction with the
 * fine-scale response of the pressure mode; opts->lin.pc is ignored (the
 * learned correction is trained on condensed blocks).  Synchronising. */
int vms_full_newton_step(vms_ctx* ctx, double* u, double* beta, const double* u_prev, double Re,
                         double dt, const double* body, const vms_newton_opts* opts,
                         vms_newton_info* info, hipStream_t stream);

/* ---- learned block-Jacobi correction ------------------------------------
 * Per node i: features x_i (25 floats) from the condensed tangent,
 *   [ D_i/||D_i||_F (16), log||D_i||_F, log(1 + sum_{j!=i} ||A_ij[r,:]||_1/|D_i[r,r]|) (4),
 *     Dirichlet flags of the node's 4 dofs (4) ];
 * MLP h = tanh(W1 x + b1) (64), y = W2 h + b2 (16) = Delta_i (4x4 row-major),
 * Delta_i zeroed on the rows and columns of Dirichlet dofs,
 * P_i = D_i^-1 (I + Delta_i).  Weights (float, VMS_PC_NWEIGHTS) packed as
 * [W1 64x25 row-major, b1 64, W2 16x64, b2 16]. */
#define VMS_PC_NIN 25
#define VMS_PC_NHID 64
#define VMS_PC_NOUT 16
#define VMS_PC_NWEIGHTS (VMS_PC_NHID * VMS_PC_NIN + VMS_PC_NHID + VMS_PC_NOUT * VMS_PC_NHID + VMS_PC_NOUT)

/* feats float [n_nodes][25].  Not synchronising. */
int vms_pc_features(vms_ctx* ctx, const void* bsr_vals, float* feats, hipStream_t stream);

/* Preconditioner blocks P float [n_nodes][16] (weights NULL: plain
 * block-Jacobi D_i^-1).  Not synchronising. */
int vms_pc_blocks(vms_ctx* ctx, const void* bsr_vals, const float* weights, float* P,
                  hipStream_t stream);

/* One training step on a batch of residual samples r_batch float
 * [nbatch][n_nodes][4]:
 *   loss = mean_s ||r_s - A P r_s||^2 / ||r_s||^2, gradient by the library's
 *   backward kernels, then Adam (beta1 0.9, beta2 0.999, eps 1e-8) on
 *   weights in place.  adam_state float [2][VMS_PC_NWEIGHTS] (m, v; zero
 *   before the first step); step = 1, 2, ... (bias correction).
 *   grad_out (float [VMS_PC_NWEIGHTS], may be NULL) receives the gradient;
 *   loss_out (device float[1], may be NULL) the loss before the update.
 *   lr <= 0 computes loss and gradient without updating.
 * Not synchronising. */
int vms_pc_train_step(vms_ctx* ctx, const void* bsr_vals, const float* r_batch, int32_t nbatch,
                      float* weights, float* adam_state, int32_t step, float lr,
                      float* grad_out, float* loss_out, hipStream_t stream);

/* ---- phase timers ----------------------------------------------------------
 * While enabled, every launch of a hot kernel is bracketed by two hipEvents
 * on its stream, and the algorithmic bytes the launch must move (inputs read
 * once, outputs written once; no credit for scratch, atomics or re-reads)
 * are added to its phase.  Each timed launch costs two event records on the
 * stream, which lengthens the step around it. */
enum {
    VMS_PH_CONDENSE = 0,       /* element residual + tangent + condensation + scatter kernel */
    VMS_PH_RESIDUAL = 1,       /* residual-only element kernel                            */
    VMS_PH_RECOVER = 2,        /* fine-scale recovery kernel                              */
    VMS_PH_PCSETUP = 3,        /* preconditioner block setup                              */
    VMS_PH_PCAPPLY = 4,        /* A P formed once per solve (the Arnoldi SpMV applies P);
                                  with basis_fp64 on a mixed ctx, P applied at every step  */
    VMS_PH_SPMV = 5,           /* block-CSR SpMV with A P in the Arnoldi step             */
    VMS_PH_DOTS = 6,           /* Gram-Schmidt dot products (Q^T u, Q^T w, norms)         */
    VMS_PH_UPDATE = 7,         /* Gram-Schmidt update (q_j and the next vector), with the
                                  step's sums of the dot partials and the Hessenberg
                                  columns and Givens rotations in one of its workgroups     */
    VMS_PH_FILL = 8,           /* zero fill of the assembled outputs                      */
    VMS_NPHASES = 9
};
/* phase_mask: bit p enables phase p (VMS_PROFILE_ALL: every phase), 0 disables.
 * every >= 1: only every every-th launch of an enabled phase is timed (a sample;
 * the accumulators then cover the sampled launches only).  A full GMRES restart
 * cycle is replayed from a recorded HIP graph, and events cannot time launches
 * inside a graph: there the sample is every every-th cycle, launched directly,
 * with each of its launches of an enabled phase timed (the environment variable
 * VMS_CYCLE_GRAPHS=0 turns the graphs off).  Each call clears the accumulators.
 * Timing one phase, sparsely, keeps the event cost off the rest. */
#define VMS_PROFILE_ALL ((1u << VMS_NPHASES) - 1u)
int vms_profile(vms_ctx* ctx, uint32_t phase_mask, int32_t every);
/* Synchronising.  Each array has VMS_NPHASES entries; any may be NULL. */
int vms_profile_read(vms_ctx* ctx, double* ms, int64_t* launches, double* alg_bytes);

/* ---- linearisation ----------------------------------------------------------
 * The paper linearises consistently (Newton-Raphson, Section 4.2) and, in its
 * introduction, contrasts this with fixed-point iteration, which holds the
 * advecting velocity of (v . grad) v at the current iterate.  VMS_LIN_PICARD
 * switches every tangent this context forms (vms_element_tangents,
 * vms_condense_assemble, vms_newton_step, the recovery, the uncondensed path)
 * to that fixed-point tangent: the terms from the derivative of the advecting
 * coarse and fine velocity are dropped, everything else is unchanged.  The
 * residual is the same, so a converged solve reaches the same solution, at a
 * linear instead of a quadratic rate.  Default VMS_LIN_NEWTON.  Not
 * synchronising; VMS_EINVAL for another value. */
int vms_set_linearization(vms_ctx* ctx, int kind);

#ifdef __cplusplus
}
#endif
#endif /* VMS_H */
