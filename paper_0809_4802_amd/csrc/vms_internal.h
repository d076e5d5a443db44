// Internal declarations of libvms (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "vms.h"

namespace vms {

constexpr int kBlock = 256;          // threads per workgroup for streaming kernels
constexpr int kRedBlocks = 1024;     // workgroups of the grid-wide reductions
constexpr int kMaxRestart = 128;

// Device-resident state of one GMRES cycle (Hessenberg matrix, Givens
// rotations, residual estimate).  Updated by single-lane finalisers so that
// the Arnoldi loop never waits for the host.
struct GmresState {
    double H[(kMaxRestart + 1) * kMaxRestart];   // Hessenberg, column-major, ld = kMaxRestart + 1
    double R[(kMaxRestart + 1) * kMaxRestart];   // its Givens-rotated triangle, same layout
    double cs[kMaxRestart];
    double sn[kMaxRestart];
    double g[kMaxRestart + 1];
    double y[kMaxRestart];
    double hcol[kMaxRestart + 1];  // CGS coefficients of the current step
    double tol_abs;                // stop when |g[k]| <= tol_abs
    double beta;                   // norm of the cycle's initial residual
    double norm;                   // scratch: a finished reduction
    int k;                         // Arnoldi steps completed in this cycle
    int done;                      // 1: converged or breakdown, later kernels idle
    unsigned counter;              // arrival counter of last-block reductions
};

// Grid-wide reduction scratch.
struct RedScratch {
    double partial[kRedBlocks * (kMaxRestart + 1)];
    double acc_slots[64 * 8];      // atomically accumulated scalars, one per 64-byte line
    unsigned counter;
};

}  // namespace vms

struct vms_ctx {
    int device = 0;
    int32_t n_nodes = 0;
    int32_t n_elems = 0;
    int64_t nb = 0;
    vms_precision prec = VMS_FP64;
    int32_t max_restart = 50;
    int32_t n_dir = 0;

    // mesh (device, library-owned copies)
    double4* xyz4 = nullptr;         // [n_nodes] (x, y, z, 0)
    int4* tets = nullptr;            // [n_elems]
    uint8_t* dmask = nullptr;        // [n_nodes] bit c set: dof 4i+c is Dirichlet
    int32_t* dlist = nullptr;        // [n_dir] Dirichlet dofs

    // block pattern (device)
    int32_t* rowptr = nullptr;       // [n_nodes + 1]
    int32_t* colidx = nullptr;       // [nb]
    int32_t* diagpos = nullptr;      // [n_nodes]
    int32_t* tpos = nullptr;         // [nb] position of the transposed block
    int32_t* epos = nullptr;         // [16][n_elems] block of local pair (a, b), SoA

    // Newton workspaces (device)
    void* A = nullptr;               // [nb][16] of the ctx precision
    double* rhs = nullptr;           // [4 n_nodes]
    double* du = nullptr;            // [4 n_nodes]
    double* rglob = nullptr;         // [4 n_nodes]
    double* rnorm = nullptr;         // [4] device scalars
    int32_t* flags = nullptr;        // [4] device error flags (bad element, singular K_ff)

    // Krylov workspaces (device); T = double (FP64 ctx) or float (mixed)
    void* V = nullptr;               // [(max_restart + 1)][4 n_nodes]
    void* w = nullptr;               // [4 n_nodes]
    void* z = nullptr;               // [4 n_nodes]
    void* d = nullptr;               // [4 n_nodes] correction accumulated by a solve
    void* r = nullptr;               // [4 n_nodes] inner residual
    void* Minv = nullptr;            // [n_nodes][16] preconditioner blocks
    double* x64 = nullptr;           // [4 n_nodes]
    double* r64 = nullptr;           // [4 n_nodes]
    vms::GmresState* gs = nullptr;
    vms::RedScratch* red = nullptr;

    // learned preconditioner (device, float)
    float* feats = nullptr;          // [n_nodes][25]
    float* hid = nullptr;            // [n_nodes][64]
    float* pblk = nullptr;           // [n_nodes][16]
    float* gblk = nullptr;           // [n_nodes][16] dL/dDelta
    float* tvec = nullptr;           // [3][4 n_nodes] training vectors
    float* wgrad = nullptr;          // [kRedBlocks][VMS_PC_NWEIGHTS] partial weight gradients
    float* fscal = nullptr;          // [8] float scalars

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::string err;
};

namespace vms {

int set_error(vms_ctx* ctx, int code, const std::string& msg);
int check_hip(vms_ctx* ctx, hipError_t e, const char* what);
inline size_t elt_size(const vms_ctx* c) { return c->prec == VMS_FP64 ? 8 : 4; }

// element kernels (element.hip)
int launch_condense(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                    double nu, double inv_dt, const double* body, void* A, double* rhs,
                    double* rglob, double* red_acc, hipStream_t s);
int launch_residual(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                    double nu, double inv_dt, const double* body, double* rglob, double* red_acc,
                    hipStream_t s);
int launch_norm_finalize(vms_ctx* ctx, const double* rglob, const double* red_acc, double* out,
                         hipStream_t s);
int check_element_flags(vms_ctx* ctx, hipStream_t s);

// linear algebra (krylov.hip)
int launch_fill(void* p, size_t bytes, hipStream_t s);
int launch_spmv(vms_ctx* ctx, const void* A, const void* x, void* y, hipStream_t s);
int launch_bj_setup(vms_ctx* ctx, const void* A, void* Minv, hipStream_t s);
int gmres_solve(vms_ctx* ctx, const void* A, const double* b, double* x,
                const vms_solve_opts* opts, vms_solve_info* info, hipStream_t s);

// learned preconditioner (learned_pc.hip)
int learned_blocks(vms_ctx* ctx, const void* A, const float* weights, void* Minv_out,
                   int out_is_double, hipStream_t s);

}  // namespace vms
