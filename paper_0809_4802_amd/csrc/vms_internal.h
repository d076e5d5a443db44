// Internal declarations of libvms (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "vms.h"

namespace vms {

constexpr int kBlock = 256;          // threads per workgroup for streaming kernels
constexpr int kRedBlocks = 1024;     // workgroups of the grid-wide reductions
constexpr int kMaxRestart = 128;
constexpr int kDrMax = 33;           // vectors kept by deflated restarting (k <= 32, +1 for a complex pair)
// Deflated restarting: what the host hands the device between two cycles, packed (doubles,
// each block column-major): the basis coefficients P ((m+1) x kk, ld m+1), the kept block of H
// ((kk+1) x kk), its triangle R (kk x kk), Q^T ((kk+1) x (kk+1)) and the free-pressure sums of
// the kept vectors (kk).
constexpr int kDrOffH = (kMaxRestart + 1) * kDrMax;
constexpr int kDrOffR = kDrOffH + (kDrMax + 1) * kDrMax;
constexpr int kDrOffQt = kDrOffR + kDrMax * kDrMax;
constexpr int kDrOffSvs = kDrOffQt + (kDrMax + 1) * (kDrMax + 1);
constexpr int kDrUpload = kDrOffSvs + kDrMax;
#ifndef VMS_DOT_CHUNKS
#define VMS_DOT_CHUNKS 64          // upper bound on the workgroups (partials) per GMRES dot slot
#endif
constexpr int kTileNodes = 64;           // max nodes owned by one assembly tile
constexpr int kTileMaxNodes = 255;       // max nodes staged by one tile (8-bit local numbers)
#ifndef VMS_TILE_BLOCKS_FP64
#define VMS_TILE_BLOCKS_FP64 280
#endif
#ifndef VMS_TILE_BLOCKS_DET
#define VMS_TILE_BLOCKS_DET 64
#endif
#ifndef VMS_TILE_BLOCKS_FP32
#define VMS_TILE_BLOCKS_FP32 870
#endif
#ifndef VMS_LDS_BLOCK_STRIDE
#define VMS_LDS_BLOCK_STRIDE 17
#endif
#ifndef VMS_MIXED_LDS_FP64
#define VMS_MIXED_LDS_FP64 1
#endif
// accumulator type of the staged blocks in the mixed-precision assembly
using MixedAcc = std::conditional_t<VMS_MIXED_LDS_FP64 != 0, double, float>;
constexpr size_t kMixedAccSize = sizeof(MixedAcc);
constexpr int kTileBlocksFP64 = VMS_TILE_BLOCKS_FP64;   // max 4x4 blocks staged in LDS per tile (FP64 values)
constexpr int kTileBlocksFP32 = VMS_TILE_BLOCKS_FP32;
constexpr int kTileBlocksDet = VMS_TILE_BLOCKS_DET;     // blocks per one-wavefront tile (deterministic contexts)   // same for FP32 values (LDS per tile stays under 64 KB)

// Dynamic LDS of a tile: block values (each 4x4 block padded to 17 entries so that the
// lanes of a wave, which update the same entry of different blocks, spread over the LDS
// banks), rhs rows and residual rows.
constexpr int kLdsBlockStride = VMS_LDS_BLOCK_STRIDE;
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline size_t tile_lds_bytes(int64_t nblocks, int64_t nnodes, size_t elt) {
    return align16(nblocks * kLdsBlockStride * elt) + 2 * nnodes * 4 * 8;
}

// Four-wide vector of a precision (one node's dofs, one block row).
template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
    using type = double4;
};
template <>
struct Vec4<float> {
    using type = float4;
};

// Lane exchanges of a double by DPP (two 32-bit moves; no LDS round trip).  CTRL: a
// quad_perm pattern, or 0x140 (row_mirror: lane i <-> 15 - i in a row of 16) and 0x141
// (row_half_mirror: lane i <-> 7 - i in a group of 8).  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the eight lanes of an aligned group (every lane gets it).
__device__ __forceinline__ double group8_sum(double v) {
    v += dpp_mov<0xB1>(v);           // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_mov<0x4E>(v);           // quad_perm [2,3,0,1]: lane ^ 2
    return v + dpp_mov<0x141>(v);    // the other quad of the eight
}

// Sum over the 64 lanes of the wave (every lane gets it): rows of 16 by DPP, then the four
// row sums read back as scalars.  Every lane of the wave must be active.
__device__ __forceinline__ double wave_sum(double v) {
    v = group8_sum(v);
    v += dpp_mov<0x140>(v);          // the other eight of the row
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Device-resident state of one GMRES cycle (Hessenberg matrix, Givens
// rotations, residual estimate).  Updated by single-lane finalisers so that
// the Arnoldi loop never waits for the host.
struct GmresState {
    double H[(kMaxRestart + 1) * kMaxRestart];   // Hessenberg, column-major, ld = kMaxRestart + 1
    double R[(kMaxRestart + 1) * kMaxRestart];   // its Givens-rotated triangle, same layout
    double cs[kMaxRestart];
    double sn[kMaxRestart];
    double g[kMaxRestart + 1];     // rotated right-hand side (final entries)
    double gin[kMaxRestart + 1];   // entry i before rotation i (gin[k] = residual estimate)
    double y[kMaxRestart];
    double scoef[kMaxRestart];     // s = Q^T u_m: second-pass coefficients of a cycle's last vector
    double svs[kMaxRestart + 1];   // free-pressure sum of every final basis vector
    double tol_abs;                // stop when |g[k]| <= tol_abs
    double beta;                   // norm of the cycle's initial residual
    double norm;                   // scratch: a finished reduction
    double kappa;                  // coarse pressure correction: 1 / (sum of free p-p entries), 0 = off
    double su;                     // sum of the free pressure entries of u_j
    double st;                     // sum of the free pressure entries of the correction V y
    double rho;                    // norm of u_j after its second pass
    double cj;                     // q_j . w
    double hh;                     // provisional subdiagonal of column j (norm estimate of u_{j+1})
    int reorth;                    // 0: one Gram-Schmidt pass; otherwise a delayed second pass
    int k;                         // Arnoldi steps completed in this cycle
    int done;                      // 0 while the cycle runs; nonzero once it stopped (converged or
                                   // breakdown), later kernels idle: 1 when the cycle start or the
                                   // tail stopped it, j + 2 when the update launch of step j did
                                   // (its other workgroups still finish step j)
    unsigned counter;              // arrival counter of last-block reductions
    unsigned gen;                  // cycle number (host-assigned) reported with the progress word
    uint64_t* progress;            // host-mapped progress word: gen << 32 | k << 1 | done
    // deflated restarting: the cycle starts with dr_k kept vectors V[0 .. dr_k-1], whose
    // columns of H (rows 0 .. dr_k) and R the host set; dr_qt is Q^T of the QR factors of that
    // (dr_k + 1) x dr_k block (column-major), dr_c the cycle's least-squares right-hand side
    int dr_k;
    double dr_qt[(kDrMax + 1) * (kDrMax + 1)];
    double dr_c[kDrMax + 1];
};
// the host staging of deflated restarting: a GmresState (padded), then the packed upload
constexpr size_t kDrStateBytes = (sizeof(GmresState) + 255) & ~size_t(255);
constexpr size_t kDrStagingBytes = kDrStateBytes + sizeof(double) * kDrUpload;

// Grid-wide reduction scratch.
struct RedScratch {
    double partial[kRedBlocks * (kMaxRestart + 1)];
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
    int32_t n_pressure_pins = 0;     // Dirichlet pressure dofs (the coarse pressure mode needs one)

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
    // assembly tiles: tile t owns the block rows of a contiguous node range and stages the nodes
    // its elements touch (owned ones first) in LDS; it works through its items, one per
    // (element e, owned vertex a), in the vertex order a, a^1, a^2, a^3: items = (e, four 8-bit
    // local node numbers, four 16-bit tile-local block slots of the owned row; bit 15 of the
    // first slot marks a = 0)
    int32_t n_tiles = 0;
    int4* tile_meta = nullptr;       // [n_tiles][2]: (first node, end node, first block, blocks),
                                     // (first item, end item, first staged node, staged nodes)
    int32_t* tile_nodes = nullptr;   // [staged nodes of all tiles]
    uint4* items = nullptr;          // [4 n_elems]
    uint16_t* bmask = nullptr;       // [nb] Dirichlet bits of the column node (0..3) and the row
                                     // node (4..7), bit 8 on diagonal blocks
    double* tile_part = nullptr;     // [n_tiles][2] partial sums of the residual norm
    int32_t tile_threads = 256;      // threads per assembly tile (64: deterministic context)
    size_t tile_lds = 0;             // dynamic LDS bytes of the largest tile (steady)
    size_t tile_lds_tr = 0;          // same with the previous velocity staged (transient)

    // Newton workspaces (device)
    void* A = nullptr;               // [nb][16] of the ctx precision
    double* rhs = nullptr;           // [4 n_nodes]
    double* du = nullptr;            // [4 n_nodes]
    double* rnorm = nullptr;         // [4] device scalars
    int32_t* flags = nullptr;        // [8] device flags: [2] singular preconditioner blocks, [3] non-finite
                                     // learned blocks; [4..7] the two 64-bit element flags (element.hip)
    uint32_t elem_gen = 0;           // call number of the element flags (advanced by each element launch)

    // Krylov workspaces (device); T = double (FP64 ctx) or float (mixed)
    void* V = nullptr;               // [(max_restart + 1)][4 n_nodes]
    void* w = nullptr;               // [4 n_nodes]
    void* z = nullptr;               // [4 n_nodes]
    void* d = nullptr;               // [4 n_nodes] correction accumulated by a solve
    void* r = nullptr;               // [4 n_nodes] inner residual
    void* Minv = nullptr;            // [n_nodes][16] preconditioner blocks
    void* AP = nullptr;              // [nb][16] A P: each block times the preconditioner block of its column
    void* Az = nullptr;              // [4 n_nodes] A z, z = 1 on every free pressure dof
    double* x64 = nullptr;           // [4 n_nodes] the iterate before a deflated GMRES cycle
    // mixed context, GMRES with an FP64 basis: its basis, w and z (allocated on first use)
    double* V64 = nullptr;           // [(max_restart + 1)][4 n_nodes]
    double* w64 = nullptr;
    double* z64 = nullptr;
    double* r64 = nullptr;           // [4 n_nodes]
    vms::GmresState* gs = nullptr;
    vms::RedScratch* red = nullptr;
    // progress of the running GMRES cycle, written by the device into pinned host memory so
    // that the host can follow it without synchronising the stream
    uint64_t* progress_host = nullptr;
    uint64_t* progress_dev = nullptr;
    // GMRES norms the host reads after a stream synchronisation (the true residual, the inner
    // residual, the right-hand side), written by the device into the same pinned allocation,
    // 64 bytes after the progress word: no copy kernel per read
    double* scal_host = nullptr;
    double* scal_dev = nullptr;
    uint64_t scal_seq = 0;               // tag of the last norm launched (words 1 .. 3 of the progress page)
    uint32_t cycle_gen = 0;
    std::vector<int64_t> cycle_timed;    // timed launches of the cycle: (step, slot, generation)
    // a full restart cycle's Arnoldi steps recorded once as a graph (replayed with one launch)
    hipStream_t cap_stream = nullptr;    // stream the graph is captured on
    hipGraphExec_t cycle_exec = nullptr;
    int cycle_exec_m = 0;                // restart length of cycle_exec, times 2, + 1 for an FP64 basis
    // graphs of deflated cycles (steps j0 .. m-1), keyed by (m, j0)
    hipGraphExec_t dr_exec[4] = {nullptr, nullptr, nullptr, nullptr};
    int dr_exec_key[4] = {0, 0, 0, 0};
    double* dr_p = nullptr;              // [kDrUpload] device copy of the packed upload
    void* dr_pinned = nullptr;           // pinned host [kDrStagingBytes]: a GmresState read back
                                         // (kDrStateBytes), then the packed upload
    int dr_k_dev = 0;                    // the dr_k last written to the device state
    int64_t prof_cycles = 0;             // cycles seen while the phase timers are on
    bool prof_force = false;             // a sampled cycle: every launch of a timed phase is timed

    // uncondensed system (vms_create_opts.full_system): a solver-only child context over the
    // n_nodes + n_elems block rows (its n_nodes field counts block rows), and the positions of
    // the element contributions in its pattern
    vms_ctx* full = nullptr;
    int32_t* full_cc = nullptr;      // [nb] position of condensed-pattern block k in the full pattern
    int32_t* full_epos = nullptr;    // [n_elems][9]: (node a, elem) a = 0..3, (elem, node b) b = 0..3, (elem, elem)
    int32_t linearization = VMS_LIN_NEWTON;   // tangent of the element kernels (vms_set_linearization)
    int32_t full_nodes = 0;          // in the child: number of node block rows (0 in other contexts)
    double* zfull = nullptr;         // in the child: [4 n_nodes] coarse vector (free pressures + fine response)

    // learned preconditioner (device, float)
    float* feats = nullptr;          // [n_nodes][25]
    float* hid = nullptr;            // [n_nodes][64]
    float* pblk = nullptr;           // [n_nodes][16]
    float* gblk = nullptr;           // [n_nodes][16] D^-1 blocks (features, training)
    float* gdel = nullptr;           // [n_nodes][16] dL/dDelta (training)
    float* tvec = nullptr;           // [3][4 n_nodes] training vectors
    float* wgrad = nullptr;          // [kRedBlocks][VMS_PC_NWEIGHTS] partial weight gradients
    float* fscal = nullptr;          // [8] float scalars

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::string err;

    // phase timers
    uint32_t prof_mask = 0;                // phases being timed
    int32_t prof_every = 1;                // time every n-th launch of a phase
    int64_t prof_seen[VMS_NPHASES] = {};   // launches seen per phase
    int64_t prof_gen = 0;                  // pending-slot generation (bumped by each flush)
    std::vector<hipEvent_t> prof_ev;       // pairs
    std::vector<int> prof_phase;           // pending slot -> phase
    std::vector<double> prof_bytes;        // pending slot -> algorithmic bytes
    int prof_used = 0;
    double prof_ms[VMS_NPHASES] = {};
    double prof_acc_bytes[VMS_NPHASES] = {};
    int64_t prof_count[VMS_NPHASES] = {};
};

namespace vms {

int set_error(vms_ctx* ctx, int code, const std::string& msg);
int check_hip(vms_ctx* ctx, hipError_t e, const char* what);
inline size_t elt_size(const vms_ctx* c) { return c->prec == VMS_FP64 ? 8 : 4; }
inline unsigned long long* element_flags(vms_ctx* c) { return reinterpret_cast<unsigned long long*>(c->flags + 4); }

// phase timers (ctx.cpp): a scope records an event pair around the launches it encloses
int prof_begin(vms_ctx* c, int phase, double bytes, hipStream_t s);
void prof_end(vms_ctx* c, int slot, hipStream_t s);
// Drops a pending timed launch (one that returned without work) from the accumulators.
void prof_void(vms_ctx* c, int slot, int64_t gen);
struct PhaseScope {
    vms_ctx* c;
    int slot;
    int64_t gen;
    hipStream_t s;
    PhaseScope(vms_ctx* c_, int phase, double bytes, hipStream_t s_) : c(c_), slot(-1), gen(0), s(s_) {
        if ((c->prof_mask >> phase) & 1u) {
            slot = prof_begin(c, phase, bytes, s);
            gen = c->prof_gen;
        }
    }
    ~PhaseScope() {
        if (slot >= 0) prof_end(c, slot, s);
    }
};

// element kernels (element.hip)
hipError_t tile_kernels_configure(vms_ctx* ctx);
// rglob (may be null) receives the assembled residual rows; every launch leaves the norm's
// partial sums per tile in ctx->tile_part, which launch_norm_finalize adds into out.
int launch_condense(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                    double nu, double inv_dt, const double* body, void* A, double* rhs,
                    double* rglob, hipStream_t s);
int launch_residual(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta,
                    double nu, double inv_dt, const double* body, double* rglob, hipStream_t s);
int launch_norm_finalize(vms_ctx* ctx, double* out, hipStream_t s);
int check_element_flags(vms_ctx* ctx, hipStream_t s);
// Resolves this device's address of the no-allocation entry point's static scratch (once per
// device; called by vms_create with the context's device current).
int noalloc_scratch_init(vms_ctx* ctx);
// Uncondensed system (ctx->full must exist): assembly into vals / rhs of the full pattern, and
// the Newton update from its solution dx.
int launch_full_assemble(vms_ctx* ctx, const double* u, const double* u_prev, const double* beta, double nu,
                         double inv_dt, const double* body, void* vals, double* rhs, hipStream_t s);
int launch_full_update(vms_ctx* ctx, const double* dx, double* u, double* beta, hipStream_t s);

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
