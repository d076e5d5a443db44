// Condensed-system linear algebra on gfx950: 4x4 block-CSR SpMV, block
// preconditioners and restarted GMRES(m).
//
// The paper solves each Newton system with a Krylov method at tolerance 1e-12
// and a 50-iteration cap and aborts on failure (Section 6); the method and the
// preconditioner are left to PETSc defaults.  This library uses right-
// preconditioned restarted GMRES with 4x4 block-Jacobi (or its learned
// correction), judges success by the true residual ||b - A x|| recomputed at
// every restart, and reports failure instead of aborting.
//
// GPU layout: all vectors are node-interleaved (4 n_nodes entries, dofs
// (vx, vy, vz, p) of a node adjacent) so that a 4x4 block multiplies one
// 32-byte (FP64) or 16-byte (FP32) segment.  The Hessenberg matrix, the Givens
// rotations and the residual estimate live in device memory and are updated
// by single-workgroup reduction kernels, so an Arnoldi step is a fixed
// sequence of launches with no host round trip; the host looks at the
// convergence flag only every few steps.
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <vector>

#include "deflate.h"
#include "vms_internal.h"

namespace vms {
namespace {

inline int grid_for(int64_t n, int block = kBlock) { return (int)((n + block - 1) / block); }

// Workgroups are dispatched to the 8 XCDs round-robin by linear id, and each XCD has its own
// L2, which keeps its lines across kernel boundaries.  The Arnoldi kernels (SpMV, dots, update)
// give XCD k the k-th eighth of the rows, so that the slices of a vector one of them writes
// and the next one reads (and most SpMV gathers, the mesh being numbered brick by brick) stay
// in the same XCD's L2: slot of workgroup b in a grid of g (a multiple of 8).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_slot(int b, int g) { return (b % kXcds) * (g / kXcds) + b / kXcds; }
inline int xcd_round(int g) { return (g + kXcds - 1) / kXcds * kXcds; }

__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


__global__ void fill_kernel(uint4* p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------------- SpMV
// Eight lanes per block row.  Lane (q, r), q = 0, 1 and r = 0..3, owns output dof r and the
// row's blocks q, q + 2, q + 4, ...: it reads row r of each (4 contiguous values) and the
// 4-vector of the column node.  The first kSpmvUnroll blocks of a lane are all loaded before
// any is used, so that its loads are in flight together (a row of this mesh has at most 15
// blocks, i.e. 8 per lane); the two halves of a row are summed with one lane exchange.
// MODE 0: y = A x.  MODE 1: y = b - A x.  MODE 2: y = A x + (kappa S) b with kappa and S (the
// coarse pressure scale and the free-pressure sum of x) taken from the GMRES state.  Grids of at
// most kSpmvXcdMaxGrid workgroups (about one round of residency) take their rows through
// xcd_slot; larger ones keep the linear order, in which the whole chip streams one window of
// the matrix (measured at 64^3: 53.9 us linear, 56.5 us mapped; at 32^3 8.5 and 8.3 us).
constexpr int kSpmvLanes = 8;
constexpr int kSpmvXcdMaxGrid = 2048;
constexpr int kSpmvUnroll = 8;

// Component I of a quad's four values (lane r of the quad holds component r): a DPP quad_perm
// broadcast.  Every lane of the quad must be active.
template <int I>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), I * 0x55, 0xF, 0xF, false));
}
template <int I>
__device__ __forceinline__ double quad_bcast(double v) {
    return dpp_mov<I * 0x55>(v);
}

// The four lanes of a block row need the same 4-vector x of the block's column: each loads one
// component and the quad exchanges them by DPP, so that x is requested once per quad instead
// of four times (as many bytes as the matrix block otherwise).  The four lanes share the row
// and the block sequence, so a quad is active or inactive as a whole.
template <typename TA, typename TX, typename TY, typename TACC, int MODE, typename TB = double>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int n_rows, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const TA* __restrict__ A, const TX* __restrict__ x,
                                                      const TB* __restrict__ b, TY* __restrict__ y,
                                                      const int* __restrict__ done, const GmresState* gs) {
    // a finished GMRES cycle (done != NULL and set) reads no blocks and stores nothing; the
    // flag is read alongside the row bounds, which the block loads wait for anyway
    const int skip = done ? *done : 0;
    constexpr int Q = kSpmvLanes / 4;
    using VA = typename Vec4<TA>::type;
    const int slot = gridDim.x <= kSpmvXcdMaxGrid ? xcd_slot(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tid = slot * blockDim.x + threadIdx.x;
    const int row = tid / kSpmvLanes, sub = tid % kSpmvLanes;
    const int q = sub >> 2, r = sub & 3;
    TACC acc = TACC(0);
    if (row < n_rows) {
        const int k0 = rowptr[row], k1 = skip ? k0 : rowptr[row + 1];
        int cols[kSpmvUnroll];
#pragma unroll
        for (int u = 0; u < kSpmvUnroll; ++u) {
            const int k = k0 + q + u * Q;
            cols[u] = k < k1 ? colidx[k] : -1;
        }
        VA av[kSpmvUnroll];
        TX xr[kSpmvUnroll];
#pragma unroll
        for (int u = 0; u < kSpmvUnroll; ++u) {
            if (cols[u] >= 0) {
                av[u] = *reinterpret_cast<const VA*>(A + (size_t)(k0 + q + u * Q) * 16 + r * 4);
                xr[u] = x[(size_t)cols[u] * 4 + r];
            } else {
                av[u] = VA{TA(0), TA(0), TA(0), TA(0)};
                xr[u] = TX(0);
            }
        }
#pragma unroll
        for (int u = 0; u < kSpmvUnroll; ++u) {
            const TX x0 = quad_bcast<0>(xr[u]), x1 = quad_bcast<1>(xr[u]), x2 = quad_bcast<2>(xr[u]),
                     x3 = quad_bcast<3>(xr[u]);
            acc += TACC(av[u].x) * TACC(x0) + TACC(av[u].y) * TACC(x1) + TACC(av[u].z) * TACC(x2) +
                   TACC(av[u].w) * TACC(x3);
        }
        // rows longer than kSpmvUnroll blocks per lane (other meshes)
        for (int k = k0 + q + kSpmvUnroll * Q; k < k1; k += Q) {
            const VA a = *reinterpret_cast<const VA*>(A + (size_t)k * 16 + r * 4);
            const TX xc = x[(size_t)colidx[k] * 4 + r];
            const TX x0 = quad_bcast<0>(xc), x1 = quad_bcast<1>(xc), x2 = quad_bcast<2>(xc), x3 = quad_bcast<3>(xc);
            acc += TACC(a.x) * TACC(x0) + TACC(a.y) * TACC(x1) + TACC(a.z) * TACC(x2) + TACC(a.w) * TACC(x3);
        }
    }
    acc += __shfl_xor(acc, 4, 64);       // lanes 4q + r of a row: q = 0 and q = 1
    if (row < n_rows && q == 0 && !skip) {
        if (MODE == 1)
            y[4 * (size_t)row + r] = TY(TACC(b[4 * (size_t)row + r]) - acc);
        else if (MODE == 2)
            y[4 * (size_t)row + r] = TY(acc + TACC(gs->kappa * gs->su) * TACC(b[4 * (size_t)row + r]));
        else
            y[4 * (size_t)row + r] = TY(acc);
    }
}

inline int spmv_grid(int n_rows) { return xcd_round((int)(((int64_t)kSpmvLanes * n_rows + kBlock - 1) / kBlock)); }

// --------------------------------------------------------------------------- block-Jacobi
// Inverse of each 4x4 diagonal block in FP64 (Gauss-Jordan, partial pivoting),
// stored in the preconditioner precision.  A singular block is replaced by the
// identity and counted in flags[2].
// Inverts the FP64 4x4 block D into out (precision TM); a singular block becomes the
// identity and is counted in flags[2].
template <typename TM>
__device__ void invert_block_store(const double (&D)[4][4], TM* __restrict__ out, int32_t* flags) {
    double m[4][8];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            m[r][c] = D[r][c];
            m[r][4 + c] = (r == c) ? 1.0 : 0.0;
        }
    bool ok = true;
#pragma unroll
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        double best = fabs(m[col][col]);
#pragma unroll
        for (int r = col + 1; r < 4; ++r)
            if (fabs(m[r][col]) > best) {
                best = fabs(m[r][col]);
                piv = r;
            }
        if (!(best > 0.0)) {
            ok = false;
            break;
        }
        if (piv != col) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const double t = m[col][c];
                m[col][c] = m[piv][c];
                m[piv][c] = t;
            }
        }
        const double ip = 1.0 / m[col][col];
#pragma unroll
        for (int c = 0; c < 8; ++c) m[col][c] *= ip;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == col) continue;
            const double f = m[r][col];
#pragma unroll
            for (int c = 0; c < 8; ++c) m[r][c] -= f * m[col][c];
        }
    }
    if (!ok) atomicAdd(&flags[2], 1);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) out[r * 4 + c] = ok ? TM(m[r][4 + c]) : TM(r == c ? 1 : 0);
}

template <typename TA, typename TM>
__global__ void bj_setup_kernel(int n, const int32_t* __restrict__ diagpos, const TA* __restrict__ A,
                                TM* __restrict__ Minv, int32_t* flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const TA* Dp = A + (size_t)diagpos[i] * 16;
    double D[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) D[r][c] = double(Dp[r * 4 + c]);
    invert_block_store<TM>(D, Minv + (size_t)i * 16, flags);
}

// Uncondensed system (node rows 0..nn, element rows after them; each element row holds the
// element's K_fc blocks, its K_ff block padded to 4x4 and nothing else).  The node diagonal
// blocks of that system have a zero pressure-pressure entry, so their plain inverse is no
// preconditioner.  Node row i instead gets the inverse of the diagonal block of the Schur
// complement, K_cc(i,i) - sum_e K_cf(i,e) K_ff(e)^-1 K_fc(e,i) (Section 5), formed from the
// assembled blocks and the element rows' inverses already in Minv.
template <typename TA, typename TM>
__global__ void schur_diag_pc_kernel(int nn, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                     const int32_t* __restrict__ diagpos, const TA* __restrict__ A,
                                     TM* __restrict__ Minv, int32_t* flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    double D[4][4];
    {
        const TA* Dp = A + (size_t)diagpos[i] * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) D[r][c] = double(Dp[r * 4 + c]);
    }
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int e = colidx[k];
        if (e < nn) continue;
        int kf = -1;                                   // block (e, i) in element row e
        for (int q = rowptr[e]; q < rowptr[e + 1]; ++q)
            if (colidx[q] == i) kf = q;
        if (kf < 0) continue;
        const TA* Cf = A + (size_t)k * 16;
        const TA* Fc = A + (size_t)kf * 16;
        const TM* P = Minv + (size_t)e * 16;
        double W[4][4];                                // K_ff^-1 K_fc (padded)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) t += double(P[r * 4 + q]) * double(Fc[q * 4 + c]);
                W[r][c] = t;
            }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) t += double(Cf[r * 4 + q]) * W[q][c];
                D[r][c] -= t;
            }
    }
    invert_block_store<TM>(D, Minv + (size_t)i * 16, flags);
}

// ------------------------------------------------------------------------ reductions
// Block-level sum of NV values per thread into s[0..NV) (result valid in thread 0).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[w * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double t = 0.0;
            for (int ww = 0; ww < kBlock / 64; ++ww) t += lds[ww * NV + q];
            v[q] = t;
        }
    }
}

// Last-arriving workgroup detection (partials written before the fence).
__device__ __forceinline__ bool arrive_last(unsigned* counter) {
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    return last;
}

// Inside the last-arriving workgroup: out[i] = sum_k part[i * ld + k], k < nk, for i < nvec.
// Threads form groups of P lanes (P a power of two, P <= 64) per vector; each lane sums a
// fixed stride of partials and the group combines them with shuffles (fixed order).
__device__ void reduce_partials(const double* part, int ld, int nvec, int nk, double* out) {
    int P = 64;
    while (P > 1 && P * nvec > (int)blockDim.x) P >>= 1;
    const int i = threadIdx.x / P, lane = threadIdx.x % P;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < nvec) {
        const double* pi = part + (size_t)i * ld;
        int k = lane;
        for (; k + 3 * P < nk; k += 4 * P) {
            s0 += ld_agent(pi + k);
            s1 += ld_agent(pi + k + P);
            s2 += ld_agent(pi + k + 2 * P);
            s3 += ld_agent(pi + k + 3 * P);
        }
        for (; k < nk; k += P) s0 += ld_agent(pi + k);
    }
    double sum = (s0 + s1) + (s2 + s3);
    for (int off = P / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (i < nvec && lane == 0) out[i] = sum;
}

// dof idx is a pressure dof without a Dirichlet condition
__device__ __forceinline__ bool free_pressure(const uint8_t* __restrict__ dmask, int idx) {
    return (idx & 3) == 3 && !(dmask[idx >> 2] & 8u);
}

// Coarse correction on the constant pressure mode: kappa = 1 / sum of the entries of A
// that couple two free pressure dofs (= 1 / (z^T A z) for z = 1 on the free pressure dofs).
// That sum is the Galerkin coarse operator of the mode.  It is only meaningful when the mode
// is nearly singular because one pressure dof is pinned: there the sum is the coupling to the
// pinned dof, about 1 / (2 n_nodes) of the summed magnitudes.  Without a pin (open or
// traction-free boundaries) the pressure-pressure block annihilates constants and the sum is
// rounding noise: the caller then passes enabled = 0 (the noise of FP32-stored entries can
// exceed any fixed fraction of the magnitudes, and kappa = 1 / noise would swamp the Krylov
// space).  As a guard, the correction is also off when |sum| <= 1e-8 x the summed magnitudes.
template <typename TA>
__global__ __launch_bounds__(kBlock) void coarse_setup_kernel(int n_nodes, const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ colidx,
                                                              const TA* __restrict__ A,
                                                              const uint8_t* __restrict__ dmask, int enabled,
                                                              RedScratch* red, GmresState* gs) {
    __shared__ double lds[(kBlock / 64) * 2];
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes; i += gridDim.x * blockDim.x) {
        if (dmask[i] & 8u) continue;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (!(dmask[colidx[k]] & 8u)) {
                const double a = double(A[(size_t)k * 16 + 15]);
                v[0] += a;
                v[1] += fabs(a);
            }
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        red->partial[blockIdx.x] = v[0];
        red->partial[kRedBlocks + blockIdx.x] = v[1];
    }
    if (!arrive_last(&red->counter)) return;
    __threadfence();
    __shared__ double tot[2];
    reduce_partials(red->partial, kRedBlocks, 2, gridDim.x, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool usable = isfinite(tot[0]) && fabs(tot[0]) > 1e-8 * tot[1];
        gs->kappa = (enabled && usable) ? 1.0 / tot[0] : 0.0;
        red->counter = 0u;
    }
}

// Coarse vector of the uncondensed system: 1 on the free node pressures and, on each element
// row, the fine response -K_ff^-1 K_fc 1_p (K_fc columns of prescribed dofs are zero).  The
// response vanishes up to rounding unless the element touches a pinned pressure (the
// gradients of an element sum to zero); with it, 1_p^T A z equals the Schur complement's
// 1_p^T S 1_p, which the plain indicator (zero pressure-pressure block) would miss.
template <typename TA, typename TM>
__global__ void full_coarse_vector_kernel(int nn, int n_rows, const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ colidx, const TA* __restrict__ A,
                                          const TM* __restrict__ Minv, const uint8_t* __restrict__ dmask,
                                          double* __restrict__ zvec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    double* zi = zvec + 4 * (size_t)i;
    if (i < nn) {
        zi[0] = zi[1] = zi[2] = 0.0;
        zi[3] = (dmask[i] & 8u) ? 0.0 : 1.0;
        return;
    }
    double t[3] = {0.0, 0.0, 0.0};
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int b = colidx[k];
        if (b >= nn || (dmask[b] & 8u)) continue;
#pragma unroll
        for (int q = 0; q < 3; ++q) t[q] += double(A[(size_t)k * 16 + 4 * q + 3]);
    }
    const TM* P = Minv + (size_t)i * 16;
#pragma unroll
    for (int r = 0; r < 3; ++r)
        zi[r] = -(double(P[4 * r]) * t[0] + double(P[4 * r + 1]) * t[1] + double(P[4 * r + 2]) * t[2]);
    zi[3] = 0.0;
}

// kappa = 1 / (1_p^T A z) for the explicit coarse vector z, switched off (as for the condensed
// system) when the sum is below 1e-8 x the summed magnitudes of the free pressure rows' terms.
template <typename TA>
__global__ __launch_bounds__(kBlock) void full_coarse_setup_kernel(int nn, const int32_t* __restrict__ rowptr,
                                                                   const int32_t* __restrict__ colidx,
                                                                   const TA* __restrict__ A,
                                                                   const uint8_t* __restrict__ dmask,
                                                                   const double* __restrict__ zvec, int enabled,
                                                                   RedScratch* red, GmresState* gs) {
    __shared__ double lds[(kBlock / 64) * 2];
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += gridDim.x * blockDim.x) {
        if (dmask[i] & 8u) continue;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const double* zc = zvec + 4 * (size_t)colidx[k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double a = double(A[(size_t)k * 16 + 12 + q]);
                v[0] += a * zc[q];
                v[1] += fabs(a * zc[q]);
            }
        }
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        red->partial[blockIdx.x] = v[0];
        red->partial[kRedBlocks + blockIdx.x] = v[1];
    }
    if (!arrive_last(&red->counter)) return;
    __threadfence();
    __shared__ double tot[2];
    reduce_partials(red->partial, kRedBlocks, 2, gridDim.x, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool usable = isfinite(tot[0]) && fabs(tot[0]) > 1e-8 * tot[1];
        gs->kappa = (enabled && usable) ? 1.0 / tot[0] : 0.0;
        red->counter = 0u;
    }
}

// Publishes the cycle's progress (completed columns k, done flag) to the host-mapped word.
__device__ __forceinline__ void report_progress(uint64_t* progress, unsigned gen, int k, int done) {
    const uint64_t word = ((uint64_t)gen << 32) | ((uint64_t)k << 1) | (uint64_t)(done ? 1 : 0);
    __hip_atomic_store(progress, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void report_progress(GmresState* gs, int k, int done) {
    report_progress(gs->progress, gs->gen, k, done);
}

// norm of a vector -> gs->beta, initialises the cycle (g = beta e_1, k = 0, done flag).
template <typename T>
__global__ __launch_bounds__(kBlock) void cycle_start_kernel(int n, const T* __restrict__ r,
                                                             const uint8_t* __restrict__ dmask, RedScratch* red,
                                                             GmresState* gs, double tol_abs, int reorth,
                                                             unsigned gen) {
    __shared__ double lds[(kBlock / 64) * 2];
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double x = double(r[i]);
        v[0] += x * x;
        if (free_pressure(dmask, i)) v[1] += x;
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        red->partial[blockIdx.x] = v[0];
        red->partial[kRedBlocks + blockIdx.x] = v[1];
    }
    __shared__ double tot[2];
    const bool last = arrive_last(&red->counter);
    if (last) {
        __threadfence();
        reduce_partials(red->partial, kRedBlocks, 2, gridDim.x, tot);
        __syncthreads();
    }
    if (last && threadIdx.x == 0) {
        const double nrm = sqrt(tot[0]);
        gs->su = nrm > 0.0 ? tot[1] / nrm : 0.0;
        gs->beta = nrm;
        gs->g[0] = nrm;
        gs->gin[0] = nrm;
        gs->k = 0;
        gs->tol_abs = tol_abs;
        gs->done = (nrm <= tol_abs || !(nrm > 0.0)) ? 1 : 0;
        gs->norm = nrm;
        gs->reorth = reorth;
        gs->gen = gen;
        red->counter = 0u;
        report_progress(gs, 0, gs->done);
    }
}

// Deflated restarting: V[c] = sum_l P(l, c) V[l] for the kept columns c < kk (l < mv), in
// place -- each thread owns one entry of every vector and reads all of them before it writes.
// P is staged in LDS (every thread reads the same entry: a broadcast); KMAX >= kk bounds the
// accumulators.
template <typename T, int KMAX>
__global__ __launch_bounds__(kBlock) void dr_basis_kernel(int n, int mv, int kk, const double* __restrict__ P,
                                                          int ldp, T* __restrict__ V) {
    __shared__ double Pl[(kMaxRestart + 1) * KMAX];     // Pl[l KMAX + c]
    for (int e = threadIdx.x; e < mv * KMAX; e += blockDim.x) {
        const int l = e / KMAX, c = e % KMAX;
        Pl[e] = c < kk ? P[(size_t)c * ldp + l] : 0.0;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t N = (size_t)n;
    double acc[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (int l = 0; l < mv; ++l) {
        const double v = double(V[(size_t)l * N + i]);
#pragma unroll
        for (int c = 0; c < KMAX; ++c) acc[c] += Pl[l * KMAX + c] * v;
    }
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
        if (c < kk) V[(size_t)c * N + i] = T(acc[c]);
}

template <typename T>
void launch_dr_basis(int n, int mv, int kk, const double* P, int ldp, T* V, hipStream_t s) {
    if (kk <= 12)
        dr_basis_kernel<T, 12><<<grid_for(n), kBlock, 0, s>>>(n, mv, kk, P, ldp, V);
    else if (kk <= 20)
        dr_basis_kernel<T, 20><<<grid_for(n), kBlock, 0, s>>>(n, mv, kk, P, ldp, V);
    else
        dr_basis_kernel<T, kDrMax><<<grid_for(n), kBlock, 0, s>>>(n, mv, kk, P, ldp, V);
}

// Deflated restarting: the kept block of H and its factors from the packed upload into the
// cycle state (columns 0 .. kk-1 of H and R, zero below their last row), and dr_k = kk.  kk = 0
// only switches deflation off.  One workgroup.
__global__ __launch_bounds__(kBlock) void dr_load_kernel(int kk, const double* __restrict__ up, GmresState* gs) {
    constexpr int ld = kMaxRestart + 1;
    const int tid = threadIdx.x;
    if (tid == 0) gs->dr_k = kk;
    for (int e = tid; e < kk * ld; e += blockDim.x) {
        const int col = e / ld, row = e % ld;
        gs->H[e] = row <= kk ? up[kDrOffH + col * (kk + 1) + row] : 0.0;
        gs->R[e] = row < kk ? up[kDrOffR + col * kk + row] : 0.0;
    }
    for (int e = tid; e < (kk + 1) * (kk + 1); e += blockDim.x) gs->dr_qt[e] = up[kDrOffQt + e];
    for (int e = tid; e < kk; e += blockDim.x) gs->svs[e] = up[kDrOffSvs + e];
}

// V[0] = r / beta (V0 = V + j0 n for a deflated cycle)
template <typename T>
__global__ void cycle_v0_kernel(int n, const T* __restrict__ r, T* __restrict__ V0, const GmresState* gs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double b = gs->beta;
    V0[i] = b > 0.0 ? T(double(r[i]) / b) : T(0);
}

// A P for the Arnoldi steps: block (i, b) times the preconditioner block of node b, so that
// the step's SpMV applies the preconditioner on the fly.  Four lanes per block, lane r forms
// row r; the product is summed in FP64 and stored in T.
template <typename T>
__global__ void ap_blocks_kernel(int64_t nb, const int32_t* __restrict__ colidx, const T* __restrict__ A,
                                 const T* __restrict__ Minv, T* __restrict__ AP) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t k = tid >> 2;
    const int r = (int)(tid & 3);
    if (k >= nb) return;
    using V4 = typename Vec4<T>::type;
    const V4 a = *reinterpret_cast<const V4*>(A + k * 16 + r * 4);
    const T* M = Minv + (size_t)colidx[k] * 16;
    double o[4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
        o[cc] = double(a.x) * double(M[cc]) + double(a.y) * double(M[4 + cc]) + double(a.z) * double(M[8 + cc]) +
                double(a.w) * double(M[12 + cc]);
    *reinterpret_cast<V4*>(AP + k * 16 + r * 4) = V4{T(o[0]), T(o[1]), T(o[2]), T(o[3])};
}

// A z for z = 1 on every free pressure dof: per row, the sum of the pressure columns of the
// blocks whose column node has a free pressure.  Four lanes per block row.
template <typename T>
__global__ void coarse_column_kernel(int n_rows, const int32_t* __restrict__ rowptr,
                                     const int32_t* __restrict__ colidx, const T* __restrict__ A,
                                     const uint8_t* __restrict__ dmask, T* __restrict__ Az) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = tid >> 2, r = tid & 3;
    if (row >= n_rows) return;
    double acc = 0.0;
    for (int k = rowptr[row]; k < rowptr[row + 1]; ++k)
        if (!(dmask[colidx[k]] & 8u)) acc += double(A[(size_t)k * 16 + r * 4 + 3]);
    Az[4 * (size_t)row + r] = T(acc);
}

// t = P v = Minv v + z kappa S(v), S(v) = gs->su (the free-pressure sum of the step's vector):
// the preconditioner of an Arnoldi step applied on its own, for steps whose matrix is stored
// in a lower precision than the basis (the step then multiplies by A itself, so that its
// operator is exactly A P, the one the FP64 residual and the correction P V y see).  Idle once
// the cycle has stopped.
template <typename TM, typename T>
__global__ void precond_apply_kernel(int n_nodes, const TM* __restrict__ Minv, const T* __restrict__ v,
                                     const uint8_t* __restrict__ dmask, const double* __restrict__ zvec,
                                     const GmresState* gs, T* __restrict__ t) {
    if (gs->done) return;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = tid >> 2, r = tid & 3;
    if (node >= n_nodes) return;
    using M4 = typename Vec4<TM>::type;
    using V4 = typename Vec4<T>::type;
    const M4 m = *reinterpret_cast<const M4*>(Minv + (size_t)node * 16 + r * 4);
    const V4 x = *reinterpret_cast<const V4*>(v + 4 * (size_t)node);
    double acc = double(m.x) * double(x.x) + double(m.y) * double(x.y) + double(m.z) * double(x.z) +
                 double(m.w) * double(x.w);
    if (zvec)
        acc += gs->kappa * gs->su * zvec[4 * (size_t)node + r];
    else if (r == 3 && !(dmask[node] & 8u))
        acc += gs->kappa * gs->su;
    t[4 * (size_t)node + r] = T(acc);
}

// ------------------------------------------------------------------- Arnoldi step kernels
// Gram-Schmidt with delayed reorthogonalisation and a single reduction per step (the DCGS2
// scheme of Swirydowicz et al. / Bielich et al., written here for right-preconditioned
// Arnoldi).  Entering step j, q_0 .. q_{j-1} are final and V[j] holds u_j, the next vector
// after one classical Gram-Schmidt pass, normalised by an estimate; column j-1 of H is
// provisional.  B = A P is the preconditioned operator, S(v) the sum of the free pressure
// entries of v.
//   spmv         w = (A P) u_j + kappa S(u_j) A z = B u_j, from the stored blocks of A P (S(u_j)
//                carried in gs); a step whose matrix is stored in a lower precision than its
//                basis instead applies P (precond_apply) and then A
//   dots         slots per (chunk, y): y < j -> (q_y . u_j, q_y . w);  y = j -> (u_j . u_j,
//                u_j . w);  y = j + 1 -> (w . w, S(w))    -> part[slot][chunk], stride = chunks
//   update       every workgroup sums the slots itself (step_scalars, same order everywhere):
//                s = Q^T u_j, rho = sqrt(u_j . u_j - |s|^2), so that q_j = (u_j - Q s)/rho is
//                u_j's second pass; with t = Q^T w and c = (t, c_j), c_j = (u_j . w - s . t) / rho
//                = q_j . w, and the provisional subdiagonal of column j is
//                hh = sqrt(w . w - |c|^2) / rho (Pythagoras).  Then q_j = (u_j - Q s) / rho over
//                V[j] and u_{j+1} = (w - Q t - c_j q_j) / (rho hh) to V[j+1].  Workgroup 0
//                instead does the Hessenberg columns (arnoldi_columns): column j-1 becomes final,
//                H(0:j-1, j-1) += hh' s and H(j, j-1) = hh' rho (hh': its provisional
//                subdiagonal), with its Givens rotation, residual estimate and done flag; then
//                H(0:j, j) = (c - H s) / rho and H(j+1, j) = hh.
// Three launches per step (a separate one-workgroup reduction cost more than every update
// workgroup summing the partials of kFusedChunks chunks again).  The tail of a cycle, the
// second pass of the last vector, is dots + reduce_kernel + columns_kernel.
// An estimate that loses digits to cancellation only scales u_{j+1}; the next step measures
// its norm directly (u . u), so the final subdiagonal hh rho is exact to rounding.  With
// reorthogonalisation off, s is taken as 0 (one Gram-Schmidt pass, the norm still measured).
// The chunks of a slot go to the XCDs through xcd_slot (when their count is a multiple of 8),
// matching the rows the update and the SpMV give each XCD.
constexpr int kDotChunks = VMS_DOT_CHUNKS;       // bound on the chunks (partials) per dot slot
constexpr int kDotThreads = 256;
constexpr int kDotUnrollF32 = 3;     // strides per pass for FP32 vectors (FP64: 1, register-bound)
static_assert(2 * (kMaxRestart + 2) * kDotChunks <= kRedBlocks * (kMaxRestart + 1), "dot slots exceed scratch");


// One thread's share of a chunk [i0, i1) of one dot slot: KIND 0 (q . u, q . w), 1 (u . u, u . w),
// 2 (w . w, S(w)).  kDotUnroll strides per pass, all loaded before any is used; indices past
// the chunk are clamped to its last node and weighted 0 (no branch around a load).  Three
// strides for FP32 vectors (the slot's loads then take one memory round at 32^3); FP64 keeps
// one, where nine 32-byte loads in flight cost more occupancy than they save.
template <int KIND, typename V4>
__device__ __forceinline__ void dot_chunk(const V4* __restrict__ q4, const V4* __restrict__ u4,
                                          const V4* __restrict__ w4, const uint8_t* __restrict__ dmask, int i0,
                                          int i1, double& a0, double& a1) {
    constexpr int kDotUnroll = sizeof(V4) <= 16 ? kDotUnrollF32 : 1;
    for (int ib = i0 + (int)threadIdx.x; ib < i1; ib += kDotUnroll * (int)blockDim.x) {
        V4 bv[kDotUnroll], xv[kDotUnroll], uv[kDotUnroll];
        uint8_t mk[kDotUnroll];
#pragma unroll
        for (int r = 0; r < kDotUnroll; ++r) {
            const int i = min(ib + r * (int)blockDim.x, i1 - 1);
            bv[r] = w4[i];
            if (KIND == 0) xv[r] = q4[i];
            if (KIND <= 1) uv[r] = u4[i];
            if (KIND == 2) mk[r] = dmask[i];
        }
#pragma unroll
        for (int r = 0; r < kDotUnroll; ++r) {
            const double wt = ib + r * (int)blockDim.x < i1 ? 1.0 : 0.0;
            const V4 b = bv[r];
            if (KIND == 0) {
                const V4 q = xv[r], u = uv[r];
                a0 += wt * double(q.x * u.x + q.y * u.y + q.z * u.z + q.w * u.w);
                a1 += wt * double(q.x * b.x + q.y * b.y + q.z * b.z + q.w * b.w);
            } else if (KIND == 1) {
                const V4 u = uv[r];
                a0 += wt * double(u.x * u.x + u.y * u.y + u.z * u.z + u.w * u.w);
                a1 += wt * double(u.x * b.x + u.y * b.y + u.z * b.z + u.w * b.w);
            } else {
                a0 += wt * double(b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w);
                a1 += (mk[r] & 8u) ? 0.0 : wt * double(b.w);
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kDotThreads) void dots_kernel(int n_nodes, int j, const T* __restrict__ V,
                                                           const T* __restrict__ w,
                                                           const uint8_t* __restrict__ dmask,
                                                           double* __restrict__ part, const GmresState* gs) {
    // a finished cycle reads nothing (the replayed steps after convergence cost only their
    // launches); its partials are left as they are, and the update and the tail test the flag too
    if (gs->done) return;
    using V4 = typename Vec4<T>::type;
    const int y = blockIdx.y;
    const int kind = y < j ? 0 : (y == j ? 1 : 2);
    const size_t N4 = (size_t)n_nodes;          // float4 / double4 entries per vector
    const V4* u4 = reinterpret_cast<const V4*>(V) + (size_t)j * N4;
    const V4* w4 = reinterpret_cast<const V4*>(w);
    const V4* q4 = reinterpret_cast<const V4*>(V) + (size_t)(kind == 0 ? y : 0) * N4;
    const int per = (n_nodes + gridDim.x - 1) / gridDim.x;
    const int chunk = gridDim.x % kXcds == 0 ? xcd_slot(blockIdx.x, gridDim.x) : blockIdx.x;
    const int i0 = chunk * per, i1 = min(n_nodes, i0 + per);
    double a0 = 0.0, a1 = 0.0;
    if (kind == 0)
        dot_chunk<0>(q4, u4, w4, dmask, i0, i1, a0, a1);
    else if (kind == 1)
        dot_chunk<1>(q4, u4, w4, dmask, i0, i1, a0, a1);
    else
        dot_chunk<2>(q4, u4, w4, dmask, i0, i1, a0, a1);
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    __shared__ double lds[2][kDotThreads / 64];
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = a0;
        lds[1][threadIdx.x >> 6] = a1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double t = 0.0;
        for (int k = 0; k < kDotThreads / 64; ++k) t += lds[threadIdx.x][k];
        part[(size_t)(2 * y + threadIdx.x) * gridDim.x + chunk] = t;
    }
}

// Values the Givens rotations read from the cycle state, loaded ahead of the chain.
struct GivensCtx {
    double tol_abs;
    uint64_t* progress;
    unsigned gen;
};

// Givens rotation of column jc (held in LDS, rows 0 .. jc+1), with the rotations of columns
// 0 .. jc-1 in LDS (cl, sl) and gj the rotated right-hand side entry jc.  The rotated column
// (rows 0 .. jc) goes to Rl in LDS, for the workgroup to store; the rotation, g, the residual
// estimate, k and the done flag go to the cycle state, and the progress is published.
// Returns 1 when the cycle stops.  Called by one thread, which issues no memory access in the
// chain (inside a launch that streams vectors, every such access would queue behind the
// stream); the LDS operands are fetched four at a time.
__device__ int givens_column(int jc, const double* col, double* cl, double* sl, double gj, double* Rl,
                             const GivensCtx& gc, GmresState* gs, int done_val, int i0 = 0, double x0 = 0.0) {
    // i0 > 0: rows 0 .. i0-1 of the column were already rotated (Rl) and x0 is row i0
    double x = i0 > 0 ? x0 : col[0];
    int i = i0;
    for (; i + 4 <= jc; i += 4) {
        double c4[4], s4[4], y4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c4[q] = cl[i + q];
            s4[q] = sl[i + q];
            y4[q] = col[i + q + 1];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Rl[i + q] = c4[q] * x + s4[q] * y4[q];
            x = -s4[q] * x + c4[q] * y4[q];
        }
    }
    for (; i < jc; ++i) {
        const double yv = col[i + 1];
        Rl[i] = cl[i] * x + sl[i] * yv;
        x = -sl[i] * x + cl[i] * yv;
    }
    const double hn = col[jc + 1];
    const double d = hypot(x, hn);
    const double cs = d > 0.0 ? x / d : 1.0;
    const double sn = d > 0.0 ? hn / d : 0.0;
    const double gnext = -sn * gj;
    const bool conv = fabs(gnext) <= gc.tol_abs;
    const bool breakdown = !(hn > 1e-300 * (fabs(d) + 1e-300)) || !isfinite(hn) || !isfinite(gnext);
    Rl[jc] = d;
    gs->cs[jc] = cs;
    gs->sn[jc] = sn;
    cl[jc] = cs;
    sl[jc] = sn;
    gs->g[jc] = cs * gj;
    gs->gin[jc + 1] = gnext;
    gs->k = jc + 1;
    const int stop = (conv || breakdown) ? 1 : 0;
    if (stop) gs->done = done_val;
    report_progress(gc.progress, gc.gen, jc + 1, stop);
    return stop;
}


// The tail of a cycle (one workgroup of kRedThreads): the dot slots of the last vector u_m are
// summed (eight lanes per slot, eight chunks each, loaded in one predicated round), and one wave
// forms rho (the norm of u_m after its second pass), S(q_m) and s, which arnoldi_columns needs
// to make column m-1 final.  eps_dot: relative accuracy of the dot products (precision of the
// stored vectors); a squared norm that cancels below eps_dot times its input is a numerical
// breakdown.  A vanished or non-finite rho is stored as 0, which makes arnoldi_columns close
// the cycle at column m-1.  (Inside a cycle the update launch forms the same sums itself,
// step_scalars below.)
constexpr int kRedThreads = 1024;
constexpr int kSlotLanes = 8;                               // lanes per dot slot
constexpr int kSlotChunks = 64 / kSlotLanes;                // chunks per lane
constexpr int kSlotGroups = kRedThreads / kSlotLanes;       // slots per round
constexpr int kSlotRounds = (2 * (kMaxRestart + 2) + kSlotGroups - 1) / kSlotGroups;
static_assert(kDotChunks <= 64, "a slot has at most 64 chunks");

__global__ __launch_bounds__(kRedThreads) void reduce_kernel(int j, int nchunks, const double* __restrict__ part,
                                                             GmresState* gs, double eps_dot) {
    __shared__ double sums[2 * (kMaxRestart + 2)];
    __shared__ double svl[kMaxRestart + 1];
    __shared__ double su_l;
    __shared__ int flags[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ns = 2 * (j + 2);
    const int grp = tid / kSlotLanes, sub = tid % kSlotLanes;
    double pv[kSlotRounds][kSlotChunks];
#pragma unroll
    for (int r = 0; r < kSlotRounds; ++r) {
        const int slot = grp + kSlotGroups * r;
#pragma unroll
        for (int c = 0; c < kSlotChunks; ++c) {
            const int ch = sub * kSlotChunks + c;
            pv[r][c] = (slot < ns && ch < nchunks) ? part[(size_t)slot * nchunks + ch] : 0.0;
        }
    }
    if (tid < j) svl[tid] = gs->svs[tid];
    if (tid == 0) {
        flags[0] = gs->done;
        flags[1] = gs->reorth;
        su_l = gs->su;
    }
#pragma unroll
    for (int r = 0; r < kSlotRounds; ++r) {
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < kSlotChunks; ++c) a += pv[r][c];
        a = group8_sum(a);
        const int slot = grp + kSlotGroups * r;
        if (sub == 0 && slot < ns) sums[slot] = a;
    }
    __syncthreads();
    if (flags[0]) return;
    const int reorth = flags[1];
    // sums: s_i = sums[2i] (i < j), then u.u at 2j (the t slots are not used here)
    for (int i = tid; i < j; i += kRedThreads) gs->scoef[i] = reorth ? sums[2 * i] : 0.0;
    if (wave != 0) return;
    // |s|^2 and s.S(q) over i < j
    double a[2] = {0.0, 0.0};
    for (int i = lane; i < j; i += 64) {
        const double si = reorth ? sums[2 * i] : 0.0;
        a[0] += si * si;
        a[1] += si * svl[i];
    }
    a[0] = wave_sum(a[0]);
    a[1] = wave_sum(a[1]);
    if (lane != 0) return;
    const double r2 = sums[2 * j] - a[0];
    double rho = j > 0 ? (r2 > eps_dot * sums[2 * j] ? sqrt(r2) : 0.0) : 1.0;
    if (!(rho > 0.0) || !isfinite(rho)) rho = 0.0;
    gs->svs[j] = j == 0 ? su_l : (rho > 0.0 ? (su_l - a[1]) / rho : 0.0);     // S(q_j)
    gs->rho = rho;
}

// Sum over the four lanes of an aligned group (every lane gets it; all lanes active).
__device__ __forceinline__ double group4_sum(double v) {
    v += dpp_mov<0xB1>(v);
    return v + dpp_mov<0x4E>(v);
}

// The Hessenberg bookkeeping of step j, for one workgroup of kBlock threads.  It needs the
// step's sums, and nothing of the Arnoldi recurrence waits for it, so it runs as workgroup 0 of
// the update launch, with the sums that workgroup formed in LDS (in), and, for the cycle's
// tail, as a launch of its own after reduce_kernel (in = nullptr: column j-1 only, inputs from
// the cycle state).
//  * u_j's second pass makes column j-1 final: H(0:j-1, j-1) += hh' s and H(j, j-1) = hh' rho,
//    hh' being the provisional subdiagonal stored at step j-1; its Givens rotation gives the
//    residual estimate, k = j and, on convergence or breakdown, the done flag.
//  * column j: H(0:j, j) = (c - H s) / rho with c = (t, c_j), H(j+1, j) = hh.  A zero hh means
//    an invariant Krylov space: column j is final and closes the cycle.
// Every value is loaded in one round before the first test, the columns 0 .. j-2 that H s needs
// included (lane = row, wave w = the columns l = w mod 4, kFirst of them per lane; more in
// batches).  Column j is written even when column j-1 closes the cycle: it lies beyond the
// final basis and the next cycle rebuilds it.
struct StepIn {
    const double* sums;     // s_i = sums[2i] (before the reorthogonalisation switch), t_i = sums[2i+1]
    double rho, cj, hh;
    int reorth;
};

__device__ void arnoldi_columns(int j, GmresState* gs, const StepIn* in) {
    constexpr int ld = kMaxRestart + 1;
    constexpr int kWaves = kBlock / 64;
    constexpr int kFirst = 12;                          // H loads per lane in the first round
    constexpr int kBatch = 4;                           // then per batch
    static_assert(kMaxRestart <= 128 && kBlock >= 64 + kMaxRestart, "two row passes; rows on waves 1..");
    __shared__ double Hc[kMaxRestart + 2];              // column j-1, final
    __shared__ double colj[kMaxRestart + 2];            // column j
    __shared__ double sv[kMaxRestart];                  // s
    __shared__ double cl[kMaxRestart], sl[kMaxRestart];
    __shared__ double hpart[kWaves][kMaxRestart];       // H s, per column class
    __shared__ double Rl[2][kMaxRestart + 1];           // rotated columns j-1 and j
    __shared__ double dr_v[kDrMax + 1];                 // deflated restarting: c, then Q^T c
    __shared__ double dr_x0;                            // row dk of a column after Q^T
    __shared__ int flags[1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // deflated restarting: columns 0 .. dk-1 of H are the kept block (rows 0 .. dk), set by the
    // host together with their rotated form (R) and Q^T; step dk starts the Arnoldi recurrence
    const int dk = gs->dr_k;
    const bool dr_first = dk > 0 && j == dk;
    auto rowmax = [&](int l) { return l < dk ? dk : l + 1; };   // last nonzero row of column l
    const int r = tid - 64;                             // row of column j (waves 1 ..)
    const bool last = in == nullptr;                    // the tail: column j-1 only
    const bool hs_on = !last && j > 1;                  // columns 0 .. j-2 take part in H s
    const int done = in ? 0 : gs->done;                 // the fused update has tested it
    // a stop found by the update launch of step j is stored as j + 2, which that launch's other
    // workgroups read as "not yet stopped": they still write q_j, which the closing column needs
    const int done_val = in ? j + 2 : 1;
    const int reorth = in ? in->reorth : gs->reorth;
    const double rho = in ? in->rho : gs->rho, hh = in ? in->hh : gs->hh, cj = in ? in->cj : gs->cj;
    const double gprev = j > 0 ? gs->gin[j - 1] : 0.0;
    const double hprev = j > 0 ? gs->H[(size_t)(j - 1) * ld + j] : 0.0;
    const GivensCtx gc{gs->tol_abs, gs->progress, gs->gen};
    double s_t = 0.0, hp = 0.0, cs_t = 0.0, sn_t = 0.0, t_r = 0.0;
    if (tid < j) {
        s_t = in ? in->sums[2 * tid] : gs->scoef[tid];
        hp = gs->H[(size_t)(j - 1) * ld + tid];
    }
    if (tid + 1 < j) {
        cs_t = gs->cs[tid];
        sn_t = gs->sn[tid];
    }
    if (!last && r >= 0 && r < j) t_r = in->sums[2 * r + 1];
    double hv[kFirst];
#pragma unroll
    for (int q = 0; q < kFirst; ++q) {
        const int l = wave + kWaves * q;
        hv[q] = (hs_on && l <= j - 2 && lane <= rowmax(l)) ? gs->H[(size_t)l * ld + lane] : 0.0;
    }
    if (done) return;                                   // uniform: written by an earlier launch
    if (tid < j) sv[tid] = reorth ? s_t : 0.0;
    if (tid + 1 < j) {
        cl[tid] = cs_t;
        sl[tid] = sn_t;
    }
    __syncthreads();
    if (j > 0 && tid <= j) {
        if (dr_first) {
            // column dk-1 is the kept block's last column: final as the host set it
            Hc[tid] = gs->H[(size_t)(j - 1) * ld + tid];
        } else {
            const double h = tid < j ? hp + hprev * sv[tid] : hprev * rho;
            Hc[tid] = h;
            gs->H[(size_t)(j - 1) * ld + tid] = h;
        }
    }
    if (dr_first && tid <= dk) dr_v[tid] = gs->beta * (tid < dk ? sv[tid] : rho);
    if (hs_on) {
        double acc[2] = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < kFirst; ++q) {
            const int l = wave + kWaves * q;
            if (l <= j - 2) acc[0] += hv[q] * sv[l];
        }
        for (int p = 0; p < 2; ++p) {
            const int i = lane + 64 * p;
            if (i > j) break;
            const int lbeg = wave + (p == 0 ? kWaves * kFirst : kWaves * (63 / kWaves));
            for (int l0 = lbeg; l0 <= j - 2; l0 += kWaves * kBatch) {
                double hb[kBatch];
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    const int l = l0 + kWaves * q;
                    hb[q] = (l <= j - 2 && i <= rowmax(l)) ? gs->H[(size_t)l * ld + i] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    const int l = l0 + kWaves * q;
                    if (l <= j - 2) acc[p] += hb[q] * sv[l];
                }
            }
        }
        if (lane <= j) hpart[wave][lane] = acc[0];
        if (lane + 64 <= j) hpart[wave][lane + 64] = acc[1];
    }
    __syncthreads();
    // deflated restarting: Q^T of the kept block on rows 0 .. dk -- of the cycle's right-hand
    // side c = beta (s, rho) at step dk, of column j-1 at later steps
    if (dk > 0 && j >= dk && !(j == dk && last)) {
        double t = 0.0;
        if (tid <= dk) {
            const double* src = dr_first ? dr_v : Hc;
            for (int l = 0; l <= dk; ++l) t += gs->dr_qt[l * (dk + 1) + tid] * src[l];
        }
        __syncthreads();
        if (tid <= dk) {
            if (dr_first) {
                gs->dr_c[tid] = dr_v[tid];
                if (tid < dk) gs->g[tid] = t;
                else dr_x0 = t;
            } else if (tid < dk) {
                Rl[0][tid] = t;
            } else {
                dr_x0 = t;
            }
        }
        __syncthreads();
    }
    // wave 0: the rotation of column j-1;  waves 1 ..: column j
    if (tid == 0) {
        int st = 0;
        if (dr_first) {
            // the kept block's residual estimate; the columns 0 .. dk-1 are done
            gs->gin[dk] = dr_x0;
            gs->k = dk;
            st = (fabs(dr_x0) <= gc.tol_abs || !(rho > 0.0) || !isfinite(dr_x0)) ? 1 : 0;
            if (st) gs->done = done_val;
            report_progress(gc.progress, gc.gen, dk, st);
        } else if (j > 0) {
            st = dk > 0 ? givens_column(j - 1, Hc, cl, sl, gprev, Rl[0], gc, gs, done_val, dk, dr_x0)
                        : givens_column(j - 1, Hc, cl, sl, gprev, Rl[0], gc, gs, done_val);
            if (!(rho > 0.0)) {
                st = 1;                      // u_j vanished: column j-1 closes the cycle
                gs->done = done_val;
                report_progress(gc.progress, gc.gen, j, 1);
            }
        }
        flags[0] = st;
    }
    const bool col_on = !last && rho > 0.0;
    if (col_on && r >= 0 && r <= j) {
        double hs = 0.0;
        if (j > 0 && reorth) {
            if (hs_on)
                for (int w = 0; w < kWaves; ++w) hs += hpart[w][r];
            hs += Hc[r] * sv[j - 1];
        }
        const double h = ((r < j ? t_r : cj) - hs) / rho;
        colj[r] = h;
        gs->H[(size_t)j * ld + r] = h;
        if (r == j) gs->H[(size_t)j * ld + j + 1] = hh;
    }
    __syncthreads();
    if (j > 0 && tid < j && !dr_first) gs->R[(size_t)(j - 1) * ld + tid] = Rl[0][tid];
    if (!(col_on && !flags[0] && !(hh > 0.0))) return;  // uniform
    // the Krylov space is invariant: column j is final with a zero subdiagonal
    if (dk > 0) {                                       // Q^T of the kept block on its rows 0 .. dk
        double t = 0.0;
        if (tid <= dk)
            for (int l = 0; l <= dk; ++l) t += gs->dr_qt[l * (dk + 1) + tid] * colj[l];
        __syncthreads();
        if (tid < dk) Rl[1][tid] = t;
        if (tid == dk) dr_x0 = t;
        __syncthreads();
    }
    if (tid == 0) {
        colj[j + 1] = 0.0;
        const double gj = gs->gin[j];
        if (dk > 0) givens_column(j, colj, cl, sl, gj, Rl[1], gc, gs, done_val, dk, dr_x0);
        else givens_column(j, colj, cl, sl, gj, Rl[1], gc, gs, done_val);
        gs->done = done_val;
        report_progress(gc.progress, gc.gen, j + 1, 1);
    }
    __syncthreads();
    if (tid <= j) gs->R[(size_t)j * ld + tid] = Rl[1][tid];
}

// The tail of a cycle: column j-1 from the last vector's second pass.
__global__ __launch_bounds__(kBlock) void columns_kernel(int j, GmresState* gs) { arnoldi_columns(j, gs, nullptr); }

// ------------------------------------------------------------- fused step (3 launches per step)
// The update launch forms the step's sums itself: every workgroup reads the dot partials
// (kFusedChunks per slot, four lanes per slot) and forms rho, c_j, hh exactly as the reduction
// kernel does, in the same order everywhere, so all workgroups agree bitwise.  The basis loads
// of the first batch are issued before, and wait out, that work.  Workgroup 0 also stores the
// free-pressure sums S(q_j), S(u_{j+1}) for later steps and runs arnoldi_columns from LDS.
constexpr int kFusedChunks = 16;                                     // dot partials per slot
constexpr int kFusedLanes = 4;                                       // lanes per slot
constexpr int kFusedPer = kFusedChunks / kFusedLanes;                // partials per lane
constexpr int kFusedSlots = kBlock / kFusedLanes;                    // slots per round
constexpr int kFusedRounds = (2 * (kMaxRestart + 2) + kFusedSlots - 1) / kFusedSlots;
static_assert(kFusedChunks % kXcds == 0 && kFusedChunks <= kDotChunks, "fused dot chunks");
// Large meshes: the dots write kWideChunks partials per slot (more workgroups streaming the
// basis when j is small), slot_sum_kernel adds them, and the update reads one sum per slot.
constexpr int kWideChunks = 64;
constexpr int kWideMinNodes = 131072;
constexpr int kWideSumOffset = 2 * (kMaxRestart + 2) * kWideChunks;   // sums after the partials
static_assert(kWideChunks <= kDotChunks && kWideChunks % kXcds == 0, "wide dot chunks");
static_assert(kWideSumOffset + 2 * (kMaxRestart + 2) <= kRedBlocks * (kMaxRestart + 1), "wide sums exceed scratch");

// sums[y] = the nchunks partials of slot y added in chunk order (one workgroup; idle once the
// cycle has stopped).
__global__ __launch_bounds__(kBlock) void slot_sum_kernel(int j, int nchunks, const double* __restrict__ part,
                                                          double* __restrict__ sums, const GmresState* gs) {
    if (gs->done) return;
    const int ns = 2 * (j + 2);
    for (int y = threadIdx.x; y < ns; y += blockDim.x) {
        const double* p = part + (size_t)y * nchunks;
        double v[kWideChunks];
#pragma unroll
        for (int c = 0; c < kWideChunks; ++c) v[c] = c < nchunks ? p[c] : 0.0;
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < kWideChunks; ++c) t += v[c];
        sums[y] = t;
    }
}

struct StepLds {
    double sums[2 * (kMaxRestart + 2)];
    double svl[kMaxRestart + 1];
    double su;              // S(u_j)
    int flags[2];           // done, reorth
};

struct StepOut {
    double rho, cj, hh;
    double su_next;         // S(u_{j+1})
    double svj;             // S(q_j)
};

// Returns false (uniformly) when the cycle is done.  Every thread of the workgroup calls it.
__device__ __forceinline__ bool step_scalars(int j, int nchunks, const double* __restrict__ part, const GmresState* gs,
                                             double eps_dot, StepLds& L, StepOut& o) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int ns = 2 * (j + 2);
    const int grp = tid / kFusedLanes, sub = tid % kFusedLanes;
    // part[slot][0 .. nchunks) is contiguous (stride nchunks): lane sub of a slot reads its
    // kFusedPer consecutive partials.  Only the rounds that hold slots are issued; inside one,
    // every load is unconditional (slot and chunk clamped to valid ones) and weighted 0 when
    // absent, since a load under a per-lane condition becomes a branch with a full wait.
    const int rounds = (ns + kFusedSlots - 1) / kFusedSlots;
    double pv[kFusedRounds][kFusedPer];
#pragma unroll
    for (int r = 0; r < kFusedRounds; ++r) {
        const int slot = grp + kFusedSlots * r;
        const size_t base = (size_t)min(slot, ns - 1) * nchunks;
#pragma unroll
        for (int c = 0; c < kFusedPer; ++c) pv[r][c] = 0.0;
        if (r < rounds) {
#pragma unroll
            for (int c = 0; c < kFusedPer; ++c) {
                const int ch = sub * kFusedPer + c;
                const double wt = (slot < ns && ch < nchunks) ? 1.0 : 0.0;
                pv[r][c] = wt * part[base + min(ch, nchunks - 1)];
            }
        }
    }
    if (tid < j) L.svl[tid] = gs->svs[tid];
    if (tid == 0) {
        L.flags[0] = gs->done;
        L.flags[1] = gs->reorth;
        L.su = gs->su;
    }
#pragma unroll
    for (int r = 0; r < kFusedRounds; ++r) {
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < kFusedPer; ++c) a += pv[r][c];
        a = group4_sum(a);
        const int slot = grp + kFusedSlots * r;
        if (sub == 0 && slot < ns) L.sums[slot] = a;
    }
    __syncthreads();
    // stopped by an earlier launch (cycle start: 1; the update of step j' < j: j' + 2); a stop
    // that workgroup 0 of this launch publishes (j + 2) does not count, since q_j is still due
    const int dw = L.flags[0];
    if (dw != 0 && dw <= j + 1) return false;
    // every wave forms the scalars itself (the wave sums leave them in every lane), so that no
    // second barrier is needed; all lanes and workgroups do the same operations in the same order
    const int reorth = L.flags[1];
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = lane; i < j; i += 64) {
        const double si = reorth ? L.sums[2 * i] : 0.0, ti = L.sums[2 * i + 1], pi = L.svl[i];
        a[0] += si * si;
        a[1] += si * ti;
        a[2] += si * pi;
        a[3] += ti * ti;
        a[4] += ti * pi;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) a[q] = wave_sum(a[q]);
    const double su = L.su;
    const double r2 = L.sums[2 * j] - a[0];
    double rho = j > 0 ? (r2 > eps_dot * L.sums[2 * j] ? sqrt(r2) : 0.0) : 1.0;
    if (!(rho > 0.0) || !isfinite(rho)) rho = 0.0;
    const double svj = j == 0 ? su : (rho > 0.0 ? (su - a[2]) / rho : 0.0);
    double cj = 0.0, hh = 0.0, sun = 0.0;
    if (rho > 0.0) {
        cj = (L.sums[2 * j + 1] - a[1]) / rho;
        const double cc = a[3] + cj * cj;
        const double pw = L.sums[2 * j + 3] - a[4] - cj * svj;
        const double h2 = L.sums[2 * j + 2] - cc;
        hh = h2 > eps_dot * L.sums[2 * j + 2] ? sqrt(h2) / rho : 0.0;
        if (!isfinite(hh)) hh = 0.0;
        sun = hh > 0.0 ? pw / (rho * hh) : 0.0;
    }
    o = StepOut{rho, cj, hh, sun, svj};
    return true;
}

// The vector rows are split in eighths of xrows rows, one per XCD: the rows whose dot products
// the dots launch formed on that XCD, so that their reads here hit its L2.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void update_fused_kernel(int n, int xrows, int j, T* __restrict__ V,
                                                              const T* __restrict__ w, int nchunks,
                                                              const double* __restrict__ part, GmresState* gs,
                                                              double eps_dot) {
    __shared__ StepLds L;
    StepOut o;
    if (blockIdx.x == 0) {
        if (!step_scalars(j, nchunks, part, gs, eps_dot, L, o)) return;
        if (threadIdx.x == 0) {
            gs->rho = o.rho;
            gs->cj = o.cj;
            gs->hh = o.hh;
            gs->su = o.su_next;     // S(u_{j+1}); the other workgroups read only S(u_j), unused there
            gs->svs[j] = o.svj;
        }
        const StepIn in{L.sums, o.rho, o.cj, o.hh, L.flags[1]};
        arnoldi_columns(j, gs, &in);
        return;
    }
    // R rows per thread, each row's loads coalesced across the workgroup; workgroup b runs on
    // XCD b mod 8 and takes the (b-1)/8-th block of R * blockDim rows of that XCD's eighth
    const int bb = blockIdx.x - 1;
    const int base = ((bb + 1) % kXcds) * xrows, end = min(n, base + xrows);
    int idx[R], ix[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        idx[r] = base + ((bb / kXcds) * R + r) * (int)blockDim.x + (int)threadIdx.x;
        ix[r] = idx[r] < n ? idx[r] : n - 1;     // every thread takes part in the step's sums
    }
    const size_t N = (size_t)n;
    T* uj = V + (size_t)j * N;
    double aq[R], aw[R];
    T v0[8][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        aq[r] = double(uj[ix[r]]);
        aw[r] = double(w[ix[r]]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) v0[q][r] = V[(size_t)min(q, max(j - 1, 0)) * N + ix[r]];
    if (!step_scalars(j, nchunks, part, gs, eps_dot, L, o)) return;
    const bool reorth = L.flags[1] != 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (q < j) {
            const double sq = reorth ? L.sums[2 * q] : 0.0, tq = L.sums[2 * q + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                aq[r] -= sq * double(v0[q][r]);
                aw[r] -= tq * double(v0[q][r]);
            }
        }
    }
    int i = 8;
    for (; i + 8 <= j; i += 8) {
        double vv[8][R];
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) vv[q][r] = double(V[(size_t)(i + q) * N + ix[r]]);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double sq = reorth ? L.sums[2 * (i + q)] : 0.0, tq = L.sums[2 * (i + q) + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                aq[r] -= sq * vv[q][r];
                aw[r] -= tq * vv[q][r];
            }
        }
    }
    for (; i < j; ++i) {
        const double sq = reorth ? L.sums[2 * i] : 0.0, tq = L.sums[2 * i + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double v = double(V[(size_t)i * N + ix[r]]);
            aq[r] -= sq * v;
            aw[r] -= tq * v;
        }
    }
    const double rho = o.rho, cj = o.cj, hh = o.hh;
    if (!(rho > 0.0)) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (idx[r] >= end) continue;             // beyond the vector or this XCD's eighth
        const double q = aq[r] / rho;
        uj[idx[r]] = T(q);
        if (hh > 0.0) V[(size_t)(j + 1) * N + idx[r]] = T((aw[r] - cj * q) / (rho * hh));
    }
}

// y = R^{-1} g for the k x k triangle of the rotated Hessenberg matrix (one workgroup): the
// triangle and the reciprocals of its diagonal are staged in LDS (column batches, loads in
// flight together), then one wave eliminates
// column by column, lane l holding entries l and l + 64 of the right-hand side; the pivot
// entry is broadcast with readlane, so the sequential chain is a multiply and an FMA per column.
__global__ __launch_bounds__(kBlock) void backsub_kernel(GmresState* gs) {
    const int k = gs->k;
    if (k == 0) return;
    constexpr int ld = kMaxRestart + 1;
    __shared__ double Rl[kMaxRestart * kMaxRestart];
    __shared__ double rinv[kMaxRestart];
    // staging: lane = row (two halves), wave w = the columns col = w mod 4, eight columns of a
    // lane loaded before any is stored (clamped column, so no branch around a load)
    constexpr int kWaves = kBlock / 64, kCols = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = wave; c0 < k; c0 += kWaves * kCols) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int row = lane + 64 * half;
            if (row >= k) break;
            double rv[kCols];
#pragma unroll
            for (int q = 0; q < kCols; ++q) rv[q] = gs->R[(size_t)min(c0 + kWaves * q, k - 1) * ld + row];
#pragma unroll
            for (int q = 0; q < kCols; ++q) {
                const int col = c0 + kWaves * q;
                if (col < k && row <= col) {
                    Rl[col * k + row] = rv[q];
                    if (row == col) rinv[col] = 1.0 / rv[q];
                }
            }
        }
    }
    double g0 = 0.0, g1 = 0.0;
    if (threadIdx.x < 64) {
        g0 = threadIdx.x < k ? gs->g[threadIdx.x] : 0.0;
        g1 = threadIdx.x + 64 < k ? gs->g[threadIdx.x + 64] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int l = threadIdx.x;
    for (int col = k - 1; col >= 0; --col) {
        const double yc = read_lane(col < 64 ? g0 : g1, col & 63) * rinv[col];
        if (l == 0) gs->y[col] = yc;
        if (l < col) g0 -= Rl[col * k + l] * yc;
        if (l + 64 < col) g1 -= Rl[col * k + l + 64] * yc;
    }
}

// t = sum_{i<k} y_i V_i
template <typename T>
__global__ __launch_bounds__(kBlock) void combine_kernel(int n, const T* __restrict__ V, const GmresState* gs,
                                                         T* __restrict__ t) {
    const int k = gs->k;
    if (k == 0) return;
    __shared__ double ys[kMaxRestart];
    for (int i = threadIdx.x; i < k; i += blockDim.x) ys[i] = gs->y[i];
    __syncthreads();
    const int idx = xcd_slot(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;   // basis slices in this XCD's L2
    if (idx >= n) return;
    const size_t N = (size_t)n;
    double sacc = 0.0;
    int i = 0;
    for (; i + 8 <= k; i += 8) {
        double vv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) vv[q] = double(V[(size_t)(i + q) * N + idx]);
#pragma unroll
        for (int q = 0; q < 8; ++q) sacc += ys[i + q] * vv[q];
    }
    for (; i < k; ++i) sacc += ys[i] * double(V[(size_t)i * N + idx]);
    t[idx] = T(sacc);
}

// gs->st = sum of the free pressure entries of t (for the coarse term of P t)
template <typename T>
__global__ __launch_bounds__(kBlock) void free_pressure_sum_kernel(int n_nodes, const T* __restrict__ t,
                                                                   const uint8_t* __restrict__ dmask,
                                                                   RedScratch* red, GmresState* gs) {
    if (gs->k == 0) return;
    __shared__ double lds[kBlock / 64];
    double v[1] = {0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes; i += gridDim.x * blockDim.x)
        if (!(dmask[i] & 8u)) v[0] += double(t[4 * (size_t)i + 3]);
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) red->partial[blockIdx.x] = v[0];
    if (!arrive_last(&red->counter)) return;
    __threadfence();
    __shared__ double tot;
    reduce_partials(red->partial, kRedBlocks, 1, gridDim.x, &tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        gs->st = tot;
        red->counter = 0u;
    }
}

// x += xscale P t = xscale (Minv t + z kappa (1_p^T t))  (x in TX: double for the FP64 solution,
// float for an inner correction; xscale is the norm of the residual an FP32 cycle was given
// scaled to one).  z is the indicator of the free pressure dofs 1_p, or the explicit vector zvec.
template <typename TM, typename T, typename TX>
__global__ void precond_accumulate_kernel(int n_nodes, const TM* __restrict__ Minv, const T* __restrict__ t,
                                          const uint8_t* __restrict__ dmask, const double* __restrict__ zvec,
                                          const GmresState* gs, double xscale, TX* __restrict__ x) {
    if (gs->k == 0) return;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = tid >> 2, r = tid & 3;
    if (node >= n_nodes) return;
    using M4 = typename Vec4<TM>::type;
    using V4 = typename Vec4<T>::type;
    const M4 m = *reinterpret_cast<const M4*>(Minv + (size_t)node * 16 + r * 4);
    const V4 v = *reinterpret_cast<const V4*>(t + 4 * (size_t)node);
    double s = double(m.x) * double(v.x) + double(m.y) * double(v.y) + double(m.z) * double(v.z) +
               double(m.w) * double(v.w);
    if (zvec)
        s += gs->kappa * gs->st * zvec[4 * (size_t)node + r];
    else if (r == 3 && !(dmask[node] & 8u))
        s += gs->kappa * gs->st;
    x[4 * (size_t)node + r] = TX(double(x[4 * (size_t)node + r]) + xscale * s);
}

// FP64 norm of a vector of any precision into out (device) via partials.
template <typename T>
__global__ __launch_bounds__(kBlock) void norm_kernel(int n, const T* __restrict__ r, RedScratch* red,
                                                      double* out, uint64_t* tag_out, uint64_t tag) {
    __shared__ double lds[kBlock / 64];
    double v[1] = {0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double x = double(r[i]);
        v[0] += x * x;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) red->partial[blockIdx.x] = v[0];
    if (!arrive_last(&red->counter)) return;
    __threadfence();
    __shared__ double tot;
    reduce_partials(red->partial, kRedBlocks, 1, gridDim.x, &tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        // out and tag_out are pinned host memory (the context's mapped page): the value, then its
        // tag with release order, which the host polls for
        __hip_atomic_store(out, sqrt(tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        red->counter = 0u;
        __hip_atomic_store(tag_out, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ void zero_count_kernel(int32_t* p) {
    if (threadIdx.x == 0) *p = 0;
}

template <typename TS, typename TD>
__global__ void convert_kernel(int n, const TS* __restrict__ s, TD* __restrict__ d, double scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = TD(double(s[i]) * scale);
}

template <typename T>
__global__ void axpy64_kernel(int n, double alpha, const T* __restrict__ d, double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += alpha * double(d[i]);
}

// Workgroups of a grid-wide reduction: each one pays a device-scope fence and an atomic on the
// arrival counter, which costs more than streaming a few more elements per thread.
#ifndef VMS_RED_GRID_MAX
#define VMS_RED_GRID_MAX 128
#endif
static_assert(VMS_RED_GRID_MAX <= kRedBlocks, "reduction grid exceeds the partials");
inline int red_grid(int64_t n) { return std::max(1, std::min(VMS_RED_GRID_MAX, grid_for(n))); }

// Reads a device double with a stream sync.
// Launches the norm of r (n entries) into mapped scalar k with a fresh tag.
template <typename T>
void launch_norm(vms_ctx* c, int n, const T* r, int k, hipStream_t s) {
    norm_kernel<T><<<red_grid(n), kBlock, 0, s>>>(n, r, c->red, c->scal_dev + k, c->progress_dev + 1 + k,
                                                  ++c->scal_seq);
}

// Waits for mapped scalar k of the last launch_norm: spins on its tag in pinned memory (the
// launches after it on the stream are already ordered), with a stream query every 256 spins so
// that a failed or drained stream ends the wait.
int read_scalar(vms_ctx* c, int k, double* h, hipStream_t s) {
    const uint64_t want = c->scal_seq;
    const uint64_t* tag = c->progress_host + 1 + k;
    for (unsigned spin = 0;; ++spin) {
        if (__atomic_load_n(tag, __ATOMIC_ACQUIRE) == want) break;
        if ((spin & 255u) == 255u) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {
                if (__atomic_load_n(tag, __ATOMIC_ACQUIRE) == want) break;
                return set_error(c, VMS_EHIP, "read scalar: the stream finished without the value");
            }
            if (q != hipErrorNotReady) return check_hip(c, q, "read scalar: stream query");
        }
    }
    *h = *reinterpret_cast<volatile const double*>(c->scal_host + k);
    return VMS_OK;
}

#ifndef VMS_LEAD_STEPS
#define VMS_LEAD_STEPS 3
#endif
constexpr int kLeadSteps = VMS_LEAD_STEPS;   // Arnoldi steps the host may issue ahead of the device

// The device's progress word for cycle gen: completed columns (-1 before the cycle has
// reported), *done = 1 once the cycle stopped (converged or broke down).
int read_progress(const vms_ctx* c, uint32_t gen, int* done) {
    const uint64_t word = __atomic_load_n(c->progress_host, __ATOMIC_ACQUIRE);
    if ((uint32_t)(word >> 32) != gen) {
        *done = 0;
        return -1;
    }
    *done = (int)(word & 1u);
    return (int)((word >> 1) & 0x7fffffffu);
}

// Waits, without synchronising the stream, until cycle gen has completed `need` columns or
// stopped.  Returns 1 if it stopped, 0 if the columns are there (or the stream ran dry), a
// negative status on a HIP error.
int wait_progress(vms_ctx* c, uint32_t gen, int need, hipStream_t s) {
    for (unsigned spin = 0;; ++spin) {
        int done = 0;
        const int k = read_progress(c, gen, &done);
        if (done) return 1;
        if (k >= need) return 0;
        if ((spin & 255u) == 255u) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {           // every launch has finished: the word is final
                read_progress(c, gen, &done);
                return done;
            }
            if (q != hipErrorNotReady) {
                (void)check_hip(c, q, "gmres: stream query");
                return -1;
            }
        }
    }
}

// Launches one GMRES(m) cycle on A d = r0 with right preconditioner Minv, adding the Krylov
// correction xscale Minv (V y) (+ coarse term) to x (double or float).  r0 is the cycle's initial
// residual (precision T).  The host follows the device's progress through the mapped word,
// keeps at most kLeadSteps steps queued ahead of it and stops issuing steps once the cycle has
// converged; nothing here synchronises the stream.  finish_cycle gives the number of steps
// once the caller has synchronised.
// Cycle graphs are on unless VMS_CYCLE_GRAPHS=0 in the environment (read at every cycle).
inline bool cycle_graphs_enabled() {
    const char* e = std::getenv("VMS_CYCLE_GRAPHS");
    return !(e && e[0] == '0');
}

// The Krylov basis and work vectors of precision T: the context's own (its precision), or the
// FP64 set a mixed context allocates for solves with an FP64 basis.
template <typename T>
T* basis_vectors(vms_ctx* c, int which) {
    const bool own = sizeof(T) == elt_size(c);
    void* p[3] = {own ? c->V : c->V64, own ? c->w : c->w64, own ? c->z : c->z64};
    return static_cast<T*>(p[which]);
}

// One restart cycle: T the precision of the basis and of its arithmetic, TM that of the stored
// matrix, its A P blocks, A z and the preconditioner blocks, TX that of the iterate x.
// With TM != T the steps apply P and A (Amat) in two passes instead of the stored A P blocks.
template <typename T, typename TX, typename TM = T>
int run_cycle(vms_ctx* c, const T* r0, const TM* Minv, TX* x, double tol_abs, int m, int budget, int cgs2,
              hipStream_t s, double xscale = 1.0, int j0 = 0, const TM* Amat = nullptr) {
    constexpr bool split = !std::is_same<TM, T>::value;
    if (split && !Amat) return set_error(c, VMS_EINVAL, "gmres: no matrix for the split operator");
    const int n = 4 * c->n_nodes;
    const TM* AP = (const TM*)c->AP;
    const TM* Az = (const TM*)c->Az;
    T* V = basis_vectors<T>(c, 0);
    T* w = basis_vectors<T>(c, 1);
    T* z = basis_vectors<T>(c, 2);
    // recorded graphs are told apart by restart length, kept vectors and basis precision
    const int pbit = sizeof(T) == 8 ? 1 : 0;
    const uint32_t gen = ++c->cycle_gen;
    c->cycle_timed.clear();
    cycle_start_kernel<T><<<red_grid(n), kBlock, 0, s>>>(n, r0, c->dmask, c->red, c->gs, tol_abs, cgs2, gen);
    // a deflated cycle puts the residual after the kept vectors and runs steps j0 .. m-1
    cycle_v0_kernel<T><<<grid_for(n), kBlock, 0, s>>>(n, r0, V + (size_t)j0 * n, c->gs);
    const int steps = std::min(m - j0, budget);
    const double vb = (double)n * sizeof(T);      // bytes of one Krylov vector
    // algorithmic bytes of the Arnoldi SpMV: blocks and column indices, row pointers, the input
    // and output vectors once (the coarse-pressure vector A z it also reads is not credited)
    const double spmv_bytes = (double)c->nb * (16.0 * sizeof(TM) + 4.0) + 4.0 * (c->n_nodes + 1) + 2.0 * vb;
    const bool wide = c->n_nodes >= kWideMinNodes;
    const int nch = wide ? kWideChunks : std::max(1, std::min(kFusedChunks, (c->n_nodes + kDotThreads - 1) / kDotThreads));
    // rows of the vectors whose dots the workgroups on one XCD form (the dots take their chunks
    // in xcd_slot order when there are a multiple of 8 of them), which the update reads there too
    const int xrows = nch % kXcds == 0 ? 4 * ((c->n_nodes + nch - 1) / nch) * (nch / kXcds)
                                       : (n + kXcds - 1) / kXcds;
    double* part = c->red->partial;
    const double eps_dot = sizeof(T) == 8 ? 1e-14 : 1e-6;
    // timed launches per step, so that steps issued after convergence (their kernels return
    // at once) can be dropped from the phase timers
    auto keep = [&](int jj, const PhaseScope& ph) {
        if (ph.slot >= 0) {
            c->cycle_timed.push_back(jj);
            c->cycle_timed.push_back(ph.slot);
            c->cycle_timed.push_back(ph.gen);
        }
    };
    auto timed = [&](int phase, double bytes, int j, hipStream_t st, auto&& launch) {
        PhaseScope ph(c, phase, bytes, st);
        launch();
        keep(j, ph);
    };
    // the Arnoldi steps and the tail on stream st; with lead, the host keeps at most kLeadSteps
    // steps queued ahead of the device and stops issuing once the cycle has converged
    auto issue = [&](int steps_, bool lead, hipStream_t st) -> int {
        steps_ += j0;                                     // the last column index
        for (int j = j0; j < steps_; ++j) {
            if (lead && j - j0 >= kLeadSteps) {
                const int sw = wait_progress(c, gen, j - kLeadSteps, st);
                if (sw < 0) return VMS_EHIP;
                if (sw == 1) break;
            }
            // w = A P u_j = (A P) u_j + kappa S(u_j) A z, or A (P u_j) with z = P u_j
            if constexpr (split) {
                timed(VMS_PH_PCAPPLY, (double)c->n_nodes * (16.0 * sizeof(TM) + 8.0 * sizeof(T)), j, st, [&] {
                    precond_apply_kernel<TM, T><<<grid_for(n), kBlock, 0, st>>>(c->n_nodes, Minv, V + (size_t)j * n,
                                                                              c->dmask, c->zfull, c->gs, z);
                });
                timed(VMS_PH_SPMV, spmv_bytes, j, st, [&] {
                    spmv_kernel<TM, T, T, T, 0><<<spmv_grid(c->n_nodes), kBlock, 0, st>>>(
                        c->n_nodes, c->rowptr, c->colidx, Amat, z, (const double*)nullptr, w, &c->gs->done, c->gs);
                });
            } else {
                timed(VMS_PH_SPMV, spmv_bytes, j, st, [&] {
                    spmv_kernel<TM, T, T, T, 2, TM><<<spmv_grid(c->n_nodes), kBlock, 0, st>>>(
                        c->n_nodes, c->rowptr, c->colidx, AP, V + (size_t)j * n, Az, w, &c->gs->done, c->gs);
                });
            }
            timed(VMS_PH_DOTS, (j + 2) * vb, j, st, [&] {
                dots_kernel<T><<<dim3(nch, j + 2), kDotThreads, 0, st>>>(c->n_nodes, j, V, w, c->dmask, part,
                                                                         c->gs);
            });
            timed(VMS_PH_UPDATE, (j + 4) * vb, j, st, [&] {
                if (wide) slot_sum_kernel<<<1, kBlock, 0, st>>>(j, nch, part, part + kWideSumOffset, c->gs);
                // two vector rows per thread halve the workgroups that each form the step's
                // scalars, except for FP64 vectors on small meshes, where one row per thread
                // keeps more waves streaming the basis
                const double* sums = wide ? part + kWideSumOffset : part;
                const int nsum = wide ? 1 : nch;
                if (sizeof(T) == 4 || wide)
                    update_fused_kernel<T, 2><<<1 + kXcds * grid_for(xrows, 2 * kBlock), kBlock, 0, st>>>(
                        n, xrows, j, V, w, nsum, sums, c->gs, eps_dot);
                else
                    update_fused_kernel<T, 1><<<1 + kXcds * grid_for(xrows, kBlock), kBlock, 0, st>>>(
                        n, xrows, j, V, w, nsum, sums, c->gs, eps_dot);
            });
        }
        // the second pass of the last vector completes the last column
        dots_kernel<T><<<dim3(nch, steps_ + 2), kDotThreads, 0, st>>>(c->n_nodes, steps_, V, w, c->dmask, part,
                                                                      c->gs);
        reduce_kernel<<<1, kRedThreads, 0, st>>>(steps_, nch, part, c->gs, eps_dot);
        columns_kernel<<<1, kBlock, 0, st>>>(steps_, c->gs);
        return VMS_OK;
    };
    // With the phase timers on, every prof_every-th cycle is launched directly and every launch
    // of a timed phase in it is timed (events cannot time launches inside a graph).
    const bool graphs = steps == m - j0 && cycle_graphs_enabled();
    const bool sampled = c->prof_mask != 0 && c->prof_cycles++ % c->prof_every == 0;
    if (graphs && !sampled && j0 > 0) {
        // a full deflated cycle: one recorded graph per (m, j0), kept in a small cache
        const int key = (m * 256 + j0) * 2 + pbit;
        int slot = -1;
        for (int q = 0; q < 4; ++q)
            if (c->dr_exec[q] && c->dr_exec_key[q] == key) slot = q;
        if (slot < 0) {
            slot = 0;
            for (int q = 0; q < 4; ++q)
                if (!c->dr_exec[q]) {
                    slot = q;
                    break;
                }
            int rc = VMS_OK;
            if (!c->cap_stream &&
                (rc = check_hip(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream")))
                return rc;
            if (c->dr_exec[slot]) {
                (void)hipGraphExecDestroy(c->dr_exec[slot]);
                c->dr_exec[slot] = nullptr;
            }
            if ((rc = check_hip(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal),
                                "begin capture")))
                return rc;
            const uint32_t mask = c->prof_mask;
            c->prof_mask = 0;
            rc = issue(m - j0, false, c->cap_stream);
            c->prof_mask = mask;
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
            if (rc) return rc;
            if ((rc = check_hip(c, e, "end capture"))) return rc;
            rc = check_hip(c, hipGraphInstantiate(&c->dr_exec[slot], g, nullptr, nullptr, 0), "graph instantiate");
            (void)hipGraphDestroy(g);
            if (rc) return rc;
            c->dr_exec_key[slot] = key;
        }
        if (int rc = check_hip(c, hipGraphLaunch(c->dr_exec[slot], s), "graph launch")) return rc;
    } else if (graphs && !sampled) {
        // a full cycle: replay the recorded steps (the kernels after convergence return at once)
        if (!c->cycle_exec || c->cycle_exec_m != m * 2 + pbit) {
            int rc = VMS_OK;
            if (!c->cap_stream &&
                (rc = check_hip(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream")))
                return rc;
            if (c->cycle_exec) {
                (void)hipGraphExecDestroy(c->cycle_exec);
                c->cycle_exec = nullptr;
            }
            if ((rc = check_hip(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal),
                                "begin capture")))
                return rc;
            const uint32_t mask = c->prof_mask;      // nothing is timed inside the graph
            c->prof_mask = 0;
            rc = issue(m, false, c->cap_stream);
            c->prof_mask = mask;
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
            if (rc) return rc;
            if ((rc = check_hip(c, e, "end capture"))) return rc;
            rc = check_hip(c, hipGraphInstantiate(&c->cycle_exec, g, nullptr, nullptr, 0), "graph instantiate");
            (void)hipGraphDestroy(g);
            if (rc) return rc;
            c->cycle_exec_m = m * 2 + pbit;
        }
        if (int rc = check_hip(c, hipGraphLaunch(c->cycle_exec, s), "graph launch")) return rc;
    } else {
        c->prof_force = graphs && sampled;
        const int rc = issue(steps, true, s);
        c->prof_force = false;
        if (rc) return rc;
    }
    // y = R^{-1} g on the device
    backsub_kernel<<<1, kBlock, 0, s>>>(c->gs);
    combine_kernel<T><<<xcd_round(grid_for(n)), kBlock, 0, s>>>(n, V, c->gs, z);
    free_pressure_sum_kernel<T><<<red_grid(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, z, c->dmask, c->red, c->gs);
    precond_accumulate_kernel<TM, T, TX><<<grid_for(n), kBlock, 0, s>>>(c->n_nodes, Minv, z, c->dmask, c->zfull, c->gs,
                                                                    xscale, x);
    return check_hip(c, hipGetLastError(), "gmres cycle launch");
}

// After the caller has synchronised the stream: Arnoldi steps of the last cycle (*stopped = 1
// when the cycle ended on its own residual estimate or a breakdown, not on the step budget).
// Timed launches of steps issued after convergence are dropped.
int finish_cycle(vms_ctx* c, int* stopped = nullptr) {
    int done = 0;
    const int k = std::max(0, read_progress(c, c->cycle_gen, &done));
    if (stopped) *stopped = done;
    for (size_t i = 0; i + 2 < c->cycle_timed.size(); i += 3)
        if (c->cycle_timed[i] >= k) prof_void(c, (int)c->cycle_timed[i + 1], c->cycle_timed[i + 2]);
    c->cycle_timed.clear();
    return k;
}

// Deflated restarting after a full cycle of m steps that kept j0 vectors of its predecessor
// (the stream drained): the cycle's Hessenberg matrix, solution y and right-hand side give the
// harmonic Ritz vectors to keep (dr_setup); the kept block of H, its QR factors and the
// free-pressure sums go to the cycle state, and the basis is recombined in place.  *kk: the
// vectors the next cycle starts with (0: a plain restart; nothing was changed).
template <typename T>
int dr_restart(vms_ctx* c, int m, int j0, int deflate, hipStream_t s, int* kk) {
    constexpr int ld = kMaxRestart + 1;
    *kk = 0;
    GmresState* h = reinterpret_cast<GmresState*>(c->dr_pinned);
    double* up = reinterpret_cast<double*>(reinterpret_cast<char*>(c->dr_pinned) + kDrStateBytes);
    const size_t tail = offsetof(GmresState, y);
    int rc = check_hip(c, hipMemcpyAsync(h->H, c->gs->H, sizeof(double) * (size_t)m * ld, hipMemcpyDeviceToHost, s),
                       "read Hessenberg matrix");
    if (!rc)
        rc = check_hip(c, hipMemcpyAsync(reinterpret_cast<char*>(h) + tail, reinterpret_cast<char*>(c->gs) + tail,
                                         sizeof(GmresState) - tail, hipMemcpyDeviceToHost, s),
                       "read cycle state");
    if (!rc) rc = check_hip(c, hipStreamSynchronize(s), "sync");
    if (rc) return rc;
    const double rho = h->rho;
    if (!(rho > 0.0) || !std::isfinite(rho)) return VMS_OK;
    // Hbar (m+1) x m, entries below each column's last row cleared: the kept block's columns end
    // at row j0, an Arnoldi column j at row j + 1
    std::vector<double> Hb((size_t)(m + 1) * m, 0.0);
    for (int j = 0; j < m; ++j) {
        const int last = j < j0 ? j0 : j + 1;
        for (int i = 0; i <= last; ++i) Hb[(size_t)j * (m + 1) + i] = h->H[(size_t)j * ld + i];
    }
    // rc = c - Hbar y, c = beta e_1 (plain cycle) or beta (s, rho) in the kept basis
    std::vector<double> rcv(m + 1, 0.0);
    if (j0 > 0)
        for (int i = 0; i <= j0; ++i) rcv[i] = h->dr_c[i];
    else
        rcv[0] = h->beta;
    for (int j = 0; j < m; ++j)
        for (int i = 0; i <= m; ++i) rcv[i] -= Hb[(size_t)j * (m + 1) + i] * h->y[j];
    DrSetup S;
    const int k = dr_setup(m, deflate, Hb.data(), m + 1, rcv.data(), &S);
    if (k <= 0 || k >= m || k > kDrMax) return VMS_OK;
    // P for the stored basis: V[m] holds u_m, whose final vector is q_m = (u_m - V s) / rho
    const int mp = m + 1;
    for (int col = 0; col < k; ++col) {
        const double pm = S.P[(size_t)col * mp + m];
        for (int l = 0; l < m; ++l) up[col * mp + l] = S.P[(size_t)col * mp + l] - pm * h->scoef[l] / rho;
        up[col * mp + m] = pm / rho;
        double sv = 0.0;
        for (int l = 0; l <= m; ++l) sv += S.P[(size_t)col * mp + l] * h->svs[l];
        up[kDrOffSvs + col] = sv;
    }
    std::copy(S.Hk.begin(), S.Hk.end(), up + kDrOffH);
    std::copy(S.R.begin(), S.R.end(), up + kDrOffR);
    std::copy(S.Qt.begin(), S.Qt.end(), up + kDrOffQt);
    if ((rc = check_hip(c, hipMemcpyAsync(c->dr_p, up, sizeof(double) * kDrUpload, hipMemcpyHostToDevice, s),
                        "upload deflation data")))
        return rc;
    dr_load_kernel<<<1, kBlock, 0, s>>>(k, c->dr_p, c->gs);
    const int n = 4 * c->n_nodes;
    launch_dr_basis<T>(n, mp, k, c->dr_p, mp, basis_vectors<T>(c, 0), s);
    c->dr_k_dev = k;
    *kk = k;
    return check_hip(c, hipGetLastError(), "deflation launch");
}

// Switch deflated restarting off for the next cycle.
void dr_off(vms_ctx* c, hipStream_t s) {
    if (c->dr_k_dev == 0) return;
    dr_load_kernel<<<1, kBlock, 0, s>>>(0, c->dr_p, c->gs);
    c->dr_k_dev = 0;
}

}  // namespace

int launch_fill(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return VMS_OK;
    if (bytes % 16 != 0 || ((uintptr_t)p % 16) != 0) {
        // every buffer of the library is a multiple of 16 bytes and 16-byte aligned
        return set_error(nullptr, VMS_EINVAL, "fill: unaligned buffer");
    }
    const size_t n16 = bytes / 16;
    const int g = (int)std::min<size_t>((n16 + kBlock - 1) / kBlock, 8192);
    fill_kernel<<<g, kBlock, 0, s>>>((uint4*)p, n16);
    return VMS_OK;
}

int launch_spmv(vms_ctx* c, const void* A, const void* x, void* y, hipStream_t s) {
    const int n = 4 * c->n_nodes;
    if (c->prec == VMS_FP64)
        spmv_kernel<double, double, double, double, 0><<<spmv_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const double*)A, (const double*)x, (const double*)nullptr, (double*)y, nullptr, nullptr);
    else
        spmv_kernel<float, float, float, float, 0><<<spmv_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const float*)A, (const float*)x, (const double*)nullptr, (float*)y, nullptr, nullptr);
    return check_hip(c, hipGetLastError(), "spmv launch");
}

int launch_bj_setup(vms_ctx* c, const void* A, void* Minv, hipStream_t s) {
    zero_count_kernel<<<1, 64, 0, s>>>(c->flags + 2);      // singular blocks of this setup
    PhaseScope ph(c, VMS_PH_PCSETUP, (double)c->n_nodes * (32.0 * elt_size(c) + 4.0), s);
    if (c->prec == VMS_FP64)
        bj_setup_kernel<double, double><<<grid_for(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->diagpos,
                                                                              (const double*)A, (double*)Minv,
                                                                              c->flags);
    else
        bj_setup_kernel<float, float><<<grid_for(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->diagpos,
                                                                            (const float*)A, (float*)Minv,
                                                                            c->flags);
    return check_hip(c, hipGetLastError(), "bj setup launch");
}

// Block-Jacobi for the uncondensed system: K_ff^-1 on element rows, the Schur diagonal
// inverse on node rows.
static int launch_full_pc_setup(vms_ctx* c, const void* A, void* Minv, hipStream_t s) {
    int rc = launch_bj_setup(c, A, Minv, s);
    if (rc) return rc;
    const int nn = c->full_nodes;
    if (c->prec == VMS_FP64)
        schur_diag_pc_kernel<double, double><<<grid_for(nn), kBlock, 0, s>>>(
            nn, c->rowptr, c->colidx, c->diagpos, (const double*)A, (double*)Minv, c->flags);
    else
        schur_diag_pc_kernel<float, float><<<grid_for(nn), kBlock, 0, s>>>(
            nn, c->rowptr, c->colidx, c->diagpos, (const float*)A, (float*)Minv, c->flags);
    return check_hip(c, hipGetLastError(), "schur diagonal setup launch");
}

// A P and A z for the Arnoldi steps (after the preconditioner blocks are set).
int launch_ap_setup(vms_ctx* c, const void* A, hipStream_t s) {
    const double es = elt_size(c);
    PhaseScope ph(c, VMS_PH_PCAPPLY, (double)c->nb * (32.0 * es + 4.0) + (double)c->n_nodes * 16.0 * es, s);
    const int g = (int)((4 * c->nb + kBlock - 1) / kBlock);
    if (c->prec == VMS_FP64) {
        ap_blocks_kernel<double><<<g, kBlock, 0, s>>>(c->nb, c->colidx, (const double*)A, (const double*)c->Minv,
                                                     (double*)c->AP);
        if (c->zfull)
            spmv_kernel<double, double, double, double, 0><<<spmv_grid(c->n_nodes), kBlock, 0, s>>>(
                c->n_nodes, c->rowptr, c->colidx, (const double*)A, c->zfull, (const double*)nullptr,
                (double*)c->Az, nullptr, nullptr);
        else
            coarse_column_kernel<double><<<grid_for(4 * (int64_t)c->n_nodes), kBlock, 0, s>>>(
                c->n_nodes, c->rowptr, c->colidx, (const double*)A, c->dmask, (double*)c->Az);
    } else {
        ap_blocks_kernel<float><<<g, kBlock, 0, s>>>(c->nb, c->colidx, (const float*)A, (const float*)c->Minv,
                                                    (float*)c->AP);
        if (c->zfull)
            spmv_kernel<float, double, float, double, 0><<<spmv_grid(c->n_nodes), kBlock, 0, s>>>(
                c->n_nodes, c->rowptr, c->colidx, (const float*)A, c->zfull, (const double*)nullptr,
                (float*)c->Az, nullptr, nullptr);
        else
            coarse_column_kernel<float><<<grid_for(4 * (int64_t)c->n_nodes), kBlock, 0, s>>>(
                c->n_nodes, c->rowptr, c->colidx, (const float*)A, c->dmask, (float*)c->Az);
    }
    return check_hip(c, hipGetLastError(), "A P setup launch");
}

// FP64 residual r64 = b - A x and its norm (synchronising).
static int true_residual(vms_ctx* c, const void* A, const double* b, const double* x, double* rn, hipStream_t s) {
    const int n = 4 * c->n_nodes;
    if (c->prec == VMS_FP64)
        spmv_kernel<double, double, double, double, 1><<<spmv_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const double*)A, x, b, c->r64, nullptr, nullptr);
    else
        spmv_kernel<float, double, double, double, 1><<<spmv_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const float*)A, x, b, c->r64, nullptr, nullptr);
    launch_norm<double>(c, n, c->r64, 0, s);
    return read_scalar(c, 0, rn, s);
}

int gmres_solve(vms_ctx* c, const void* A, const double* b, double* x, const vms_solve_opts* o,
                vms_solve_info* info, hipStream_t s) {
    const int n = 4 * c->n_nodes;
    vms_solve_info inf{};
    const int m = o->restart > 0 ? std::min(o->restart, c->max_restart) : c->max_restart;
    const int max_iters = o->max_iters > 0 ? o->max_iters : 100000;
    const double rtol = o->rtol > 0 ? o->rtol : 1e-8;
    const int refine_max = o->refine_max > 0 ? o->refine_max : 30;
    // mixed ctx: inner_rtol <= 0 restarts every FP32 cycle from the FP64 residual; a positive
    // value runs FP32 restart cycles on the FP32 residual until it falls below inner_rtol
    const bool sweeps = o->inner_rtol > 0;
    const double inner_rtol = o->inner_rtol;
    // deflated restarting keeps part of every full cycle's basis; it needs the second
    // Gram-Schmidt pass (the cycle's residual is orthogonalised against the kept vectors)
    // mixed ctx with an FP64 basis: FP64 cycles on the FP32-stored matrix and preconditioner
    const bool basis64 = c->prec != VMS_FP64 && o->basis_fp64;
    const int deflate = o->deflate;
    if (deflate != 0) {
        if (deflate < 0 || deflate > kDrMax - 1 || deflate > m - 2)
            return set_error(c, VMS_EINVAL, "gmres: deflate must lie in 1 .. min(32, restart - 2)");
        if (c->prec != VMS_FP64 && !basis64 && sweeps)
            return set_error(c, VMS_EINVAL, "gmres: deflate needs inner_rtol <= 0");
        if (c->full_nodes > 0)
            return set_error(c, VMS_EINVAL, "gmres: deflate is for condensed systems only");
    }
    const int cgs2 = deflate > 0 ? 1 : o->cgs2;
    int rc;
    if (basis64 && !c->V64)
        return set_error(c, VMS_EINVAL, "gmres: basis_fp64 needs a context created with basis_fp64");
    // the constant-pressure coarse mode exists only when a pressure dof is prescribed
    const int coarse_pressure = o->coarse_pressure && c->n_pressure_pins > 0;

    // preconditioner blocks
    if (o->pc == VMS_PC_LEARNED && o->pc_weights) {
        rc = learned_blocks(c, A, o->pc_weights, c->Minv, c->prec == VMS_FP64, s);
        if (rc == VMS_ENONFINITE) {
            inf.fell_back_to_bj = 1;
            if ((rc = launch_bj_setup(c, A, c->Minv, s))) return rc;
        } else if (rc) {
            return rc;
        }
    } else if (c->full_nodes > 0) {
        if ((rc = launch_full_pc_setup(c, A, c->Minv, s))) return rc;
    } else {
        if ((rc = launch_bj_setup(c, A, c->Minv, s))) return rc;
    }
    if (c->zfull) {
        const int nn = c->full_nodes;
        if (c->prec == VMS_FP64) {
            full_coarse_vector_kernel<double, double><<<grid_for(c->n_nodes), kBlock, 0, s>>>(
                nn, c->n_nodes, c->rowptr, c->colidx, (const double*)A, (const double*)c->Minv, c->dmask, c->zfull);
            full_coarse_setup_kernel<double><<<red_grid(nn), kBlock, 0, s>>>(
                nn, c->rowptr, c->colidx, (const double*)A, c->dmask, c->zfull, coarse_pressure, c->red, c->gs);
        } else {
            full_coarse_vector_kernel<float, float><<<grid_for(c->n_nodes), kBlock, 0, s>>>(
                nn, c->n_nodes, c->rowptr, c->colidx, (const float*)A, (const float*)c->Minv, c->dmask, c->zfull);
            full_coarse_setup_kernel<float><<<red_grid(nn), kBlock, 0, s>>>(
                nn, c->rowptr, c->colidx, (const float*)A, c->dmask, c->zfull, coarse_pressure, c->red, c->gs);
        }
    } else if (c->prec == VMS_FP64) {
        coarse_setup_kernel<double><<<red_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const double*)A, c->dmask, coarse_pressure, c->red, c->gs);
    } else {
        coarse_setup_kernel<float><<<red_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const float*)A, c->dmask, coarse_pressure, c->red, c->gs);
    }
    if ((rc = launch_ap_setup(c, A, s))) return rc;
    launch_norm<double>(c, n, b, 1, s);
    double bn = 0.0;
    if ((rc = read_scalar(c, 1, &bn, s))) return rc;
    if (!std::isfinite(bn)) return set_error(c, VMS_ENONFINITE, "gmres: non-finite right-hand side");
    // singular diagonal blocks of the preconditioner setup (applied as the identity), read
    // once the stream is drained at the end of the call
    int32_t singular = 0;
    auto read_singular = [&]() {
        return check_hip(c, hipMemcpyAsync(&singular, c->flags + 2, sizeof singular, hipMemcpyDeviceToHost, s),
                         "read singular-block count");
    };
    if (bn == 0.0) {
        if ((rc = launch_fill(x, n * sizeof(double), s))) return rc;
        if ((rc = read_singular())) return rc;
        if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
        inf.true_rel_res = 0.0;
        inf.singular_blocks = singular;
        if (info) *info = inf;
        return VMS_OK;
    }
    const double tol = rtol * bn;
    double rn = 0.0;
    int iters = 0;
    int status = VMS_OK;
    const bool learned = o->pc == VMS_PC_LEARNED && o->pc_weights && !inf.fell_back_to_bj;
    const int learned_budget = learned ? max_iters / 2 : max_iters;
    bool using_learned = learned;
    bool pending = false;          // an FP64 cycle was launched and not yet counted
    int j0 = 0;                    // vectors the cycle in flight kept from its predecessor
    bool dr_ready = false;         // the last cycle ran all its steps: its basis can be deflated
    bool dr_live = deflate > 0;    // deflation still in use in this solve
    double rn_start = 0.0;         // true residual before the cycle in flight
    dr_off(c, s);
    for (;;) {
        if ((rc = true_residual(c, A, b, x, &rn, s))) return rc;      // synchronises
        int last_k = -1;
        if (pending) {
            int stopped = 0;
            last_k = finish_cycle(c, &stopped);
            iters += last_k - j0;
            inf.restarts++;
            pending = false;
            dr_ready = dr_live && last_k == m && !stopped;
            if (j0 > 0 && !(rn <= rn_start)) {
                // A deflated cycle cannot raise the residual in exact arithmetic (y = 0 is
                // feasible); when it does, the kept block's Arnoldi relation has drifted from the
                // stored vectors (in FP32 storage the rounding of the recombined basis adds up
                // over cycles).  Its correction is undone and the solve restarts plainly.
                if ((rc = check_hip(c, hipMemcpyAsync(x, c->x64, sizeof(double) * n, hipMemcpyDeviceToDevice, s),
                                    "restore iterate")))
                    return rc;
                if ((rc = true_residual(c, A, b, x, &rn, s))) return rc;
                dr_live = dr_ready = false;
                inf.deflation_stopped = 1;
            }
        }
        if (o->log_residuals && inf.logged < o->log_max) {
            convert_kernel<double, float><<<grid_for(n), kBlock, 0, s>>>(
                n, c->r64, o->log_residuals + (size_t)inf.logged * n, 1.0);
            inf.logged++;
        }
        if (!std::isfinite(rn)) {
            status = set_error(c, VMS_ENONFINITE, "gmres: non-finite residual");
            break;
        }
        if (rn <= tol) break;
        if (last_k == 0) {
            status = set_error(c, VMS_ENOCONV_GMRES, "gmres: stagnation (no Arnoldi progress)");
            break;
        }
        if (iters >= max_iters) {
            status = set_error(c, VMS_ENOCONV_GMRES, "gmres: iteration cap reached before rtol");
            break;
        }
        if (using_learned && iters >= learned_budget) {
            // the learned blocks did not deliver within half the budget: continue from the
            // current iterate with plain block-Jacobi
            if ((rc = launch_bj_setup(c, A, c->Minv, s))) return rc;
            if ((rc = launch_ap_setup(c, A, s))) return rc;
            using_learned = false;
            inf.fell_back_to_bj = 1;
            dr_ready = false;      // the kept basis belongs to the old operator
        }
        // the next cycle's kept vectors (0: a plain restart)
        int kk = 0;
        if (dr_ready) {
            rc = (c->prec == VMS_FP64 || basis64) ? dr_restart<double>(c, m, j0, deflate, s, &kk)
                                                   : dr_restart<float>(c, m, j0, deflate, s, &kk);
            if (rc) return rc;
            dr_ready = false;
        }
        if (kk == 0) dr_off(c, s);
        j0 = kk;
        rn_start = rn;
        if (j0 > 0 &&
            (rc = check_hip(c, hipMemcpyAsync(c->x64, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "save iterate")))
            return rc;
        // while the learned blocks are on trial, no cycle runs past half of the budget, so that
        // the switch to block-Jacobi above happens there
        const int cap = using_learned ? learned_budget : max_iters;
        if (c->prec == VMS_FP64) {
            // one restart cycle on the FP64 residual; the true residual is recomputed above
            if ((rc = run_cycle<double, double>(c, c->r64, (const double*)c->Minv, x, tol, m, cap - iters,
                                                cgs2, s, 1.0, j0)))
                return rc;
            pending = true;
        } else if (basis64) {
            // the same on the FP32-stored matrix and preconditioner, applied one after the other
            // (the stored A P blocks are rounded products, not the operator the residual sees)
            if ((rc = run_cycle<double, double, float>(c, c->r64, (const float*)c->Minv, x, tol, m, cap - iters,
                                                       cgs2, s, 1.0, j0, (const float*)A)))
                return rc;
            pending = true;
        } else if (!sweeps) {
            // FP64 refinement at every restart: one FP32 cycle on A d = r / ||r|| (r = b - A x in FP64,
            // A the FP32-stored matrix), its correction added to the FP64 x as ||r|| P V y.  Every
            // cycle thus starts from a residual that is exact to FP32 rounding of a unit vector; a
            // residual recomputed in FP32 from an FP32 correction carries an error near
            // eps32 |A| |d|, which on hard systems the following cycles spend their steps on.
            inf.refinements++;
            float* rr = (float*)c->r;
            convert_kernel<double, float><<<grid_for(n), kBlock, 0, s>>>(n, c->r64, rr, 1.0 / rn);
            if ((rc = run_cycle<float, double>(c, rr, (const float*)c->Minv, x, tol / rn, m, cap - iters, cgs2,
                                               s, rn, j0)))
                return rc;
            pending = true;
        } else {
            // FP64 iterative refinement: FP32 restarted GMRES on A d = r / ||r||, then x += ||r|| d
            if (inf.refinements >= refine_max) {
                status = set_error(c, VMS_ENOCONV_GMRES, "gmres: refinement cap reached before rtol");
                break;
            }
            inf.refinements++;
            float* rr = (float*)c->r;      // unit-norm residual of this sweep
            float* d = (float*)c->d;       // FP32 correction
            float* q = c->tvec;            // inner residual rr - A d
            convert_kernel<double, float><<<grid_for(n), kBlock, 0, s>>>(n, c->r64, rr, 1.0 / rn);
            if ((rc = launch_fill(d, n * sizeof(float), s))) return rc;
            // one sweep is asked for 0.9 of the remaining reduction (never below inner_rtol)
            const double inner_tol = std::max(inner_rtol, 0.9 * tol / rn);
            const float* cycle_r = rr;
            int progress = 0;
            while (iters < cap) {
                if ((rc = run_cycle<float, float>(c, cycle_r, (const float*)c->Minv, d, inner_tol, m,
                                                  cap - iters, cgs2, s)))
                    return rc;
                spmv_kernel<float, float, float, float, 1, float><<<spmv_grid(c->n_nodes), kBlock, 0, s>>>(
                    c->n_nodes, c->rowptr, c->colidx, (const float*)A, d, rr, q, nullptr, nullptr);
                launch_norm<float>(c, n, q, 2, s);
                double qn = 0.0;
                if ((rc = read_scalar(c, 2, &qn, s))) return rc;     // synchronises
                int stopped = 0;
                const int k = finish_cycle(c, &stopped);
                iters += k;
                progress += k;
                inf.restarts++;
                if (k == 0) break;
                if (o->log_residuals && inf.logged < o->log_max) {
                    convert_kernel<float, float><<<grid_for(n), kBlock, 0, s>>>(
                        n, q, o->log_residuals + (size_t)inf.logged * n, 1.0);
                    inf.logged++;
                }
                if (!(qn > inner_tol) || !std::isfinite(qn)) break;
                // The FP32 inner residual has a rounding floor near eps32 |A| |d|: when the cycle's own
                // estimate reached inner_tol but the recomputed residual did not, the sweep ends and the
                // FP64 refinement continues from the new iterate.
                if (stopped) break;
                cycle_r = q;
            }
            axpy64_kernel<float><<<grid_for(n), kBlock, 0, s>>>(n, rn, d, x);
            if (progress == 0) {
                status = set_error(c, VMS_ENOCONV_GMRES, "gmres: stagnation (no Arnoldi progress)");
                break;
            }
        }
    }
    // the per-cycle reads above wait only for their norms; the call returns with the stream drained
    if (int rs = read_singular()) return rs;
    if (int rs = check_hip(c, hipStreamSynchronize(s), "sync")) return rs;
    inf.singular_blocks = singular;
    inf.iters = iters;
    inf.true_rel_res = rn / bn;
    if (info) *info = inf;
    return status;
}

}  // namespace vms

using namespace vms;

extern "C" int vms_bsr_spmv(vms_ctx* c, const void* bsr_vals, const void* x, void* y, hipStream_t s) {
    if (!c || !bsr_vals || !x || !y) return set_error(c, VMS_EINVAL, "vms_bsr_spmv: NULL argument");
    return launch_spmv(c, bsr_vals, x, y, s);
}

extern "C" int vms_gmres_solve(vms_ctx* c, const void* bsr_vals, const double* b, double* x,
                               const vms_solve_opts* opts, vms_solve_info* info, hipStream_t s) {
    if (!c || !bsr_vals || !b || !x || !opts) return set_error(c, VMS_EINVAL, "vms_gmres_solve: NULL argument");
    if (opts->restart > c->max_restart)
        return set_error(c, VMS_EINVAL, "vms_gmres_solve: restart exceeds the allocated basis");
    return gmres_solve(c, bsr_vals, b, x, opts, info, s);
}
