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
// by the last workgroup of each reduction, so an Arnoldi step is a fixed
// sequence of launches with no host round trip; the host looks at the
// convergence flag only every few steps.
#include <cstdio>
#include <vector>

#include "vms_internal.h"

namespace vms {
namespace {

inline int grid_for(int64_t n, int block = kBlock) { return (int)((n + block - 1) / block); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

__global__ void fill_kernel(uint4* p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------------- SpMV
// Four lanes per block row; lane r owns output dof r of its node and walks the
// row's blocks, reading row r of each block (4 contiguous values) and the
// 4-vector of the column node.  MODE 0: y = A x.  MODE 1: y = b - A x.
template <typename TA, typename TX, typename TY, typename TACC, int MODE, typename TB = double>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int n_rows, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const TA* __restrict__ A, const TX* __restrict__ x,
                                                      const TB* __restrict__ b, TY* __restrict__ y,
                                                      const int* __restrict__ done) {
    if (done && *done) return;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = tid >> 2;
    const int r = tid & 3;
    if (row >= n_rows) return;
    using VA = typename Vec4<TA>::type;
    using VX = typename Vec4<TX>::type;
    TACC acc = TACC(0);
    const int k0 = rowptr[row], k1 = rowptr[row + 1];
    for (int k = k0; k < k1; ++k) {
        const int col = colidx[k];
        const VA a = *reinterpret_cast<const VA*>(A + (size_t)k * 16 + r * 4);
        const VX xv = *reinterpret_cast<const VX*>(x + (size_t)col * 4);
        acc += TACC(a.x) * TACC(xv.x) + TACC(a.y) * TACC(xv.y) + TACC(a.z) * TACC(xv.z) +
               TACC(a.w) * TACC(xv.w);
    }
    if (MODE == 1)
        y[4 * (size_t)row + r] = TY(TACC(b[4 * (size_t)row + r]) - acc);
    else
        y[4 * (size_t)row + r] = TY(acc);
}

// --------------------------------------------------------------------------- block-Jacobi
// Inverse of each 4x4 diagonal block in FP64 (Gauss-Jordan, partial pivoting),
// stored in the preconditioner precision.  A singular block is replaced by the
// identity and counted in flags[2].
template <typename TA, typename TM>
__global__ void bj_setup_kernel(int n, const int32_t* __restrict__ diagpos, const TA* __restrict__ A,
                                TM* __restrict__ Minv, int32_t* flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const TA* D = A + (size_t)diagpos[i] * 16;
    double m[4][8];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            m[r][c] = double(D[r * 4 + c]);
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
    TM* out = Minv + (size_t)i * 16;
    if (!ok) atomicAdd(&flags[2], 1);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) out[r * 4 + c] = ok ? TM(m[r][4 + c]) : TM(r == c ? 1 : 0);
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
template <typename TA>
__global__ __launch_bounds__(kBlock) void coarse_setup_kernel(int n_nodes, const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ colidx,
                                                              const TA* __restrict__ A,
                                                              const uint8_t* __restrict__ dmask, int enabled,
                                                              RedScratch* red, GmresState* gs) {
    __shared__ double lds[kBlock / 64];
    double v[1] = {0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes; i += gridDim.x * blockDim.x) {
        if (dmask[i] & 8u) continue;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (!(dmask[colidx[k]] & 8u)) v[0] += double(A[(size_t)k * 16 + 15]);
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) red->partial[blockIdx.x] = v[0];
    if (!arrive_last(&red->counter)) return;
    __threadfence();
    __shared__ double tot;
    reduce_partials(red->partial, kRedBlocks, 1, gridDim.x, &tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        gs->kappa = (enabled && tot != 0.0 && isfinite(tot)) ? 1.0 / tot : 0.0;
        red->counter = 0u;
    }
}

// norm of a vector -> gs->beta, initialises the cycle (g = beta e_1, k = 0, done flag).
template <typename T>
__global__ __launch_bounds__(kBlock) void cycle_start_kernel(int n, const T* __restrict__ r,
                                                             const uint8_t* __restrict__ dmask, RedScratch* red,
                                                             GmresState* gs, double tol_abs) {
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
        gs->sv = nrm > 0.0 ? tot[1] / nrm : 0.0;
        gs->beta = nrm;
        gs->g[0] = nrm;
        gs->k = 0;
        gs->tol_abs = tol_abs;
        gs->done = (nrm <= tol_abs || !(nrm > 0.0)) ? 1 : 0;
        gs->norm = nrm;
        red->counter = 0u;
    }
}

// V[0] = r / beta
template <typename T>
__global__ void cycle_v0_kernel(int n, const T* __restrict__ r, T* __restrict__ V0, const GmresState* gs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double b = gs->beta;
    V0[i] = b > 0.0 ? T(double(r[i]) / b) : T(0);
}

// Arnoldi step j, part 1: v_j = w / h(j, j-1) (j > 0), z = Minv v_j.
template <typename T>
__global__ void arnoldi_pc_kernel(int n_nodes, int j, T* __restrict__ V, const T* __restrict__ w,
                                  const T* __restrict__ Minv, const uint8_t* __restrict__ dmask, T* __restrict__ z,
                                  const GmresState* gs) {
    if (gs->done) return;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = tid >> 2, r = tid & 3;
    if (node >= n_nodes) return;
    const size_t N = 4 * (size_t)n_nodes;
    using V4 = typename Vec4<T>::type;
    T* vj = V + (size_t)j * N;
    V4 v4;
    if (j > 0) {
        const double h = gs->H[j + (j - 1) * (kMaxRestart + 1)];
        const double ih = 1.0 / h;
        const V4 w4 = *reinterpret_cast<const V4*>(w + 4 * (size_t)node);
        v4.x = T(double(w4.x) * ih);
        v4.y = T(double(w4.y) * ih);
        v4.z = T(double(w4.z) * ih);
        v4.w = T(double(w4.w) * ih);
        const T mine = r == 0 ? v4.x : r == 1 ? v4.y : r == 2 ? v4.z : v4.w;
        vj[4 * (size_t)node + r] = mine;
    } else {
        v4 = *reinterpret_cast<const V4*>(vj + 4 * (size_t)node);
    }
    const V4 m = *reinterpret_cast<const V4*>(Minv + (size_t)node * 16 + r * 4);
    T zz = m.x * v4.x + m.y * v4.y + m.z * v4.z + m.w * v4.w;
    if (r == 3 && !(dmask[node] & 8u)) zz += T(gs->kappa * gs->sv);
    z[4 * (size_t)node + r] = zz;
}

// Classical Gram-Schmidt dots: h_i = V_i . w for i <= j.  Grid (chunks, groups of 8
// vectors); each workgroup writes 8 partial sums, the last one to arrive sums all partials in
// a fixed order into gs->hcol.
constexpr int kDotVecs = 8;
constexpr int kDotItems = 4;     // elements per thread per pass

template <typename T>
__global__ __launch_bounds__(kBlock) void cgs_dots_kernel(int n, int j, const T* __restrict__ V,
                                                          const T* __restrict__ w, RedScratch* red,
                                                          GmresState* gs) {
    if (gs->done) return;
    __shared__ double lds[(kBlock / 64) * kDotVecs];
    const size_t N = (size_t)n;
    const int i0 = blockIdx.y * kDotVecs;
    const int nv = min(kDotVecs, j + 1 - i0);
    double acc[kDotVecs];
#pragma unroll
    for (int q = 0; q < kDotVecs; ++q) acc[q] = 0.0;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x + threadIdx.x; base < n; base += stride * kDotItems) {
        double wv[kDotItems];
#pragma unroll
        for (int it = 0; it < kDotItems; ++it) {
            const int idx = base + it * stride;
            wv[it] = idx < n ? double(w[idx]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kDotVecs; ++q) {
            if (q < nv) {
                const T* vq = V + (size_t)(i0 + q) * N;
#pragma unroll
                for (int it = 0; it < kDotItems; ++it) {
                    const int idx = base + it * stride;
                    if (idx < n) acc[q] += double(vq[idx]) * wv[it];
                }
            }
        }
    }
    block_sum<kDotVecs>(acc, lds);
    const int nblk = gridDim.x * gridDim.y;
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < kDotVecs; ++q)
            if (q < nv) red->partial[(size_t)(i0 + q) * kRedBlocks + blockIdx.x] = acc[q];
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(&red->counter, 1u);
        last = prev == (unsigned)nblk - 1;
    }
    __syncthreads();
    (void)bid;
    if (last) {
        __threadfence();
        reduce_partials(red->partial, kRedBlocks, j + 1, gridDim.x, gs->hcol);
        __syncthreads();
        if (threadIdx.x == 0) red->counter = 0u;
    }
}

// w -= sum_i hcol_i V_i; ||w||^2 partials; the last workgroup adds hcol into
// column j of H and, on the final pass, sets h(j+1, j), applies the Givens
// rotations and updates the residual estimate and the done flag.
template <typename T>
__global__ __launch_bounds__(kBlock) void cgs_update_kernel(int n, int j, const T* __restrict__ V,
                                                            T* __restrict__ w, const uint8_t* __restrict__ dmask,
                                                            RedScratch* red, GmresState* gs, int first_pass,
                                                            int final_pass) {
    if (gs->done) return;
    __shared__ double hs[kMaxRestart + 1];
    __shared__ double lds[(kBlock / 64) * 2];
    for (int i = threadIdx.x; i <= j; i += blockDim.x) hs[i] = gs->hcol[i];
    __syncthreads();
    const size_t N = (size_t)n;
    double v[2] = {0.0, 0.0};
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
        double s = double(w[idx]);
        int i = 0;
        // groups of 8 independent loads keep several memory requests in flight per lane
        for (; i + 8 <= j + 1; i += 8) {
            double vv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) vv[q] = double(V[(size_t)(i + q) * N + idx]);
#pragma unroll
            for (int q = 0; q < 8; ++q) s -= hs[i + q] * vv[q];
        }
        for (; i <= j; ++i) s -= hs[i] * double(V[(size_t)i * N + idx]);
        const T sv = T(s);
        w[idx] = sv;
        v[0] += double(sv) * double(sv);
        if (free_pressure(dmask, idx)) v[1] += double(sv);
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        red->partial[blockIdx.x] = v[0];
        red->partial[kRedBlocks + blockIdx.x] = v[1];
    }
    if (!arrive_last(&red->counter)) return;
    __threadfence();
    constexpr int ld = kMaxRestart + 1;
    __shared__ double col[kMaxRestart + 2], csl[kMaxRestart], snl[kMaxRestart];
    __shared__ double tot[2];
    double* Hj = gs->H + (size_t)j * ld;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        const double h = first_pass ? hs[i] : Hj[i] + hs[i];
        Hj[i] = h;
        col[i] = h;
    }
    if (final_pass) {
        for (int i = threadIdx.x; i < j; i += blockDim.x) {
            csl[i] = gs->cs[i];
            snl[i] = gs->sn[i];
        }
        reduce_partials(red->partial, kRedBlocks, 2, gridDim.x, tot);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (final_pass) {
            const double hn = sqrt(tot[0]);
            Hj[j + 1] = hn;
            gs->sv = hn > 0.0 ? tot[1] / hn : 0.0;   // free-pressure sum of the next basis vector
            // previous rotations on the new column: the running entry is carried in a register
            double* Rj = gs->R + (size_t)j * ld;
            double x = col[0];
            for (int i = 0; i < j; ++i) {
                const double y = col[i + 1];
                Rj[i] = csl[i] * x + snl[i] * y;
                x = -snl[i] * x + csl[i] * y;
            }
            const double d = hypot(x, hn);
            const double cs = d > 0.0 ? x / d : 1.0;
            const double sn = d > 0.0 ? hn / d : 0.0;
            gs->cs[j] = cs;
            gs->sn[j] = sn;
            Rj[j] = d;
            const double gj = gs->g[j];
            gs->g[j + 1] = -sn * gj;
            gs->g[j] = cs * gj;
            gs->k = j + 1;
            const bool conv = fabs(gs->g[j + 1]) <= gs->tol_abs;
            const bool breakdown = !(hn > 1e-300 * (fabs(d) + 1e-300)) || !isfinite(hn);
            if (conv || breakdown || !isfinite(gs->g[j + 1])) gs->done = 1;
        }
        red->counter = 0u;
    }
}

// t = sum_{i<k} y_i V_i
template <typename T>
__global__ void combine_kernel(int n, const T* __restrict__ V, const GmresState* gs, T* __restrict__ t) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int k = gs->k;
    const size_t N = (size_t)n;
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += gs->y[i] * double(V[(size_t)i * N + idx]);
    t[idx] = T(s);
}

// gs->st = sum of the free pressure entries of t (for the coarse term of P t)
template <typename T>
__global__ __launch_bounds__(kBlock) void free_pressure_sum_kernel(int n_nodes, const T* __restrict__ t,
                                                                   const uint8_t* __restrict__ dmask,
                                                                   RedScratch* red, GmresState* gs) {
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

// x += P t = Minv t + z kappa (z^T t)  (x in TX: double for the FP64 solution, float for an inner correction)
template <typename T, typename TX>
__global__ void precond_accumulate_kernel(int n_nodes, const T* __restrict__ Minv, const T* __restrict__ t,
                                          const uint8_t* __restrict__ dmask, const GmresState* gs,
                                          TX* __restrict__ x) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = tid >> 2, r = tid & 3;
    if (node >= n_nodes) return;
    using V4 = typename Vec4<T>::type;
    const V4 m = *reinterpret_cast<const V4*>(Minv + (size_t)node * 16 + r * 4);
    const V4 v = *reinterpret_cast<const V4*>(t + 4 * (size_t)node);
    double s = double(m.x) * double(v.x) + double(m.y) * double(v.y) + double(m.z) * double(v.z) +
               double(m.w) * double(v.w);
    if (r == 3 && !(dmask[node] & 8u)) s += gs->kappa * gs->st;
    x[4 * (size_t)node + r] = TX(double(x[4 * (size_t)node + r]) + s);
}

// FP64 norm of a vector of any precision into out (device) via partials.
template <typename T>
__global__ __launch_bounds__(kBlock) void norm_kernel(int n, const T* __restrict__ r, RedScratch* red,
                                                      double* out) {
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
        out[0] = sqrt(tot);
        red->counter = 0u;
    }
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

inline int red_grid(int64_t n) { return std::max(1, std::min(kRedBlocks, grid_for(n))); }

// Reads a device double with a stream sync.
int read_scalar(vms_ctx* c, const double* dptr, double* h, hipStream_t s) {
    int rc = check_hip(c, hipMemcpyAsync(h, dptr, sizeof(double), hipMemcpyDeviceToHost, s), "read scalar");
    if (rc) return rc;
    return check_hip(c, hipStreamSynchronize(s), "sync");
}

struct CycleStatus {
    int k;
    int done;
};

// One GMRES(m) cycle on A d = r0 with right preconditioner Minv; the Krylov
// correction Minv (V y) is added to x (double or float).  r0 is the cycle's
// initial residual (precision T).  Returns the number of Arnoldi steps.
template <typename T, typename TX>
int run_cycle(vms_ctx* c, const T* A, const T* r0, const T* Minv, TX* x, double tol_abs, int m, int budget,
              int cgs2, CycleStatus* st, hipStream_t s) {
    const int n = 4 * c->n_nodes;
    T* V = (T*)c->V;
    T* w = (T*)c->w;
    T* z = (T*)c->z;
    cycle_start_kernel<T><<<red_grid(n), kBlock, 0, s>>>(n, r0, c->dmask, c->red, c->gs, tol_abs);
    cycle_v0_kernel<T><<<grid_for(n), kBlock, 0, s>>>(n, r0, V, c->gs);
    const int steps = std::min(m, budget);
    const int check_every = 5;
    const double vb = (double)n * sizeof(T);      // bytes of one Krylov vector
    const double spmv_bytes = (double)c->nb * (16.0 * sizeof(T) + 4.0) + 4.0 * (c->n_nodes + 1) + 2.0 * vb;
    for (int j = 0; j < steps; ++j) {
        {
            PhaseScope ph(c, VMS_PH_PCAPPLY, 3.0 * vb + 4.0 * vb, s);
            arnoldi_pc_kernel<T><<<grid_for(n), kBlock, 0, s>>>(c->n_nodes, j, V, w, Minv, c->dmask, z, c->gs);
        }
        {
            PhaseScope ph(c, VMS_PH_SPMV, spmv_bytes, s);
            spmv_kernel<T, T, T, T, 0><<<grid_for(n), kBlock, 0, s>>>(c->n_nodes, c->rowptr, c->colidx, A, z,
                                                                      (const double*)nullptr, w, &c->gs->done);
        }
        const int passes = cgs2 ? 2 : 1;
        for (int p = 0; p < passes; ++p) {
            {
                PhaseScope ph(c, VMS_PH_DOTS, (j + 2) * vb, s);
                const int groups = (j + kDotVecs) / kDotVecs;
                const int gx = std::max(1, std::min(kRedBlocks, std::min(grid_for(n, kBlock * kDotItems),
                                                                         std::max(1, 2048 / groups))));
                cgs_dots_kernel<T><<<dim3(gx, groups), kBlock, 0, s>>>(n, j, V, w, c->red, c->gs);
            }
            {
                PhaseScope ph(c, VMS_PH_UPDATE, (j + 3) * vb, s);
                cgs_update_kernel<T><<<std::min(kRedBlocks, grid_for(n)), kBlock, 0, s>>>(n, j, V, w, c->dmask, c->red,
                                                                                           c->gs, p == 0,
                                                                    p == passes - 1);
            }
        }
        if ((j + 1) % check_every == 0 || j + 1 == steps) {
            int h[2];
            if (check_hip(c, hipMemcpyAsync(h, &c->gs->k, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "read k"))
                return -1;
            if (check_hip(c, hipStreamSynchronize(s), "sync")) return -1;
            st->k = h[0];
            st->done = h[1];
            if (h[1]) break;
        }
    }
    if (st->k > 0) {
        // back substitution R y = g on the host (R is at most kMaxRestart square)
        const int k = st->k;
        constexpr int ld = kMaxRestart + 1;
        std::vector<double> R((size_t)k * ld), g(k), y(k);
        if (check_hip(c, hipMemcpyAsync(R.data(), c->gs->R, R.size() * sizeof(double), hipMemcpyDeviceToHost, s),
                      "read R") ||
            check_hip(c, hipMemcpyAsync(g.data(), c->gs->g, k * sizeof(double), hipMemcpyDeviceToHost, s), "read g") ||
            check_hip(c, hipStreamSynchronize(s), "sync"))
            return -1;
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int cc = i + 1; cc < k; ++cc) acc -= R[(size_t)cc * ld + i] * y[cc];
            y[i] = acc / R[(size_t)i * ld + i];
        }
        if (check_hip(c, hipMemcpyAsync(c->gs->y, y.data(), k * sizeof(double), hipMemcpyHostToDevice, s), "write y") ||
            check_hip(c, hipStreamSynchronize(s), "sync"))
            return -1;
        combine_kernel<T><<<grid_for(n), kBlock, 0, s>>>(n, V, c->gs, z);
        free_pressure_sum_kernel<T><<<red_grid(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, z, c->dmask, c->red, c->gs);
        precond_accumulate_kernel<T, TX><<<grid_for(n), kBlock, 0, s>>>(c->n_nodes, Minv, z, c->dmask, c->gs, x);
    }
    return st->k;
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
        spmv_kernel<double, double, double, double, 0><<<grid_for(n), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const double*)A, (const double*)x, (const double*)nullptr, (double*)y, nullptr);
    else
        spmv_kernel<float, float, float, float, 0><<<grid_for(n), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const float*)A, (const float*)x, (const double*)nullptr, (float*)y, nullptr);
    return check_hip(c, hipGetLastError(), "spmv launch");
}

int launch_bj_setup(vms_ctx* c, const void* A, void* Minv, hipStream_t s) {
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

// FP64 residual r64 = b - A x64 and its norm (synchronising).
static int true_residual(vms_ctx* c, const void* A, const double* b, const double* x, double* rn, hipStream_t s) {
    const int n = 4 * c->n_nodes;
    if (c->prec == VMS_FP64)
        spmv_kernel<double, double, double, double, 1><<<grid_for(n), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const double*)A, x, b, c->r64, nullptr);
    else
        spmv_kernel<float, double, double, double, 1><<<grid_for(n), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const float*)A, x, b, c->r64, nullptr);
    norm_kernel<double><<<red_grid(n), kBlock, 0, s>>>(n, c->r64, c->red, c->rnorm + 2);
    return read_scalar(c, c->rnorm + 2, rn, s);
}

int gmres_solve(vms_ctx* c, const void* A, const double* b, double* x, const vms_solve_opts* o,
                vms_solve_info* info, hipStream_t s) {
    const int n = 4 * c->n_nodes;
    vms_solve_info inf{};
    const int m = o->restart > 0 ? std::min(o->restart, c->max_restart) : c->max_restart;
    const int max_iters = o->max_iters > 0 ? o->max_iters : 100000;
    const double rtol = o->rtol > 0 ? o->rtol : 1e-8;
    const int refine_max = o->refine_max > 0 ? o->refine_max : 30;
    const double inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : 1e-5;
    int rc;

    // preconditioner blocks
    if (o->pc == VMS_PC_LEARNED && o->pc_weights) {
        rc = learned_blocks(c, A, o->pc_weights, c->Minv, c->prec == VMS_FP64, s);
        if (rc == VMS_ENONFINITE) {
            inf.fell_back_to_bj = 1;
            if ((rc = launch_bj_setup(c, A, c->Minv, s))) return rc;
        } else if (rc) {
            return rc;
        }
    } else {
        if ((rc = launch_bj_setup(c, A, c->Minv, s))) return rc;
    }
    if (c->prec == VMS_FP64)
        coarse_setup_kernel<double><<<red_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const double*)A, c->dmask, o->coarse_pressure, c->red, c->gs);
    else
        coarse_setup_kernel<float><<<red_grid(c->n_nodes), kBlock, 0, s>>>(
            c->n_nodes, c->rowptr, c->colidx, (const float*)A, c->dmask, o->coarse_pressure, c->red, c->gs);
    norm_kernel<double><<<red_grid(n), kBlock, 0, s>>>(n, b, c->red, c->rnorm + 3);
    double bn = 0.0;
    if ((rc = read_scalar(c, c->rnorm + 3, &bn, s))) return rc;
    if (!std::isfinite(bn)) return set_error(c, VMS_ENONFINITE, "gmres: non-finite right-hand side");
    if (bn == 0.0) {
        if ((rc = launch_fill(x, n * sizeof(double), s))) return rc;
        inf.true_rel_res = 0.0;
        if (info) *info = inf;
        return check_hip(c, hipStreamSynchronize(s), "sync");
    }
    const double tol = rtol * bn;
    double rn = 0.0;
    int iters = 0;
    int status = VMS_OK;
    const bool learned = o->pc == VMS_PC_LEARNED && o->pc_weights && !inf.fell_back_to_bj;
    const int learned_budget = learned ? max_iters / 2 : max_iters;
    bool using_learned = learned;
    for (;;) {
        if (using_learned && iters >= learned_budget) {
            // the learned blocks did not deliver within half the budget: continue from the
            // current iterate with plain block-Jacobi
            if ((rc = launch_bj_setup(c, A, c->Minv, s))) return rc;
            using_learned = false;
            inf.fell_back_to_bj = 1;
        }
        if ((rc = true_residual(c, A, b, x, &rn, s))) return rc;
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
        if (iters >= max_iters) {
            status = set_error(c, VMS_ENOCONV_GMRES, "gmres: iteration cap reached before rtol");
            break;
        }
        CycleStatus st{0, 0};
        if (c->prec == VMS_FP64) {
            // one restart cycle on the FP64 residual; the true residual is recomputed above
            const int k = run_cycle<double, double>(c, (const double*)A, c->r64, (const double*)c->Minv, x, tol,
                                                    m, max_iters - iters, o->cgs2, &st, s);
            if (k < 0) return VMS_EHIP;
            iters += k;
            inf.restarts++;
            if (k == 0) {
                status = set_error(c, VMS_ENOCONV_GMRES, "gmres: stagnation (no Arnoldi progress)");
                break;
            }
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
            float* Ad = c->tvec + n;
            convert_kernel<double, float><<<grid_for(n), kBlock, 0, s>>>(n, c->r64, rr, 1.0 / rn);
            if ((rc = launch_fill(d, n * sizeof(float), s))) return rc;
            const double inner_tol = std::max(inner_rtol, 0.3 * tol / rn);
            const float* cycle_r = rr;
            int progress = 0;
            while (iters < max_iters) {
                const int k = run_cycle<float, float>(c, (const float*)A, cycle_r, (const float*)c->Minv, d, inner_tol,
                                                      m, max_iters - iters, o->cgs2, &st, s);
                if (k < 0) return VMS_EHIP;
                iters += k;
                progress += k;
                inf.restarts++;
                if (k == 0) break;
                spmv_kernel<float, float, float, float, 1, float><<<grid_for(n), kBlock, 0, s>>>(
                    c->n_nodes, c->rowptr, c->colidx, (const float*)A, d, rr, q, nullptr);
                (void)Ad;
                if (o->log_residuals && inf.logged < o->log_max) {
                    convert_kernel<float, float><<<grid_for(n), kBlock, 0, s>>>(
                        n, q, o->log_residuals + (size_t)inf.logged * n, 1.0);
                    inf.logged++;
                }
                norm_kernel<float><<<red_grid(n), kBlock, 0, s>>>(n, q, c->red, c->rnorm + 2);
                double qn = 0.0;
                if ((rc = read_scalar(c, c->rnorm + 2, &qn, s))) return rc;
                if (!(qn > inner_tol) || !std::isfinite(qn)) break;
                cycle_r = q;
            }
            axpy64_kernel<float><<<grid_for(n), kBlock, 0, s>>>(n, rn, d, x);
            if (progress == 0) {
                status = set_error(c, VMS_ENOCONV_GMRES, "gmres: stagnation (no Arnoldi progress)");
                break;
            }
        }
    }
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
