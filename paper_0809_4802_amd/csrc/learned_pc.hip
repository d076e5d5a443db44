// Learned correction of the 4x4 block-Jacobi preconditioner (FP32 kernels).
//
// The paper leaves the Krylov preconditioner open (Section 6).  Per node i a
// two-layer perceptron maps 25 features of the condensed tangent's block row
// to a 4x4 correction Delta_i, and the preconditioner block becomes
// P_i = D_i^-1 (I + Delta_i) with Delta_i zeroed on Dirichlet rows/columns.
// With a zero output layer this is exactly block-Jacobi.  Training minimises
// mean_s ||r_s - A P r_s||^2 / ||r_s||^2 over residual samples produced by the
// method's own GMRES solves:
//   e = r - A P r,  ds = dL/d(P r) = -2 A^T e / ||r||^2,
//   dL/dDelta_i = D_i^-T ds_i r_i^T (masked),  then the MLP backward and Adam.
// A^T e uses the transposed-block map of the symmetric block pattern.  Weight
// gradients are reduced per workgroup and then across workgroups in a fixed
// order (deterministic).
#include "vms_internal.h"

namespace vms {
namespace {

constexpr int NIN = VMS_PC_NIN, NHID = VMS_PC_NHID, NOUT = VMS_PC_NOUT, NW = VMS_PC_NWEIGHTS;
constexpr int OFF_W1 = 0, OFF_B1 = NHID * NIN, OFF_W2 = OFF_B1 + NHID, OFF_B2 = OFF_W2 + NOUT * NHID;

inline int grid_for(int64_t n, int block = kBlock) { return (int)((n + block - 1) / block); }

// Gauss-Jordan inverse of a 4x4 block in FP64 with partial pivoting; false if singular.
__device__ bool invert4(const double in[16], double out[16]) {
    double m[4][8];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            m[r][c] = in[r * 4 + c];
            m[r][4 + c] = r == c ? 1.0 : 0.0;
        }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        double best = fabs(m[col][col]);
        for (int r = col + 1; r < 4; ++r)
            if (fabs(m[r][col]) > best) {
                best = fabs(m[r][col]);
                piv = r;
            }
        if (!(best > 0.0)) return false;
        if (piv != col)
            for (int c = 0; c < 8; ++c) {
                const double t = m[col][c];
                m[col][c] = m[piv][c];
                m[piv][c] = t;
            }
        const double ip = 1.0 / m[col][col];
        for (int c = 0; c < 8; ++c) m[col][c] *= ip;
        for (int r = 0; r < 4; ++r) {
            if (r == col) continue;
            const double f = m[r][col];
            for (int c = 0; c < 8; ++c) m[r][c] -= f * m[col][c];
        }
    }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) out[r * 4 + c] = m[r][4 + c];
    return true;
}

// Features of node i (see vms.h) and D_i^-1 (float, row-major).
template <typename TA>
__global__ void features_kernel(int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ diagpos,
                                const TA* __restrict__ A, const uint8_t* __restrict__ dmask,
                                float* __restrict__ feats, float* __restrict__ dinv, int32_t* flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int dp = diagpos[i];
    double D[16];
    double fro = 0.0;
    for (int q = 0; q < 16; ++q) {
        D[q] = double(A[(size_t)dp * 16 + q]);
        fro += D[q] * D[q];
    }
    fro = sqrt(fro);
    double off[4] = {0, 0, 0, 0};
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        if (k == dp) continue;
        const TA* b = A + (size_t)k * 16;
        for (int r = 0; r < 4; ++r)
            off[r] += fabs(double(b[r * 4])) + fabs(double(b[r * 4 + 1])) + fabs(double(b[r * 4 + 2])) +
                      fabs(double(b[r * 4 + 3]));
    }
    float* x = feats + (size_t)i * NIN;
    const double ifro = fro > 0.0 ? 1.0 / fro : 0.0;
    for (int q = 0; q < 16; ++q) x[q] = float(D[q] * ifro);
    x[16] = float(log(fmax(fro, 1e-300)));
    const uint32_t dm = dmask[i];
    for (int r = 0; r < 4; ++r) {
        x[17 + r] = float(log1p(off[r] / fmax(fabs(D[r * 5]), 1e-300)));
        x[21 + r] = (dm & (1u << r)) ? 1.f : 0.f;
    }
    double Di[16];
    if (!invert4(D, Di)) {
        atomicAdd(&flags[2], 1);
        for (int q = 0; q < 16; ++q) Di[q] = (q % 5 == 0) ? 1.0 : 0.0;
    }
    if (dinv)
        for (int q = 0; q < 16; ++q) dinv[(size_t)i * 16 + q] = float(Di[q]);
}

// MLP forward per node and P_i = D_i^-1 (I + Delta_i); hidden activations kept for backward.
template <typename TM>
__global__ __launch_bounds__(kBlock) void forward_kernel(int n, const float* __restrict__ feats,
                                                         const float* __restrict__ wts,
                                                         const float* __restrict__ dinv,
                                                         const uint8_t* __restrict__ dmask,
                                                         float* __restrict__ hid, TM* __restrict__ P,
                                                         int32_t* flags) {
    __shared__ float w[NW];
    for (int q = threadIdx.x; q < NW; q += blockDim.x) w[q] = wts[q];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[NIN];
    for (int q = 0; q < NIN; ++q) x[q] = feats[(size_t)i * NIN + q];
    float y[NOUT];
    for (int o = 0; o < NOUT; ++o) y[o] = w[OFF_B2 + o];
    for (int h = 0; h < NHID; ++h) {
        float z = w[OFF_B1 + h];
        for (int q = 0; q < NIN; ++q) z += w[OFF_W1 + h * NIN + q] * x[q];
        const float a = tanhf(z);
        if (hid) hid[(size_t)i * NHID + h] = a;
        for (int o = 0; o < NOUT; ++o) y[o] += w[OFF_W2 + o * NHID + h] * a;
    }
    const uint32_t dm = dmask[i];
    float M[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            const bool masked = (dm & (1u << r)) || (dm & (1u << c));
            M[r * 4 + c] = (r == c ? 1.f : 0.f) + (masked ? 0.f : y[r * 4 + c]);
        }
    bool finite = true;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            float s = 0.f;
            for (int k = 0; k < 4; ++k) s += dinv[(size_t)i * 16 + r * 4 + k] * M[k * 4 + c];
            finite = finite && isfinite(s);
            P[(size_t)i * 16 + r * 4 + c] = TM(s);
        }
    if (!finite) atomicAdd(&flags[3], 1);
}

// t = P r (node-local 4x4 products)
__global__ void block_apply_kernel(int n, const float* __restrict__ P, const float* __restrict__ r,
                                   float* __restrict__ t) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = tid >> 2, q = tid & 3;
    if (i >= n) return;
    const float* p = P + (size_t)i * 16 + q * 4;
    const float* v = r + (size_t)i * 4;
    t[tid] = p[0] * v[0] + p[1] * v[1] + p[2] * v[2] + p[3] * v[3];
}

// y = b - A x (MODE 0) or y = A^T x (MODE 1, via the transposed-block map), FP32 vectors.
template <typename TA, int MODE>
__global__ void spmv_f32_kernel(int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                const int32_t* __restrict__ tpos, const TA* __restrict__ A,
                                const float* __restrict__ x, const float* __restrict__ b, float* __restrict__ y) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = tid >> 2, r = tid & 3;
    if (row >= n) return;
    float acc = 0.f;
    for (int k = rowptr[row]; k < rowptr[row + 1]; ++k) {
        const float* xv = x + (size_t)colidx[k] * 4;
        if (MODE == 0) {
            const TA* a = A + (size_t)k * 16 + r * 4;
            acc += float(a[0]) * xv[0] + float(a[1]) * xv[1] + float(a[2]) * xv[2] + float(a[3]) * xv[3];
        } else {
            const TA* a = A + (size_t)tpos[k] * 16 + r;   // column r of the block (col, row)
            acc += float(a[0]) * xv[0] + float(a[4]) * xv[1] + float(a[8]) * xv[2] + float(a[12]) * xv[3];
        }
    }
    y[tid] = MODE == 0 ? b[tid] - acc : acc;
}

// sums of squares of two vectors, per workgroup: part[b] and part[gridDim.x + b] (no atomics,
// so that training is reproducible run to run; sumsq2_finalize_kernel adds them in order)
__global__ __launch_bounds__(kBlock) void sumsq2_kernel(int n, const float* __restrict__ a,
                                                        const float* __restrict__ b, double* __restrict__ part) {
    double sa = 0.0, sb = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        sa += double(a[i]) * double(a[i]);
        sb += double(b[i]) * double(b[i]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        sa += __shfl_down(sa, off, 64);
        sb += __shfl_down(sb, off, 64);
    }
    __shared__ double ls[2][kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        ls[0][threadIdx.x >> 6] = sa;
        ls[1][threadIdx.x >> 6] = sb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            ta += ls[0][w];
            tb += ls[1][w];
        }
        part[blockIdx.x] = ta;
        part[gridDim.x + blockIdx.x] = tb;
    }
}

// out[0], out[1] = the sums of the nb partials of sumsq2_kernel, in a fixed order (one
// workgroup of kBlock threads: strided serial sums, then a pairwise tree in LDS)
__global__ __launch_bounds__(kBlock) void sumsq2_finalize_kernel(int nb, const double* __restrict__ part,
                                                                 double* __restrict__ out) {
    __shared__ double ls[2][kBlock];
    double sa = 0.0, sb = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) {
        sa += part[i];
        sb += part[nb + i];
    }
    ls[0][threadIdx.x] = sa;
    ls[1][threadIdx.x] = sb;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            ls[0][threadIdx.x] += ls[0][threadIdx.x + h];
            ls[1][threadIdx.x] += ls[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = ls[0][0];
        out[1] = ls[1][0];
    }
}

// gdelta_i += scale * D_i^-T g_i r_i^T, scale = -2 / (S ||r||^2); loss += ||e||^2 / (S ||r||^2)
__global__ void grad_delta_kernel(int n, const float* __restrict__ dinv, const float* __restrict__ g,
                                  const float* __restrict__ r, const double* __restrict__ sums, int nbatch,
                                  float* __restrict__ gdelta, float* __restrict__ loss) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const double rr = sums[1];
    const float scale = rr > 0.0 ? float(-2.0 / (nbatch * rr)) : 0.f;
    if (tid == 0 && rr > 0.0) loss[0] += float(sums[0] / (nbatch * rr));
    const int i = tid >> 4, q = tid & 15;
    if (i >= n) return;
    const int row = q >> 2, col = q & 3;
    const float* di = dinv + (size_t)i * 16;
    const float* gi = g + (size_t)i * 4;
    // (D^-T g)_row = sum_k D^-1[k][row] g_k
    const float dg = di[row] * gi[0] + di[4 + row] * gi[1] + di[8 + row] * gi[2] + di[12 + row] * gi[3];
    gdelta[(size_t)i * 16 + q] += scale * dg * r[(size_t)i * 4 + col];
}

// MLP backward over a chunk of nodes per workgroup; partial weight gradients per workgroup.
constexpr int kBwdNodes = 64;
__global__ __launch_bounds__(kBlock) void backward_kernel(int n, const float* __restrict__ feats,
                                                          const float* __restrict__ hid,
                                                          const float* __restrict__ gdelta,
                                                          const uint8_t* __restrict__ dmask,
                                                          const float* __restrict__ wts, float* __restrict__ wpart) {
    __shared__ float sx[kBwdNodes][NIN + 1];
    __shared__ float sh[kBwdNodes][NHID + 1];
    __shared__ float sgy[kBwdNodes][NOUT + 1];
    __shared__ float sgz[kBwdNodes][NHID + 1];
    float acc[(NW + kBlock - 1) / kBlock];
    for (int q = 0; q < (NW + kBlock - 1) / kBlock; ++q) acc[q] = 0.f;
    const int per_block = (n + gridDim.x - 1) / gridDim.x;
    const int i0 = blockIdx.x * per_block, i1 = min(n, i0 + per_block);
    for (int c0 = i0; c0 < i1; c0 += kBwdNodes) {
        const int cn = min(kBwdNodes, i1 - c0);
        // stage features, activations and the masked output gradient
        for (int q = threadIdx.x; q < kBwdNodes * NIN; q += blockDim.x) {
            const int a = q / NIN, f = q % NIN;
            sx[a][f] = a < cn ? feats[(size_t)(c0 + a) * NIN + f] : 0.f;
        }
        for (int q = threadIdx.x; q < kBwdNodes * NHID; q += blockDim.x) {
            const int a = q / NHID, h = q % NHID;
            sh[a][h] = a < cn ? hid[(size_t)(c0 + a) * NHID + h] : 0.f;
        }
        for (int q = threadIdx.x; q < kBwdNodes * NOUT; q += blockDim.x) {
            const int a = q / NOUT, o = q % NOUT;
            float v = 0.f;
            if (a < cn) {
                const uint32_t dm = dmask[c0 + a];
                const int rr = o >> 2, cc = o & 3;
                v = ((dm & (1u << rr)) || (dm & (1u << cc))) ? 0.f : gdelta[(size_t)(c0 + a) * 16 + o];
            }
            sgy[a][o] = v;
        }
        __syncthreads();
        // hidden gradient: gz = (W2^T gy) * (1 - h^2)
        for (int q = threadIdx.x; q < kBwdNodes * NHID; q += blockDim.x) {
            const int a = q / NHID, h = q % NHID;
            float s = 0.f;
            for (int o = 0; o < NOUT; ++o) s += wts[OFF_W2 + o * NHID + h] * sgy[a][o];
            sgz[a][h] = s * (1.f - sh[a][h] * sh[a][h]);
        }
        __syncthreads();
        // weight gradients: each thread owns a fixed set of weights
        for (int q = 0; q < (NW + kBlock - 1) / kBlock; ++q) {
            const int wi = q * kBlock + threadIdx.x;
            if (wi >= NW) break;
            float s = 0.f;
            if (wi < OFF_B1) {
                const int h = wi / NIN, f = wi % NIN;
                for (int a = 0; a < cn; ++a) s += sgz[a][h] * sx[a][f];
            } else if (wi < OFF_W2) {
                const int h = wi - OFF_B1;
                for (int a = 0; a < cn; ++a) s += sgz[a][h];
            } else if (wi < OFF_B2) {
                const int o = (wi - OFF_W2) / NHID, h = (wi - OFF_W2) % NHID;
                for (int a = 0; a < cn; ++a) s += sgy[a][o] * sh[a][h];
            } else {
                const int o = wi - OFF_B2;
                for (int a = 0; a < cn; ++a) s += sgy[a][o];
            }
            acc[q] += s;
        }
        __syncthreads();
    }
    for (int q = 0; q < (NW + kBlock - 1) / kBlock; ++q) {
        const int wi = q * kBlock + threadIdx.x;
        if (wi < NW) wpart[(size_t)blockIdx.x * NW + wi] = acc[q];
    }
}

// grad = sum of the partials (fixed order); Adam update when lr > 0.
__global__ void adam_kernel(int nparts, const float* __restrict__ wpart, float* __restrict__ wts,
                            float* __restrict__ mstate, float* __restrict__ vstate, int step, float lr,
                            float* __restrict__ grad_out) {
    const int wi = blockIdx.x * blockDim.x + threadIdx.x;
    if (wi >= NW) return;
    float g = 0.f;
    for (int p = 0; p < nparts; ++p) g += wpart[(size_t)p * NW + wi];
    if (grad_out) grad_out[wi] = g;
    if (!(lr > 0.f)) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float m = b1 * mstate[wi] + (1.f - b1) * g;
    const float v = b2 * vstate[wi] + (1.f - b2) * g * g;
    mstate[wi] = m;
    vstate[wi] = v;
    const float mh = m / (1.f - powf(b1, (float)step));
    const float vh = v / (1.f - powf(b2, (float)step));
    wts[wi] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void zero_f32_kernel(float* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}


__global__ void reset_pc_flags_kernel(int32_t* flags) {
    if (threadIdx.x == 0) {
        flags[2] = 0;
        flags[3] = 0;
    }
}

constexpr int kBwdBlocks = 256;

int features(vms_ctx* c, const void* A, float* feats, float* dinv, hipStream_t s) {
    if (c->prec == VMS_FP64)
        features_kernel<double><<<grid_for(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->rowptr, c->diagpos,
                                                                       (const double*)A, c->dmask, feats, dinv,
                                                                       c->flags);
    else
        features_kernel<float><<<grid_for(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->rowptr, c->diagpos,
                                                                      (const float*)A, c->dmask, feats, dinv,
                                                                      c->flags);
    return check_hip(c, hipGetLastError(), "features launch");
}

}  // namespace

int learned_blocks(vms_ctx* c, const void* A, const float* weights, void* Minv_out, int out_is_double,
                   hipStream_t s) {
    PhaseScope ph(c, VMS_PH_PCSETUP, (double)c->n_nodes * (32.0 * elt_size(c) + 4.0), s);
    reset_pc_flags_kernel<<<1, 64, 0, s>>>(c->flags);
    int rc = features(c, A, c->feats, c->gblk, s);   // gblk holds D^-1 here
    if (rc) return rc;
    if (out_is_double)
        forward_kernel<double><<<grid_for(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->feats, weights, c->gblk,
                                                                      c->dmask, nullptr, (double*)Minv_out, c->flags);
    else
        forward_kernel<float><<<grid_for(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->feats, weights, c->gblk,
                                                                     c->dmask, nullptr, (float*)Minv_out, c->flags);
    if ((rc = check_hip(c, hipGetLastError(), "learned blocks launch"))) return rc;
    int32_t h[4];
    if ((rc = check_hip(c, hipMemcpyAsync(h, c->flags, sizeof h, hipMemcpyDeviceToHost, s), "read flags"))) return rc;
    if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
    if (h[2] || h[3]) return set_error(c, VMS_ENONFINITE, "learned preconditioner produced a non-finite block");
    return VMS_OK;
}

}  // namespace vms

using namespace vms;

extern "C" int vms_pc_features(vms_ctx* c, const void* bsr_vals, float* feats, hipStream_t s) {
    if (!c || !bsr_vals || !feats) return set_error(c, VMS_EINVAL, "vms_pc_features: NULL argument");
    return features(c, bsr_vals, feats, nullptr, s);
}

extern "C" int vms_pc_blocks(vms_ctx* c, const void* bsr_vals, const float* weights, float* P, hipStream_t s) {
    if (!c || !bsr_vals || !P) return set_error(c, VMS_EINVAL, "vms_pc_blocks: NULL argument");
    int rc = features(c, bsr_vals, c->feats, c->gblk, s);
    if (rc) return rc;
    if (!weights) {   // plain block-Jacobi: P = D^-1
        return check_hip(c, hipMemcpyAsync(P, c->gblk, (size_t)c->n_nodes * 16 * sizeof(float),
                                           hipMemcpyDeviceToDevice, s), "copy blocks");
    }
    forward_kernel<float><<<grid_for(c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->feats, weights, c->gblk, c->dmask,
                                                                 nullptr, P, c->flags);
    return check_hip(c, hipGetLastError(), "pc blocks launch");
}

extern "C" int vms_pc_train_step(vms_ctx* c, const void* bsr_vals, const float* r_batch, int32_t nbatch,
                                 float* weights, float* adam_state, int32_t step, float lr, float* grad_out,
                                 float* loss_out, hipStream_t s) {
    if (!c || !bsr_vals || !r_batch || !weights || nbatch <= 0)
        return set_error(c, VMS_EINVAL, "vms_pc_train_step: NULL argument or empty batch");
    if (lr > 0.f && (!adam_state || step < 1))
        return set_error(c, VMS_EINVAL, "vms_pc_train_step: Adam needs adam_state and step >= 1");
    const int n = c->n_nodes;
    const int N = 4 * n;
    float* dinv = c->gblk;             // D^-1 blocks
    float* P = c->pblk;                // preconditioner blocks
    float* t = c->tvec;                // P r
    float* e = c->tvec + N;            // r - A P r
    float* g = c->tvec + 2 * (size_t)N;  // A^T e
    float* gdelta = c->gdel;           // [n][16]
    double* sums = c->rnorm + 4;       // the two FP64 sums of the loss
    float* loss = c->fscal;
    int rc = features(c, bsr_vals, c->feats, dinv, s);
    if (rc) return rc;
    forward_kernel<float><<<grid_for(n), kBlock, 0, s>>>(n, c->feats, weights, dinv, c->dmask, c->hid, P, c->flags);
    zero_f32_kernel<<<std::min(grid_for((int64_t)16 * n), 4096), kBlock, 0, s>>>(gdelta, (size_t)16 * n);
    zero_f32_kernel<<<1, 64, 0, s>>>(loss, 1);
    for (int b = 0; b < nbatch; ++b) {
        const float* r = r_batch + (size_t)b * N;
        block_apply_kernel<<<grid_for(N), kBlock, 0, s>>>(n, P, r, t);
        if (c->prec == VMS_FP64) {
            spmv_f32_kernel<double, 0><<<grid_for(N), kBlock, 0, s>>>(n, c->rowptr, c->colidx, c->tpos,
                                                                     (const double*)bsr_vals, t, r, e);
            spmv_f32_kernel<double, 1><<<grid_for(N), kBlock, 0, s>>>(n, c->rowptr, c->colidx, c->tpos,
                                                                     (const double*)bsr_vals, e, nullptr, g);
        } else {
            spmv_f32_kernel<float, 0><<<grid_for(N), kBlock, 0, s>>>(n, c->rowptr, c->colidx, c->tpos,
                                                                    (const float*)bsr_vals, t, r, e);
            spmv_f32_kernel<float, 1><<<grid_for(N), kBlock, 0, s>>>(n, c->rowptr, c->colidx, c->tpos,
                                                                    (const float*)bsr_vals, e, nullptr, g);
        }
        const int nb = std::min(grid_for(N), 1024);
        sumsq2_kernel<<<nb, kBlock, 0, s>>>(N, e, r, c->red->partial);      // reduction scratch: idle here
        sumsq2_finalize_kernel<<<1, kBlock, 0, s>>>(nb, c->red->partial, sums);
        grad_delta_kernel<<<grid_for((int64_t)16 * n), kBlock, 0, s>>>(n, dinv, g, r, sums, nbatch, gdelta, loss);
    }
    const int nparts = std::min(kBwdBlocks, std::max(1, (n + kBwdNodes - 1) / kBwdNodes));
    backward_kernel<<<nparts, kBlock, 0, s>>>(n, c->feats, c->hid, gdelta, c->dmask, weights, c->wgrad);
    adam_kernel<<<grid_for(NW), kBlock, 0, s>>>(nparts, c->wgrad, weights, adam_state,
                                                adam_state ? adam_state + NW : nullptr, step, lr, grad_out);
    if (loss_out)
        if ((rc = check_hip(c, hipMemcpyAsync(loss_out, loss, sizeof(float), hipMemcpyDeviceToDevice, s), "loss")))
            return rc;
    return check_hip(c, hipGetLastError(), "train step launch");
}
