// Element kernels of the VMS Newton-Schur method on gfx950.
//
// One lane per element.  Every integral of the element residual (Section 4.1,
// coarse momentum R_c, continuity R_p, fine momentum R_f, plus the backward
// Euler terms of the Section 4.1 Remark) and of its consistent tangent
// (Section 4.2) is a polynomial in the barycentric coordinates of an affine
// tet, so the kernels integrate exactly with closed-form moments instead of
// quadrature.  With |T| the volume, g_a the barycentric gradients and the
// bubble b = 256 l0 l1 l2 l3 (Section 3.3 leaves its form open):
//   int l_a l_b = |T| (1 + delta_ab) / 20        int b l_a = 8 |T| / 105
//   int b = 32 |T| / 105                          int b^2 = 8192 |T| / 51975
//   int |grad b|^2 = 4096 |T| / 945 sum_a |g_a|^2
//   int grad b = 0,  int l_a grad b = -(int b) g_a,  int l_a b grad b = -(int b^2) g_a / 2,
//   int b grad b . vbar = -(int b^2) div(vbar) / 2,  int b^2 grad b = 0.
// Residual (G = grad vbar, th = div vbar, W = int b vbar, V_a = sum_b M_ab v_b):
//   R_c,a = G V_a + B1 G beta - (g_a.W + th B1) beta - C/2 (beta.g_a) beta
//           + 2 nu |T| G g_a - |T|/4 (sum p) g_a - sum_b M_ab f_b + (1/dt) sum_b M_ab (v_b - v_b^n)
//   R_p,a = -th |T| / 4 + B (beta . g_a)
//   R_f   = G W + C (G - th/2 I) beta + 2 nu Kb beta + B grad p - B1 sum f + (B1/dt) sum (v - v^n)
// Tangent blocks (3x3 unless noted):
//   K_vv(a,b) = [g_b.V_a + M_ab/dt + 2 nu |T| g_a.g_b + B1 g_b.beta] I + M_ab G - B1 beta (g_a + g_b)^T
//   K_vp(a,b) = -|T|/4 g_a,   K_pv(a,b) = -|T|/4 g_b^T,   K_pp = 0
//   K_vf(a) = B1 G - (g_a.W + th B1) I - C/2 [(beta.g_a) I + beta g_a^T],   K_pf(a) = B g_a^T
//   K_fv(b) = (g_b.W) I + B1 G + C [(g_b.beta) I - beta g_b^T / 2] + B1/dt I,  K_fp(b) = B g_b
//   K_ff = C (G - th/2 I) + 2 nu Kb I
// (B1, B, C, Kb already multiplied by |T|.)  Condensation (Section 5):
//   K* = K_cc - K_cf K_ff^-1 K_fc,  R* = R_cp - K_cf K_ff^-1 R_f,
// recovery: dbeta = K_ff^-1 (-R_f - K_fc du_e).
#include <climits>

#include "vms_internal.h"

namespace vms {
namespace {

constexpr double kB1 = 8.0 / 105.0;
constexpr double kB = 32.0 / 105.0;
constexpr double kC = 8192.0 / 51975.0;
constexpr double kKb = 4096.0 / 945.0;

struct ElemArgs {
    const double4* __restrict__ xyz4;
    const int4* __restrict__ tets;
    const uint8_t* __restrict__ dmask;
    const double* __restrict__ u;        // [n][4]
    const double* __restrict__ u_prev;   // [n][4] or null
    const double* beta;                  // [e][3] (may alias the recovery output)
    const double* __restrict__ body;     // [n][3] or null
    double nu;
    double inv_dt;
    int n_elems;
    int32_t* flags;                      // [0] first degenerate element, [1] first singular K_ff
};

// FP64 state of one element: geometry, nodal data and the derived fields.
struct Elem {
    int4 t;
    double g[4][3];
    double vol;
    double v[4][3];
    double p[4];
    double be[3];
    double G[3][3];
    double th;
    double gp[3];
    double vs[3];      // sum_a v_a
    double Wv[3];      // int b vbar = B1 sum v
    double B1, B, C, Kb;
    double dvs[3];     // sum_a (v_a - v_a^n)
    double dv[4][3];
    double fs[3];      // sum_a f_a
    double f[4][3];
    bool transient;
    bool has_body;
};

__device__ __forceinline__ bool load_element(const ElemArgs& A, int e, Elem& E) {
    E.t = A.tets[e];
    const int nid[4] = {E.t.x, E.t.y, E.t.z, E.t.w};
    double X[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double4 x = A.xyz4[nid[a]];
        X[a][0] = x.x;
        X[a][1] = x.y;
        X[a][2] = x.z;
        const double4 uu = reinterpret_cast<const double4*>(A.u)[nid[a]];
        E.v[a][0] = uu.x;
        E.v[a][1] = uu.y;
        E.v[a][2] = uu.z;
        E.p[a] = uu.w;
    }
    // J[i][k] = d x_i / d xi_k,  inverse rows = gradients of xi_k
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) J[i][k] = X[k + 1][i] - X[0][i];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det > 0.0)) return false;
    const double id = 1.0 / det;
    // inv[k][i] = d xi_k / d x_i
    const double inv00 = c00 * id, inv01 = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id,
                 inv02 = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    const double inv10 = c01 * id, inv11 = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id,
                 inv12 = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    const double inv20 = c02 * id, inv21 = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id,
                 inv22 = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    E.g[1][0] = inv00; E.g[1][1] = inv01; E.g[1][2] = inv02;
    E.g[2][0] = inv10; E.g[2][1] = inv11; E.g[2][2] = inv12;
    E.g[3][0] = inv20; E.g[3][1] = inv21; E.g[3][2] = inv22;
#pragma unroll
    for (int i = 0; i < 3; ++i) E.g[0][i] = -(E.g[1][i] + E.g[2][i] + E.g[3][i]);
    E.vol = det * (1.0 / 6.0);
    const double* bp = A.beta + 3 * (size_t)e;
    E.be[0] = bp[0];
    E.be[1] = bp[1];
    E.be[2] = bp[2];

    double gg = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) gg += E.g[a][0] * E.g[a][0] + E.g[a][1] * E.g[a][1] + E.g[a][2] * E.g[a][2];
    E.B1 = kB1 * E.vol;
    E.B = kB * E.vol;
    E.C = kC * E.vol;
    E.Kb = kKb * E.vol * gg;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            E.G[i][j] = E.v[0][i] * E.g[0][j] + E.v[1][i] * E.g[1][j] + E.v[2][i] * E.g[2][j] +
                        E.v[3][i] * E.g[3][j];
        E.gp[i] = E.p[0] * E.g[0][i] + E.p[1] * E.g[1][i] + E.p[2] * E.g[2][i] + E.p[3] * E.g[3][i];
        E.vs[i] = E.v[0][i] + E.v[1][i] + E.v[2][i] + E.v[3][i];
        E.Wv[i] = E.B1 * E.vs[i];
    }
    E.th = E.G[0][0] + E.G[1][1] + E.G[2][2];

    E.transient = A.u_prev != nullptr && A.inv_dt != 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) E.dvs[i] = 0.0;
    if (E.transient) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double4 up = reinterpret_cast<const double4*>(A.u_prev)[nid[a]];
            E.dv[a][0] = E.v[a][0] - up.x;
            E.dv[a][1] = E.v[a][1] - up.y;
            E.dv[a][2] = E.v[a][2] - up.z;
#pragma unroll
            for (int i = 0; i < 3; ++i) E.dvs[i] += E.dv[a][i];
        }
    } else {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) E.dv[a][i] = 0.0;
    }
    E.has_body = A.body != nullptr;
#pragma unroll
    for (int i = 0; i < 3; ++i) E.fs[i] = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int i = 0; i < 3; ++i) E.f[a][i] = E.has_body ? A.body[3 * (size_t)nid[a] + i] : 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) E.fs[i] += E.f[a][i];
    }
    return true;
}

// Fine-scale residual R_f (FP64).
__device__ __forceinline__ void fine_residual(const Elem& E, double nu, double inv_dt, double Rf[3]) {
    const double twonuKb = 2.0 * nu * E.Kb;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double s = E.G[i][0] * E.Wv[0] + E.G[i][1] * E.Wv[1] + E.G[i][2] * E.Wv[2];
        s += E.C * (E.G[i][0] * E.be[0] + E.G[i][1] * E.be[1] + E.G[i][2] * E.be[2] - 0.5 * E.th * E.be[i]);
        s += twonuKb * E.be[i] + E.B * E.gp[i] - E.B1 * E.fs[i] + inv_dt * E.B1 * E.dvs[i];
        Rf[i] = s;
    }
}

// Coarse residual rows of node a: R_c,a (3) and R_p,a (FP64).
__device__ __forceinline__ void coarse_residual(const Elem& E, int a, double nu, double inv_dt,
                                                double R[4]) {
    const double m0 = E.vol * (1.0 / 20.0);
    double Va[3], Fa[3], Da[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Va[i] = m0 * (E.vs[i] + E.v[a][i]);
        Fa[i] = m0 * (E.fs[i] + E.f[a][i]);
        Da[i] = m0 * (E.dvs[i] + E.dv[a][i]);
    }
    const double gW = E.g[a][0] * E.Wv[0] + E.g[a][1] * E.Wv[1] + E.g[a][2] * E.Wv[2];
    const double bg = E.be[0] * E.g[a][0] + E.be[1] * E.g[a][1] + E.be[2] * E.g[a][2];
    const double ps = E.p[0] + E.p[1] + E.p[2] + E.p[3];
    const double coef_b = gW + E.th * E.B1 + 0.5 * E.C * bg;
    const double visc = 2.0 * nu * E.vol;
    const double pq = 0.25 * E.vol * ps;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double s = E.G[i][0] * (Va[0] + E.B1 * E.be[0]) + E.G[i][1] * (Va[1] + E.B1 * E.be[1]) +
                   E.G[i][2] * (Va[2] + E.B1 * E.be[2]);
        s -= coef_b * E.be[i];
        s += visc * (E.G[i][0] * E.g[a][0] + E.G[i][1] * E.g[a][1] + E.G[i][2] * E.g[a][2]);
        s -= pq * E.g[a][i];
        s -= Fa[i];
        s += inv_dt * Da[i];
        R[i] = s;
    }
    R[3] = -E.th * E.vol * 0.25 + E.B * bg;
}

// K_ff and its inverse (FP64).  Returns false when K_ff is numerically singular.
__device__ __forceinline__ bool fine_block_inverse(const Elem& E, double nu, double Ki[3][3],
                                                   double Kff[3][3]) {
    const double d = 2.0 * nu * E.Kb - 0.5 * E.C * E.th;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Kff[i][j] = E.C * E.G[i][j] + (i == j ? d : 0.0);
    const double c00 = Kff[1][1] * Kff[2][2] - Kff[1][2] * Kff[2][1];
    const double c01 = Kff[1][2] * Kff[2][0] - Kff[1][0] * Kff[2][2];
    const double c02 = Kff[1][0] * Kff[2][1] - Kff[1][1] * Kff[2][0];
    const double det = Kff[0][0] * c00 + Kff[0][1] * c01 + Kff[0][2] * c02;
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        nrm = fmax(nrm, fabs(Kff[i][0]) + fabs(Kff[i][1]) + fabs(Kff[i][2]));
    const bool ok = fabs(det) > 1e-14 * nrm * nrm * nrm && isfinite(det);
    const double id = 1.0 / det;
    Ki[0][0] = c00 * id;
    Ki[0][1] = (Kff[0][2] * Kff[2][1] - Kff[0][1] * Kff[2][2]) * id;
    Ki[0][2] = (Kff[0][1] * Kff[1][2] - Kff[0][2] * Kff[1][1]) * id;
    Ki[1][0] = c01 * id;
    Ki[1][1] = (Kff[0][0] * Kff[2][2] - Kff[0][2] * Kff[2][0]) * id;
    Ki[1][2] = (Kff[0][2] * Kff[1][0] - Kff[0][0] * Kff[1][2]) * id;
    Ki[2][0] = c02 * id;
    Ki[2][1] = (Kff[0][1] * Kff[2][0] - Kff[0][0] * Kff[2][1]) * id;
    Ki[2][2] = (Kff[0][0] * Kff[1][1] - Kff[0][1] * Kff[1][0]) * id;
    return ok;
}

// K_fc(b): 3x4 block (velocity columns 0..2, pressure column 3), precision T.
template <typename T>
__device__ __forceinline__ void fine_coarse_block(const Elem& E, int b, double inv_dt, T K[3][4]) {
    const double gW = E.g[b][0] * E.Wv[0] + E.g[b][1] * E.Wv[1] + E.g[b][2] * E.Wv[2];
    const double gb = E.g[b][0] * E.be[0] + E.g[b][1] * E.be[1] + E.g[b][2] * E.be[2];
    const T diag = T(gW + E.C * gb + E.B1 * inv_dt);
    const T B1 = T(E.B1), hC = T(0.5 * E.C), B = T(E.B);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            K[i][j] = B1 * T(E.G[i][j]) - hC * T(E.be[i]) * T(E.g[b][j]) + (i == j ? diag : T(0));
        K[i][3] = B * T(E.g[b][i]);
    }
}

// K_cf(a): 4x3 block (velocity rows 0..2, pressure row 3), precision T.
template <typename T>
__device__ __forceinline__ void coarse_fine_block(const Elem& E, int a, T K[4][3]) {
    const double gW = E.g[a][0] * E.Wv[0] + E.g[a][1] * E.Wv[1] + E.g[a][2] * E.Wv[2];
    const double bg = E.be[0] * E.g[a][0] + E.be[1] * E.g[a][1] + E.be[2] * E.g[a][2];
    const T diag = T(-(gW + E.th * E.B1) - 0.5 * E.C * bg);
    const T B1 = T(E.B1), hC = T(0.5 * E.C), B = T(E.B);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            K[i][j] = B1 * T(E.G[i][j]) - hC * T(E.be[i]) * T(E.g[a][j]) + (i == j ? diag : T(0));
#pragma unroll
    for (int j = 0; j < 3; ++j) K[3][j] = B * T(E.g[a][j]);
}

// K_cc(a,b): 4x4 block, precision T.  Gt, gt, Vt, bt are T copies of the fields.
template <typename T>
__device__ __forceinline__ void coarse_block(const T Gt[3][3], const T gt[4][3], const T Va[3],
                                             const T bt[3], T vol, T B1, T two_nu_vol, T inv_dt,
                                             int a, int b, T K[4][4]) {
    const T mab = vol * (a == b ? T(0.1) : T(0.05));
    const T gbV = gt[b][0] * Va[0] + gt[b][1] * Va[1] + gt[b][2] * Va[2];
    const T gagb = gt[a][0] * gt[b][0] + gt[a][1] * gt[b][1] + gt[a][2] * gt[b][2];
    const T gbb = gt[b][0] * bt[0] + gt[b][1] * bt[1] + gt[b][2] * bt[2];
    const T s = gbV + mab * inv_dt + two_nu_vol * gagb + B1 * gbb;
    const T qv = T(-0.25) * vol;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            K[i][j] = mab * Gt[i][j] - B1 * bt[i] * (gt[a][j] + gt[b][j]) + (i == j ? s : T(0));
        K[i][3] = qv * gt[a][i];
        K[3][i] = qv * gt[b][i];
    }
    K[3][3] = T(0);
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
    unsafeAtomicAdd(p, v);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// -------------------------------------------------------------------------------------------
// Condense and assemble: K* into the block-CSR values, -R* into rhs, [R_c; R_p] into rglob
// (free dofs only), sum |R_f|^2 into red_slots.
template <typename T>
__global__ __launch_bounds__(kBlock) void condense_kernel(ElemArgs args, const int32_t* __restrict__ epos,
                                                          T* __restrict__ Aval, double* __restrict__ rhs,
                                                          double* __restrict__ rglob,
                                                          double* __restrict__ red_slots) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double rf2 = 0.0;
    if (e < args.n_elems) {
        Elem E;
        if (!load_element(args, e, E)) {
            atomicMin(&args.flags[0], e);
        } else {
            const double nu = args.nu, inv_dt = E.transient ? args.inv_dt : 0.0;
            double Rf[3];
            fine_residual(E, nu, inv_dt, Rf);
            rf2 = Rf[0] * Rf[0] + Rf[1] * Rf[1] + Rf[2] * Rf[2];
            double Ki[3][3], Kff[3][3];
            if (!fine_block_inverse(E, nu, Ki, Kff)) atomicMin(&args.flags[1], e);
            double z[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) z[i] = Ki[i][0] * Rf[0] + Ki[i][1] * Rf[1] + Ki[i][2] * Rf[2];
            // W(b) = K_ff^-1 K_fc(b): FP64 product, stored in T
            T Wb[4][3][4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double Kfc[3][4];
                fine_coarse_block<double>(E, b, inv_dt, Kfc);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        Wb[b][i][c] = T(Ki[i][0] * Kfc[0][c] + Ki[i][1] * Kfc[1][c] + Ki[i][2] * Kfc[2][c]);
            }
            T Gt[3][3], gt[4][3], bt[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j) Gt[i][j] = T(E.G[i][j]);
                bt[i] = T(E.be[i]);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) gt[a][i] = T(E.g[a][i]);
            const T volt = T(E.vol), B1t = T(E.B1), tnv = T(2.0 * nu * E.vol), idt = T(inv_dt);
            const int nid[4] = {E.t.x, E.t.y, E.t.z, E.t.w};
            uint32_t dm[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) dm[a] = args.dmask[nid[a]];
            const size_t ne = (size_t)args.n_elems;

#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double Rc[4];
                coarse_residual(E, a, nu, inv_dt, Rc);
                double Kcf[4][3];
                coarse_fine_block<double>(E, a, Kcf);
                const size_t row = 4 * (size_t)nid[a];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (dm[a] & (1u << r)) continue;
                    const double rs = Rc[r] - (Kcf[r][0] * z[0] + Kcf[r][1] * z[1] + Kcf[r][2] * z[2]);
                    atomic_add(&rhs[row + r], -rs);
                    atomic_add(&rglob[row + r], Rc[r]);
                }
                T Kc[4][3];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int k = 0; k < 3; ++k) Kc[r][k] = T(Kcf[r][k]);
                const double m0 = E.vol * (1.0 / 20.0);
                T Va[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) Va[i] = T(m0 * (E.vs[i] + E.v[a][i]));
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    T K[4][4];
                    coarse_block<T>(Gt, gt, Va, bt, volt, B1t, tnv, idt, a, b, K);
                    const int blk = epos[(a * 4 + b) * ne + e];
                    T* dst = Aval + (size_t)blk * 16;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (dm[a] & (1u << r)) continue;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (dm[b] & (1u << c)) continue;
                            const T val = K[r][c] - (Kc[r][0] * Wb[b][0][c] + Kc[r][1] * Wb[b][1][c] +
                                                     Kc[r][2] * Wb[b][2][c]);
                            atomic_add(&dst[r * 4 + c], val);
                        }
                    }
                }
            }
        }
    }
    rf2 = wave_sum(rf2);
    if ((threadIdx.x & 63) == 0 && rf2 != 0.0) atomic_add(&red_slots[(blockIdx.x & 63) * 8], rf2);
}

// Residual only: [R_c; R_p] into rglob (free dofs), |R_f|^2 into red_slots.
__global__ __launch_bounds__(kBlock) void residual_kernel(ElemArgs args, double* __restrict__ rglob,
                                                          double* __restrict__ red_slots) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double rf2 = 0.0;
    if (e < args.n_elems) {
        Elem E;
        if (!load_element(args, e, E)) {
            atomicMin(&args.flags[0], e);
        } else {
            const double inv_dt = E.transient ? args.inv_dt : 0.0;
            double Rf[3];
            fine_residual(E, args.nu, inv_dt, Rf);
            rf2 = Rf[0] * Rf[0] + Rf[1] * Rf[1] + Rf[2] * Rf[2];
            const int nid[4] = {E.t.x, E.t.y, E.t.z, E.t.w};
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const uint32_t dm = args.dmask[nid[a]];
                double Rc[4];
                coarse_residual(E, a, args.nu, inv_dt, Rc);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (!(dm & (1u << r))) atomic_add(&rglob[4 * (size_t)nid[a] + r], Rc[r]);
            }
        }
    }
    rf2 = wave_sum(rf2);
    if ((threadIdx.x & 63) == 0 && rf2 != 0.0) atomic_add(&red_slots[(blockIdx.x & 63) * 8], rf2);
}

// Raw element residual and 19x19 tangent (tangent blocks in T, K_ff in FP64).
template <typename T>
__global__ __launch_bounds__(kBlock) void raw_kernel(ElemArgs args, double* __restrict__ Ke,
                                                     double* __restrict__ Rv) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= args.n_elems) return;
    Elem E;
    if (!load_element(args, e, E)) {
        atomicMin(&args.flags[0], e);
        return;
    }
    const double nu = args.nu, inv_dt = E.transient ? args.inv_dt : 0.0;
    if (Rv) {
        double* R = Rv + 19 * (size_t)e;
        for (int a = 0; a < 4; ++a) {
            double Rc[4];
            coarse_residual(E, a, nu, inv_dt, Rc);
            for (int r = 0; r < 4; ++r) R[4 * a + r] = Rc[r];
        }
        double Rf[3];
        fine_residual(E, nu, inv_dt, Rf);
        for (int i = 0; i < 3; ++i) R[16 + i] = Rf[i];
    }
    if (!Ke) return;
    double* K = Ke + 361 * (size_t)e;
    T Gt[3][3], gt[4][3], bt[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Gt[i][j] = T(E.G[i][j]);
        bt[i] = T(E.be[i]);
    }
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) gt[a][i] = T(E.g[a][i]);
    const T volt = T(E.vol), B1t = T(E.B1), tnv = T(2.0 * nu * E.vol), idt = T(inv_dt);
    const double m0 = E.vol * (1.0 / 20.0);
    for (int a = 0; a < 4; ++a) {
        T Va[3];
        for (int i = 0; i < 3; ++i) Va[i] = T(m0 * (E.vs[i] + E.v[a][i]));
        for (int b = 0; b < 4; ++b) {
            T Kb[4][4];
            coarse_block<T>(Gt, gt, Va, bt, volt, B1t, tnv, idt, a, b, Kb);
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) K[(4 * a + r) * 19 + 4 * b + c] = double(Kb[r][c]);
        }
        T Kcf[4][3];
        coarse_fine_block<T>(E, a, Kcf);
        for (int r = 0; r < 4; ++r)
            for (int k = 0; k < 3; ++k) K[(4 * a + r) * 19 + 16 + k] = double(Kcf[r][k]);
        T Kfc[3][4];
        fine_coarse_block<T>(E, a, inv_dt, Kfc);
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 4; ++c) K[(16 + k) * 19 + 4 * a + c] = double(Kfc[k][c]);
    }
    double Ki[3][3], Kff[3][3];
    if (!fine_block_inverse(E, nu, Ki, Kff)) atomicMin(&args.flags[1], e);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K[(16 + i) * 19 + 16 + j] = Kff[i][j];
}

// Fine-scale recovery at the linearisation point, then beta += dbeta (FP64).
__global__ __launch_bounds__(kBlock) void recover_kernel(ElemArgs args, const double* __restrict__ du,
                                                         double* beta_out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= args.n_elems) return;
    Elem E;
    if (!load_element(args, e, E)) {
        atomicMin(&args.flags[0], e);
        return;
    }
    const double nu = args.nu, inv_dt = E.transient ? args.inv_dt : 0.0;
    double Rf[3];
    fine_residual(E, nu, inv_dt, Rf);
    const int nid[4] = {E.t.x, E.t.y, E.t.z, E.t.w};
    double rhs[3] = {-Rf[0], -Rf[1], -Rf[2]};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t dm = args.dmask[nid[b]];
        const double4 d4 = reinterpret_cast<const double4*>(du)[nid[b]];
        const double dd[4] = {(dm & 1u) ? 0.0 : d4.x, (dm & 2u) ? 0.0 : d4.y, (dm & 4u) ? 0.0 : d4.z,
                              (dm & 8u) ? 0.0 : d4.w};
        double Kfc[3][4];
        fine_coarse_block<double>(E, b, inv_dt, Kfc);
#pragma unroll
        for (int i = 0; i < 3; ++i)
            rhs[i] -= Kfc[i][0] * dd[0] + Kfc[i][1] * dd[1] + Kfc[i][2] * dd[2] + Kfc[i][3] * dd[3];
    }
    double Ki[3][3], Kff[3][3];
    if (!fine_block_inverse(E, nu, Ki, Kff)) atomicMin(&args.flags[1], e);
    double* bo = beta_out + 3 * (size_t)e;
#pragma unroll
    for (int i = 0; i < 3; ++i) bo[i] = E.be[i] + (Ki[i][0] * rhs[0] + Ki[i][1] * rhs[1] + Ki[i][2] * rhs[2]);
}

// u += du on free dofs (du zeroed on Dirichlet dofs).
__global__ void update_kernel(int n_nodes, const uint8_t* __restrict__ dmask, const double* __restrict__ du,
                              double* __restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * n_nodes) return;
    if (dmask[i >> 2] & (1u << (i & 3))) return;
    u[i] += du[i];
}

// Unit diagonal on Dirichlet dofs (their rows and columns were skipped by the scatter).
template <typename T>
__global__ void dirichlet_diag_kernel(int n_dir, const int32_t* __restrict__ dlist,
                                      const int32_t* __restrict__ diagpos, T* __restrict__ Aval) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_dir) return;
    const int d = dlist[k];
    const int c = d & 3;
    Aval[(size_t)diagpos[d >> 2] * 16 + c * 4 + c] = T(1);
}

// Newton residual norm: free-dof sum of rglob^2 plus the |R_f|^2 slots.
__global__ __launch_bounds__(kBlock) void norm_finalize_kernel(int n, const double* __restrict__ rglob,
                                                               const double* __restrict__ slots,
                                                               RedScratch* red, double* out) {
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        s += rglob[i] * rglob[i];
    s = wave_sum(s);
    __shared__ double ws[kBlock / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    __shared__ bool last;
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) b += ws[w];
        red->partial[blockIdx.x] = b;
        __threadfence();
        const unsigned prev = atomicAdd(&red->counter, 1u);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        double t = 0.0;
        for (unsigned k = 0; k < gridDim.x; ++k)
            t += __hip_atomic_load(&red->partial[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int k = 0; k < 64; ++k)
            t += __hip_atomic_load(&slots[k * 8], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        out[0] = sqrt(t);
        red->counter = 0u;
    }
}

__global__ void flags_reset_kernel(int32_t* flags) {
    if (threadIdx.x < 2) flags[threadIdx.x] = INT_MAX;
    if (threadIdx.x == 2) flags[2] = 0;
}

inline int grid_for(int64_t n, int block = kBlock) { return (int)((n + block - 1) / block); }

ElemArgs make_args(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double nu,
                   double inv_dt, const double* body) {
    ElemArgs a;
    a.xyz4 = c->xyz4;
    a.tets = c->tets;
    a.dmask = c->dmask;
    a.u = u;
    a.u_prev = u_prev;
    a.beta = beta;
    a.body = body;
    a.nu = nu;
    a.inv_dt = u_prev ? inv_dt : 0.0;
    a.n_elems = c->n_elems;
    a.flags = c->flags;
    return a;
}

double* slots_of(vms_ctx* c) { return c->red->acc_slots; }

}  // namespace

int launch_condense(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double nu,
                    double inv_dt, const double* body, void* A, double* rhs, double* rglob,
                    double* /*red_acc*/, hipStream_t s) {
    const size_t es = elt_size(c);
    int rc;
    if ((rc = launch_fill(A, (size_t)c->nb * 16 * es, s))) return rc;
    if ((rc = launch_fill(rhs, 4 * (size_t)c->n_nodes * sizeof(double), s))) return rc;
    if ((rc = launch_fill(rglob, 4 * (size_t)c->n_nodes * sizeof(double), s))) return rc;
    if ((rc = launch_fill(slots_of(c), 64 * 8 * sizeof(double), s))) return rc;
    flags_reset_kernel<<<1, 64, 0, s>>>(c->flags);
    ElemArgs a = make_args(c, u, u_prev, beta, nu, inv_dt, body);
    const int g = grid_for(c->n_elems);
    if (c->prec == VMS_FP64) {
        condense_kernel<double><<<g, kBlock, 0, s>>>(a, c->epos, (double*)A, rhs, rglob, slots_of(c));
        if (c->n_dir)
            dirichlet_diag_kernel<double><<<grid_for(c->n_dir), kBlock, 0, s>>>(c->n_dir, c->dlist, c->diagpos,
                                                                               (double*)A);
    } else {
        condense_kernel<float><<<g, kBlock, 0, s>>>(a, c->epos, (float*)A, rhs, rglob, slots_of(c));
        if (c->n_dir)
            dirichlet_diag_kernel<float><<<grid_for(c->n_dir), kBlock, 0, s>>>(c->n_dir, c->dlist, c->diagpos,
                                                                              (float*)A);
    }
    return check_hip(c, hipGetLastError(), "condense launch");
}

int launch_residual(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double nu,
                    double inv_dt, const double* body, double* rglob, double* /*red_acc*/, hipStream_t s) {
    int rc;
    if ((rc = launch_fill(rglob, 4 * (size_t)c->n_nodes * sizeof(double), s))) return rc;
    if ((rc = launch_fill(slots_of(c), 64 * 8 * sizeof(double), s))) return rc;
    flags_reset_kernel<<<1, 64, 0, s>>>(c->flags);
    ElemArgs a = make_args(c, u, u_prev, beta, nu, inv_dt, body);
    residual_kernel<<<grid_for(c->n_elems), kBlock, 0, s>>>(a, rglob, slots_of(c));
    return check_hip(c, hipGetLastError(), "residual launch");
}

int launch_norm_finalize(vms_ctx* c, const double* rglob, const double* /*red_acc*/, double* out,
                         hipStream_t s) {
    const int n = 4 * c->n_nodes;
    const int g = std::min(kRedBlocks, grid_for(n));
    norm_finalize_kernel<<<g, kBlock, 0, s>>>(n, rglob, slots_of(c), c->red, out);
    return check_hip(c, hipGetLastError(), "norm launch");
}

int check_element_flags(vms_ctx* c, hipStream_t s) {
    int32_t h[3];
    int rc = check_hip(c, hipMemcpyAsync(h, c->flags, sizeof h, hipMemcpyDeviceToHost, s), "flags");
    if (rc) return rc;
    if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
    if (h[0] != INT_MAX)
        return set_error(c, VMS_EDEGENERATE, "element " + std::to_string(h[0]) + " has det J <= 0");
    if (h[1] != INT_MAX)
        return set_error(c, VMS_ESINGULAR_KFF, "K_ff singular in element " + std::to_string(h[1]));
    return VMS_OK;
}

}  // namespace vms

using namespace vms;

static int check_state_args(vms_ctx* c, const double* u, const double* beta, double Re, double dt,
                            const double* u_prev, const char* who) {
    if (!c) return set_error(nullptr, VMS_EINVAL, std::string(who) + ": NULL ctx");
    if (!u || !beta) return set_error(c, VMS_EINVAL, std::string(who) + ": NULL u or beta");
    if (!(Re > 0.0) || !std::isfinite(Re)) return set_error(c, VMS_EINVAL, std::string(who) + ": Re must be > 0");
    if (dt > 0.0 && !u_prev) return set_error(c, VMS_EINVAL, std::string(who) + ": dt > 0 needs u_prev");
    return VMS_OK;
}

extern "C" int vms_element_tangents(vms_ctx* c, const double* u, const double* u_prev, const double* beta,
                                    double Re, double dt, const double* body, double* Ke, double* Rvec,
                                    hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_element_tangents");
    if (rc) return rc;
    flags_reset_kernel<<<1, 64, 0, s>>>(c->flags);
    ElemArgs a = make_args(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body);
    if (c->prec == VMS_FP64)
        raw_kernel<double><<<grid_for(c->n_elems), kBlock, 0, s>>>(a, Ke, Rvec);
    else
        raw_kernel<float><<<grid_for(c->n_elems), kBlock, 0, s>>>(a, Ke, Rvec);
    return check_hip(c, hipGetLastError(), "element tangents launch");
}

extern "C" int vms_condense_assemble(vms_ctx* c, const double* u, const double* u_prev, const double* beta,
                                     double Re, double dt, const double* body, void* bsr_vals, double* rhs,
                                     double* rnorm, hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_condense_assemble");
    if (rc) return rc;
    if (!bsr_vals || !rhs) return set_error(c, VMS_EINVAL, "vms_condense_assemble: NULL output");
    rc = launch_condense(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body,
                         bsr_vals, rhs, c->rglob, nullptr, s);
    if (rc) return rc;
    if (rnorm) return launch_norm_finalize(c, c->rglob, nullptr, rnorm, s);
    return VMS_OK;
}

extern "C" int vms_residual(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double Re,
                            double dt, const double* body, double* rglob, double* rnorm, hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_residual");
    if (rc) return rc;
    double* rg = rglob ? rglob : c->rglob;
    rc = launch_residual(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body, rg,
                         nullptr, s);
    if (rc) return rc;
    if (rnorm) return launch_norm_finalize(c, rg, nullptr, rnorm, s);
    return VMS_OK;
}

extern "C" int vms_recover_update(vms_ctx* c, double* u, double* beta, const double* u_prev, double Re,
                                  double dt, const double* body, const double* du, hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_recover_update");
    if (rc) return rc;
    if (!du) return set_error(c, VMS_EINVAL, "vms_recover_update: NULL du");
    flags_reset_kernel<<<1, 64, 0, s>>>(c->flags);
    ElemArgs a = make_args(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body);
    // beta is read and written by the same lane only, so the update is in place.
    recover_kernel<<<grid_for(c->n_elems), kBlock, 0, s>>>(a, du, beta);
    update_kernel<<<grid_for(4 * (int64_t)c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->dmask, du, u);
    return check_hip(c, hipGetLastError(), "recover launch");
}
