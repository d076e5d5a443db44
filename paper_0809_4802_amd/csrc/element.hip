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
#include <mutex>

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
    double adv;                          // 1: Newton tangent; 0: fixed-point tangent (advecting velocity held)
    int n_elems;
    unsigned long long* eflags;          // [0] degenerate element, [1] singular K_ff (flag_element)
    uint32_t gen;                        // call number written with a flag
};

// Element error flags: word `kind` (0: det J <= 0, 1: singular K_ff) holds gen << 32 | (2^32 - 1 - e)
// for the latest call number gen that met such an element, e the smallest of its elements: the
// maximum keeps the newest call and, within it, the smallest element.  A word of an earlier call
// reads as "no error", so no launch has to clear the flags before a kernel that sets them.
__device__ __forceinline__ void flag_element(const ElemArgs& a, int kind, int e) {
    atomicMax(&a.eflags[kind], ((unsigned long long)a.gen << 32) | (0xFFFFFFFFull - (unsigned)e));
}

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
    double adv;        // weight of the tangent's advecting-velocity terms (1 Newton, 0 fixed point)
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
    E.adv = A.adv;
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
        for (int j = 0; j < 3; ++j) Kff[i][j] = E.adv * E.C * E.G[i][j] + (i == j ? d : 0.0);
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
    const T B1 = T(E.adv * E.B1), hC = T(E.adv * 0.5 * E.C), B = T(E.B);
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
    const T B1 = T(E.adv * E.B1), hC = T(E.adv * 0.5 * E.C), B = T(E.B);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            K[i][j] = B1 * T(E.G[i][j]) - hC * T(E.be[i]) * T(E.g[a][j]) + (i == j ? diag : T(0));
#pragma unroll
    for (int j = 0; j < 3; ++j) K[3][j] = B * T(E.g[a][j]);
}

// K_cc(a,b): 4x4 block, precision T.  Gt, gt, Vt, bt are T copies of the fields; adv
// weighs the terms from the derivative of the advecting velocity (1 Newton, 0 fixed point).
template <typename T>
__device__ __forceinline__ void coarse_block(const T Gt[3][3], const T gt[4][3], const T Va[3],
                                             const T bt[3], T vol, T B1, T two_nu_vol, T inv_dt, T adv,
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
            K[i][j] = adv * (mab * Gt[i][j] - B1 * bt[i] * (gt[a][j] + gt[b][j])) + (i == j ? s : T(0));
        K[i][3] = qv * gt[a][i];
        K[3][i] = qv * gt[b][i];
    }
    K[3][3] = T(0);
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
    unsafeAtomicAdd(p, v);
}


// -------------------------------------------------------------------------------------------
// Tiled assembly.  Workgroup t owns the block rows of nodes [n0, n1) (a contiguous range, so
// its rows are the contiguous block range [rowptr[n0], rowptr[n1])) and stages them, with the
// rhs and residual rows, in LDS.  Its work items are the pairs (element e, local vertex a)
// with vertex a owned by the tile.  An item takes the element's vertices in the order
// (a, a^1, a^2, a^3), an even permutation (so the orientation and every element integral are
// unchanged), which puts the owned vertex first: every quantity of "the row's vertex" is then
// vertex 0's, with no per-lane selection.  The item forms the element's geometry, fields,
// R_f and K_ff^-1 (FP64), its own rows
//   R*_0 = R_cp,0 - K_cf(0) K_ff^-1 R_f,   Y = K_cf(0) K_ff^-1 (4x3),
// and the condensed blocks K*(0, b) = K_cc(0, b) - Y K_fc(b), b = 0..3, which it adds to the
// staged rows with LDS atomics.  The blocks are factored once per item so that each entry
// costs two or three FMAs (see block_factors).  After a barrier the tile writes its rows once
// with coalesced stores, and there the Dirichlet dofs are eliminated: a row or column of a
// prescribed dof becomes zero, its diagonal entry one, its rhs and residual entries zero (the
// per-block masks come precomputed from the host).  No global atomics, no zero fill, every
// condensed block computed exactly once.  Each tile also leaves two partial sums of the Newton
// residual norm (its free residual rows squared, and |R_f|^2 of the elements whose first
// vertex it owns), which a one-workgroup kernel adds in a fixed order.
//   CONDENSE = true : K* into Aval, -R* into rhs, R_cp into rglob (if not null), partials
//   CONDENSE = false: R_cp into rglob (if not null), partials (residual only)
//   SCHUR = false (with CONDENSE): the coarse blocks without condensation, K_cc into Aval and
//   -R_cp into rhs (the node-node part of the uncondensed system)
#ifndef VMS_TILE_THREADS
#define VMS_TILE_THREADS 256
#endif
constexpr int kTileThreads = VMS_TILE_THREADS;
// Deterministic contexts: tiles of one wavefront.  Its LDS additions then happen in program
// order (and, inside one instruction, in the hardware's fixed lane order), so every staged sum
// is formed in the same order on every run.
constexpr int kTileThreadsDet = 64;
#ifndef VMS_TILE_WAVES_PER_SIMD
#define VMS_TILE_WAVES_PER_SIMD 3
#endif

struct TileArgs {
    const int4* __restrict__ meta;        // per tile: (n0, n1, b0, nbk), (item0, item1, node base, nodes)
    const int32_t* __restrict__ nodes;
    const uint4* __restrict__ items;
    const uint16_t* __restrict__ bmask;   // per block: column node's Dirichlet bits (0..3),
                                          // row node's (4..7), diagonal block (bit 8)
};

// Factors of the condensed blocks of one item (row vertex 0), in precision T.  With
// Gt = adv G, bt = adv beta (the advecting-velocity terms), m_0b = (1 + delta_0b) |T| / 20,
// for rows r = 0..3 and velocity columns c = 0..2:
//   K*(0,b)[r][c] = P[r][c] + (r < 3) m_0b Gt[r][c] + q[r] g_b[c] - Y[r][c] d_b + delta_rc s_b
// with  P[r][c] = -B1 (bt[r] g_0[c] + (Y Gt)[r][c])  (r < 3),  P[3][c] = -B1 (Y Gt)[3][c],
//       q[r] = -B1 bt[r] + C/2 (Y bt)[r]  (r < 3),          q[3] = -|T|/4 + C/2 (Y bt)[3],
//       s_b = g_b . (V_0 + 2 nu |T| g_0 + B1 beta) + m_0b / dt,   d_b = g_b . (W + C beta) + B1 / dt,
// and the pressure column  K*(0,b)[r][3] = pc[r] - B (Y g_b)[r],  pc = (-|T|/4 g_0, 0).
// This is K_cc(0,b) - Y K_fc(b) with the closed-form blocks written out and regrouped by
// their dependence on b.
template <typename T>
struct BlockFactors {
    T Y[4][3];
    T P[4][3];
    T q[4];
    T pc[3];
    T Gt[3][3];
    T sv[3], dv[3];
    T g[4][3];
    T m0, idt, B1idt, Bm;
};

// DPP lane moves inside a quad (all four lanes active): lane ^ 1 and lane ^ 2.
template <int CTRL>
__device__ __forceinline__ float quad_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_mov(double v) {
    return dpp_mov<CTRL>(v);
}

// Reduce-scatter over the four lanes of a DPP quad of N values held as 4 rows of N/4: lane q
// receives in out the quad's sums of row 2 (q & 1) + (q >> 1).  Two exchange rounds, each
// lane sending the half it does not keep; every sum forms in the same order on every run.
template <int N, typename T>
__device__ __forceinline__ void quad_reduce_scatter(const T (&v)[N], T (&out)[N / 4], bool x1, bool x2) {
    constexpr int H = N / 2, Q = N / 4;
    T s[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const T send = x1 ? v[i] : v[H + i];
        const T keep = x1 ? v[H + i] : v[i];
        s[i] = keep + quad_mov<0xB1>(send);      // quad_perm [1,0,3,2]: lane ^ 1
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T send = x2 ? s[i] : s[Q + i];
        const T keep = x2 ? s[Q + i] : s[i];
        out[i] = keep + quad_mov<0x4E>(send);    // quad_perm [2,3,0,1]: lane ^ 2
    }
}

// The lane of a quad and the row of a 4 x k array its reduce-scatter share holds.
struct QuadLane {
    bool x1, x2;
    int row;
};
__device__ __forceinline__ QuadLane quad_lane() {
    const int q = (int)threadIdx.x & 3;
    return QuadLane{(q & 1) != 0, (q & 2) != 0, 2 * (q & 1) + (q >> 1)};
}

// Adds a 4-vector of an item (the owned row's residual entries) to rows[0..3].  With QUADS the
// four lanes of the quad share the owned row: the vector is reduce-scattered over the quad and
// each lane adds one entry (every lane of the quad must call it).
template <bool QUADS>
__device__ __forceinline__ void add_row4(double* rows, const double (&v)[4], bool live, const QuadLane& ql) {
    if (QUADS) {
        double z[4], o[1];
#pragma unroll
        for (int r = 0; r < 4; ++r) z[r] = live ? v[r] : 0.0;
        quad_reduce_scatter<4>(z, o, ql.x1, ql.x2);
        atomic_add(&rows[ql.row], o[0]);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (live) atomic_add(&rows[r], v[r]);
    }
}

// Entry (r, c) of condensed block b of one item (c = 3: the pressure column); gb = g_b and the
// block's scalars m_0b, s_b, d_b as in BlockFactors.
template <typename T>
__device__ __forceinline__ T block_entry(const BlockFactors<T>& F, const T* gb, T mab, T s_b, T d_b, int r, int c) {
    if (c < 3) {
        T x = F.P[r][c];
        if (r < 3) x += mab * F.Gt[r][c];
        x += F.q[r] * gb[c];
        x -= F.Y[r][c] * d_b;
        if (r == c) x += s_b;
        return x;
    }
    const T yg = F.Y[r][0] * gb[0] + F.Y[r][1] * gb[1] + F.Y[r][2] * gb[2];
    return (r < 3 ? F.pc[r] : T(0)) - F.Bm * yg;
}

// One item's four condensed blocks added to the staged rows.  With QUADS, block 0 (the row's
// diagonal block) is shared by the four items of a quad, and block 1 when the quad's elements
// share the edge to their vertex 1 (share1, the same for the four lanes): such a block is
// reduce-scattered over the quad, two columns at a time, and each lane adds one row of it --
// 4 LDS additions instead of 16.  The other blocks are added entry by entry by every live lane.
template <bool QUADS, typename T, typename TACC>
__device__ __forceinline__ void add_blocks(const BlockFactors<T>& F, TACC* __restrict__ blk, const uint32_t slot[4],
                                           bool live, bool share1, const QuadLane& ql) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const T* gb = F.g[b];
        const T mab = b == 0 ? T(2) * F.m0 : F.m0;
        const T s_b = gb[0] * F.sv[0] + gb[1] * F.sv[1] + gb[2] * F.sv[2] + mab * F.idt;
        const T d_b = gb[0] * F.dv[0] + gb[1] * F.dv[1] + gb[2] * F.dv[2] + F.B1idt;
        TACC* dst = blk + (size_t)slot[b] * kLdsBlockStride;
        if (QUADS && (b == 0 || (b == 1 && share1))) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                T v[8], o[2];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int k = 0; k < 2; ++k)
                        v[2 * r + k] = live ? block_entry(F, gb, mab, s_b, d_b, r, 2 * h + k) : T(0);
                quad_reduce_scatter<8>(v, o, ql.x1, ql.x2);
#pragma unroll
                for (int k = 0; k < 2; ++k) atomic_add(&dst[ql.row * 4 + 2 * h + k], TACC(o[k]));
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T v = F.P[r][c];
                    if (r < 3) v += mab * F.Gt[r][c];
                    v += F.q[r] * gb[c];
                    v -= F.Y[r][c] * d_b;
                    if (r == c) v += s_b;
                    if (live) atomic_add(&dst[r * 4 + c], TACC(v));
                }
                const T yg = F.Y[r][0] * gb[0] + F.Y[r][1] * gb[1] + F.Y[r][2] * gb[2];
                const T vp = (r < 3 ? F.pc[r] : T(0)) - F.Bm * yg;
                if (live) atomic_add(&dst[r * 4 + 3], TACC(vp));
            }
        }
    }
}

template <typename T, typename TACC, bool CONDENSE, bool SCHUR = true, int NT = kTileThreads>
__global__ __launch_bounds__(NT, VMS_TILE_WAVES_PER_SIMD) void tile_kernel(
    ElemArgs args, TileArgs ta, T* __restrict__ Aval, double* __restrict__ rhs, double* __restrict__ rglob,
    double* __restrict__ tile_part) {
    extern __shared__ __align__(16) unsigned char smem[];
    // DPP quads: the tiles of FP32 blocks take their items in quads of one row
    constexpr bool QUADS = sizeof(T) == 4;
    const QuadLane ql = quad_lane();
    const int t = blockIdx.x;
    const int4 m0 = ta.meta[2 * t], m1 = ta.meta[2 * t + 1];
    const int n0 = m0.x, nn = m0.y - m0.x, b0 = m0.z, nbk = m0.w;
    TACC* blk = reinterpret_cast<TACC*>(smem);
    const size_t off = CONDENSE ? align16((size_t)nbk * kLdsBlockStride * sizeof(TACC)) : 0;
    double* rr = reinterpret_cast<double*>(smem + off);
    double* rg = rr + (size_t)nn * 4;
    // the tile's nodes: coordinates, state and (transient) previous state, one double4 each
    const int nbase = m1.z, ntn = m1.w;
    double4* sx = reinterpret_cast<double4*>(rg + (size_t)nn * 4);
    double4* su = sx + ntn;
    double4* sup = su + ntn;
    __shared__ double wsum[NT / 64][2];

    const bool transient = args.u_prev != nullptr && args.inv_dt != 0.0;
    for (int i = threadIdx.x; i < ntn; i += blockDim.x) {
        const int g = ta.nodes[nbase + i];
        sx[i] = args.xyz4[g];
        su[i] = reinterpret_cast<const double4*>(args.u)[g];
        if (transient) sup[i] = reinterpret_cast<const double4*>(args.u_prev)[g];
    }
    // the write-out's masks, fetched now so that their latency hides behind the items: the
    // first two blocks of this thread (block masks) and its rhs entry's node (Dirichlet bits)
    constexpr int kPre = 2;
    uint32_t bm_pre[kPre];
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int kb = threadIdx.x + q * (int)blockDim.x;
        bm_pre[q] = (CONDENSE && kb < nbk) ? ta.bmask[b0 + kb] : 0u;
    }
    const uint32_t dm_pre = (int)threadIdx.x < nn * 4 ? args.dmask[n0 + (threadIdx.x >> 2)] : 0u;
    // zero the staged rows (blocks, then rhs and residual rows), 16 bytes per store; the block
    // region is padded to 16 bytes
    {
        const int nz = (CONDENSE ? (int)(off / 16) : 0) + nn * 4;
        double2* z = reinterpret_cast<double2*>(CONDENSE ? smem : smem + off);
        for (int i = threadIdx.x; i < nz; i += blockDim.x) z[i] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    const double nu = args.nu;
    const double inv_dt = transient ? args.inv_dt : 0.0;
    double rf2 = 0.0;
    const int k_end = m1.y;
    // item records are fetched one iteration ahead
    uint4 rec_next = m1.x + (int)threadIdx.x < k_end ? ta.items[m1.x + threadIdx.x] : make_uint4(0, 0, 0, 0);
    for (int k = m1.x + threadIdx.x; k < k_end; k += blockDim.x) {
        // item: element, local node numbers in the order (a, a^1, a^2, a^3) -- the owned vertex
        // first, orientation kept -- and the owned row's block slots
        const uint4 rec = rec_next;
        if (k + (int)blockDim.x < k_end) rec_next = ta.items[k + blockDim.x];
        // with QUADS, the four items of a quad (lanes 4m .. 4m+3) share the owned row and a
        // zero-weight copy pads a row's last quad; otherwise the two flag bits are zero
        const int e = (int)(rec.x & 0x7fffffffu);
        const bool dummy = (rec.x >> 31) != 0;
        const bool share1 = (rec.w >> 31) != 0;
        const int nl[4] = {(int)(rec.y & 255u), (int)((rec.y >> 8) & 255u), (int)((rec.y >> 16) & 255u),
                           (int)(rec.y >> 24)};
        // geometry
        double X[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double4 x = sx[nl[q]];
            X[q][0] = x.x;
            X[q][1] = x.y;
            X[q][2] = x.z;
        }
        double J[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) J[i][c] = X[c + 1][i] - X[0][i];
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        // a degenerate element is flagged and contributes nothing (its lane stays in its quad)
        const bool degenerate = !(det > 0.0);
        if (degenerate) flag_element(args, 0, e);
        const bool live = !dummy && !degenerate;
        const bool first = live && (rec.z & 0x8000u) != 0;   // the element's vertex 0 (R_f counted once)
        const double id = degenerate ? 0.0 : 1.0 / det;
        double g[4][3];
        g[1][0] = c00 * id;
        g[1][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
        g[1][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
        g[2][0] = c01 * id;
        g[2][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
        g[2][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
        g[3][0] = c02 * id;
        g[3][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
        g[3][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
        for (int i = 0; i < 3; ++i) g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
        const double vol = det * (1.0 / 6.0);
        double gg = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) gg += g[q][0] * g[q][0] + g[q][1] * g[q][1] + g[q][2] * g[q][2];
        const double B1 = kB1 * vol, Bm = kB * vol, Cm = kC * vol, Kb = kKb * vol * gg;
        const double m0 = vol * (1.0 / 20.0);

        // fields: G = grad vbar, grad p, sums over vertices; vertex 0's own values
        double G[3][3] = {}, gp[3] = {}, vs[3] = {}, ps = 0.0, v0[3] = {};
        double dvs[3] = {}, dv0[3] = {}, fs[3] = {}, f0[3] = {};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double4 uu = su[nl[q]];
            const double vq[3] = {uu.x, uu.y, uu.z};
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j) G[i][j] += vq[i] * g[q][j];
                gp[i] += uu.w * g[q][i];
                vs[i] += vq[i];
                if (q == 0) v0[i] = vq[i];
            }
            ps += uu.w;
            if (transient) {
                const double4 up = sup[nl[q]];
                const double d[3] = {vq[0] - up.x, vq[1] - up.y, vq[2] - up.z};
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    dvs[i] += d[i];
                    if (q == 0) dv0[i] = d[i];
                }
            }
            if (args.body) {
                const size_t gq = (size_t)ta.nodes[nbase + nl[q]];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double f = args.body[3 * gq + i];
                    fs[i] += f;
                    if (q == 0) f0[i] = f;
                }
            }
        }
        const double th = G[0][0] + G[1][1] + G[2][2];
        const double* bp = args.beta + 3 * (size_t)e;
        const double be[3] = {bp[0], bp[1], bp[2]};
        double Wv[3], Va[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Wv[i] = B1 * vs[i];
            Va[i] = m0 * (vs[i] + v0[i]);
        }
        // fine-scale residual (counted in the norm once per element: by its first vertex's item)
        double Rf[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            Rf[i] = G[i][0] * Wv[0] + G[i][1] * Wv[1] + G[i][2] * Wv[2] +
                    Cm * (G[i][0] * be[0] + G[i][1] * be[1] + G[i][2] * be[2] - 0.5 * th * be[i]) +
                    2.0 * nu * Kb * be[i] + Bm * gp[i] - B1 * fs[i] + inv_dt * B1 * dvs[i];
        if (first) rf2 += Rf[0] * Rf[0] + Rf[1] * Rf[1] + Rf[2] * Rf[2];
        // coarse residual rows of vertex 0
        const double g0W = g[0][0] * Wv[0] + g[0][1] * Wv[1] + g[0][2] * Wv[2];
        const double bg0 = be[0] * g[0][0] + be[1] * g[0][1] + be[2] * g[0][2];
        double Rc[4];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            Rc[i] = G[i][0] * (Va[0] + B1 * be[0]) + G[i][1] * (Va[1] + B1 * be[1]) + G[i][2] * (Va[2] + B1 * be[2]) -
                    (g0W + th * B1 + 0.5 * Cm * bg0) * be[i] +
                    2.0 * nu * vol * (G[i][0] * g[0][0] + G[i][1] * g[0][1] + G[i][2] * g[0][2]) -
                    0.25 * vol * ps * g[0][i] - m0 * (fs[i] + f0[i]) + inv_dt * m0 * (dvs[i] + dv0[i]);
        Rc[3] = -th * vol * 0.25 + Bm * bg0;
        const int la = nl[0];                           // owned nodes come first in the local numbering
        if constexpr (QUADS) {
            add_row4<QUADS>(&rg[4 * la], Rc, live, ql);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (live) atomic_add(&rg[4 * la + r], Rc[r]);
        }
        if (!CONDENSE) continue;

        // Y = K_cf(0) K_ff^-1 (FP64, stored in T) and R*_0; zero without condensation
        double Yd[4][3] = {};
        if (SCHUR) {
            const double dk = 2.0 * nu * Kb - 0.5 * Cm * th;
            double Kff[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) Kff[i][j] = args.adv * Cm * G[i][j] + (i == j ? dk : 0.0);
            const double k00 = Kff[1][1] * Kff[2][2] - Kff[1][2] * Kff[2][1];
            const double k01 = Kff[1][2] * Kff[2][0] - Kff[1][0] * Kff[2][2];
            const double k02 = Kff[1][0] * Kff[2][1] - Kff[1][1] * Kff[2][0];
            const double kdet = Kff[0][0] * k00 + Kff[0][1] * k01 + Kff[0][2] * k02;
            double knrm = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) knrm = fmax(knrm, fabs(Kff[i][0]) + fabs(Kff[i][1]) + fabs(Kff[i][2]));
            if (live && !(fabs(kdet) > 1e-14 * knrm * knrm * knrm)) flag_element(args, 1, e);
            const double kid = 1.0 / kdet;
            double Ki[3][3];
            Ki[0][0] = k00 * kid;
            Ki[0][1] = (Kff[0][2] * Kff[2][1] - Kff[0][1] * Kff[2][2]) * kid;
            Ki[0][2] = (Kff[0][1] * Kff[1][2] - Kff[0][2] * Kff[1][1]) * kid;
            Ki[1][0] = k01 * kid;
            Ki[1][1] = (Kff[0][0] * Kff[2][2] - Kff[0][2] * Kff[2][0]) * kid;
            Ki[1][2] = (Kff[0][2] * Kff[1][0] - Kff[0][0] * Kff[1][2]) * kid;
            Ki[2][0] = k02 * kid;
            Ki[2][1] = (Kff[0][1] * Kff[2][0] - Kff[0][0] * Kff[2][1]) * kid;
            Ki[2][2] = (Kff[0][0] * Kff[1][1] - Kff[0][1] * Kff[1][0]) * kid;
            // K_cf(0): velocity rows, then the pressure row
            const double dg = -(g0W + th * B1) - 0.5 * Cm * bg0;
            double Kcf[4][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Kcf[i][j] = args.adv * (B1 * G[i][j] - 0.5 * Cm * be[i] * g[0][j]) + (i == j ? dg : 0.0);
#pragma unroll
            for (int j = 0; j < 3; ++j) Kcf[3][j] = Bm * g[0][j];
            double zf[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) zf[i] = Ki[i][0] * Rf[0] + Ki[i][1] * Rf[1] + Ki[i][2] * Rf[2];
            // R*_0 = R_c(0) - K_cf(0) K_ff^-1 R_f, staged negated
            if constexpr (QUADS) {
                double nrs[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    nrs[r] = -(Rc[r] - (Kcf[r][0] * zf[0] + Kcf[r][1] * zf[1] + Kcf[r][2] * zf[2]));
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        Yd[r][j] = Kcf[r][0] * Ki[0][j] + Kcf[r][1] * Ki[1][j] + Kcf[r][2] * Ki[2][j];
                }
                add_row4<QUADS>(&rr[4 * la], nrs, live, ql);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double rs = Rc[r] - (Kcf[r][0] * zf[0] + Kcf[r][1] * zf[1] + Kcf[r][2] * zf[2]);
                    if (live) atomic_add(&rr[4 * la + r], -rs);
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        Yd[r][j] = Kcf[r][0] * Ki[0][j] + Kcf[r][1] * Ki[1][j] + Kcf[r][2] * Ki[2][j];
                }
            }
        } else if constexpr (QUADS) {
            const double nrc[4] = {-Rc[0], -Rc[1], -Rc[2], -Rc[3]};
            add_row4<QUADS>(&rr[4 * la], nrc, live, ql);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (live) atomic_add(&rr[4 * la + r], -Rc[r]);
        }

        // block factors in T
        BlockFactors<T> F;
        const double av = args.adv;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < 3; ++i) F.g[q][i] = T(g[q][i]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) F.Gt[i][j] = T(av * G[i][j]);
        T bt[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            bt[i] = T(av * be[i]);
            F.sv[i] = T(Va[i] + 2.0 * nu * vol * g[0][i] + B1 * be[i]);
            F.dv[i] = T(Wv[i] + Cm * be[i]);
            F.pc[i] = T(-0.25 * vol * g[0][i]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 3; ++j) F.Y[r][j] = T(Yd[r][j]);
        const T B1t = T(B1), hCt = T(0.5 * Cm);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T yb = F.Y[r][0] * bt[0] + F.Y[r][1] * bt[1] + F.Y[r][2] * bt[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T yg = F.Y[r][0] * F.Gt[0][c] + F.Y[r][1] * F.Gt[1][c] + F.Y[r][2] * F.Gt[2][c];
                F.P[r][c] = -B1t * ((r < 3 ? bt[r] * F.g[0][c] : T(0)) + yg);
            }
            F.q[r] = (r < 3 ? -B1t * bt[r] : T(-0.25 * vol)) + hCt * yb;
        }
        F.m0 = T(m0);
        F.idt = T(inv_dt);
        F.B1idt = T(B1 * inv_dt);
        F.Bm = T(Bm);
        const uint32_t slot[4] = {rec.z & 0x7fffu, rec.z >> 16, rec.w & 0xffffu, (rec.w >> 16) & 0x7fffu};
        add_blocks<QUADS, T, TACC>(F, blk, slot, live, share1, ql);
    }
    __syncthreads();
    if (CONDENSE) {
        // write the rows once, a block per thread, eliminating the Dirichlet dofs: zero rows and
        // columns, unit diagonal
        using V4 = typename Vec4<T>::type;
        for (int q = 0, kb = threadIdx.x; kb < nbk; ++q, kb += blockDim.x) {
            const uint32_t bm = q < kPre ? bm_pre[q] : ta.bmask[b0 + kb];
            const TACC* src = blk + (size_t)kb * kLdsBlockStride;
            V4* dst = reinterpret_cast<V4*>(Aval + ((size_t)b0 + kb) * 16);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T v[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    v[c] = T(src[4 * r + c]);
                    if (((bm >> (4 + r)) | (bm >> c)) & 1u) v[c] = ((bm & 0x100u) && r == c) ? T(1) : T(0);
                }
                V4 w;
                w.x = v[0];
                w.y = v[1];
                w.z = v[2];
                w.w = v[3];
                dst[r] = w;
            }
        }
    }
    double rg2 = 0.0;
    for (int i = threadIdx.x; i < nn * 4; i += blockDim.x) {
        const uint32_t dm = i == (int)threadIdx.x ? dm_pre : args.dmask[n0 + (i >> 2)];
        const bool fixed = (dm >> (i & 3)) & 1u;
        const double rv = fixed ? 0.0 : rg[i];
        rg2 += rv * rv;
        if (rglob) rglob[4 * (size_t)n0 + i] = rv;
        if (CONDENSE) rhs[4 * (size_t)n0 + i] = fixed ? 0.0 : rr[i];
    }
    rg2 = wave_sum(rg2);
    rf2 = wave_sum(rf2);
    if ((threadIdx.x & 63) == 0) {
        wsum[threadIdx.x >> 6][0] = rg2;
        wsum[threadIdx.x >> 6][1] = rf2;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += wsum[w][threadIdx.x];
        tile_part[2 * (size_t)t + threadIdx.x] = s;
    }
}

// Raw element residual and 19x19 tangent (tangent blocks in T, K_ff in FP64).
template <typename T>
__global__ __launch_bounds__(kBlock) void raw_kernel(ElemArgs args, double* __restrict__ Ke,
                                                     double* __restrict__ Rv) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= args.n_elems) return;
    Elem E;
    if (!load_element(args, e, E)) {
        flag_element(args, 0, e);
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
            coarse_block<T>(Gt, gt, Va, bt, volt, B1t, tnv, idt, T(E.adv), a, b, Kb);
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
    if (!fine_block_inverse(E, nu, Ki, Kff)) flag_element(args, 1, e);
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
        flag_element(args, 0, e);
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
    if (!fine_block_inverse(E, nu, Ki, Kff)) flag_element(args, 1, e);
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

// Newton residual norm from the assembly tiles' partial sums (free residual rows squared,
// |R_f|^2), added in a fixed order by one workgroup: thread i takes partials i, i + 1024, ...,
// then a fixed tree over the waves.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void norm_finalize_kernel(int n_tiles, const double* __restrict__ part,
                                                                     double* __restrict__ out) {
    // a thread's partials are loaded eight at a time (one memory round per batch instead of a
    // chain of dependent loads) and added in increasing index order, as before
    constexpr int kBatch = 8;
    const int n = 2 * n_tiles;
    double s = 0.0;
    for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * kFinThreads) {
        double v[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int i = i0 + b * kFinThreads;
            v[b] = part[min(i, n - 1)];
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            if (i0 + b * kFinThreads < n) s += v[b];
    }
    s = wave_sum(s);
    __shared__ double ws[kFinThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kFinThreads / 64; ++w) tot += ws[w];
        out[0] = sqrt(tot);
    }
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
    a.adv = c->linearization == VMS_LIN_PICARD ? 0.0 : 1.0;
    a.n_elems = c->n_elems;
    a.eflags = element_flags(c);
    a.gen = c->elem_gen;
    return a;
}

// Launches tile_kernel<T, TACC, CONDENSE, SCHUR> at the context's tile width (256 threads, or one
// wavefront in deterministic contexts).
template <typename T, typename TACC, bool CONDENSE, bool SCHUR = true>
void launch_tiles(const vms_ctx* c, const ElemArgs& a, const TileArgs& ta, size_t lds, T* Aval, double* rhs,
                  double* rglob, double* part, hipStream_t s) {
    if (c->tile_threads == kTileThreadsDet)
        tile_kernel<T, TACC, CONDENSE, SCHUR, kTileThreadsDet><<<c->n_tiles, kTileThreadsDet, lds, s>>>(
            a, ta, Aval, rhs, rglob, part);
    else
        tile_kernel<T, TACC, CONDENSE, SCHUR, kTileThreads><<<c->n_tiles, kTileThreads, lds, s>>>(a, ta, Aval, rhs,
                                                                                                 rglob, part);
}

// dynamic LDS of a tile launch: the previous velocity is staged only in transient launches
size_t tile_lds_of(const vms_ctx* c, const ElemArgs& a) {
    return (a.u_prev != nullptr && a.inv_dt != 0.0) ? c->tile_lds_tr : c->tile_lds;
}

TileArgs tile_args(vms_ctx* c) {
    TileArgs t;
    t.meta = c->tile_meta;
    t.nodes = c->tile_nodes;
    t.items = c->items;
    t.bmask = c->bmask;
    return t;
}

}  // namespace

hipError_t tile_kernels_configure(vms_ctx* c) {
    const int lds = (int)std::max(c->tile_lds, c->tile_lds_tr);
    const void* fns[] = {
        (const void*)tile_kernel<double, double, true, true, kTileThreads>,
        (const void*)tile_kernel<float, MixedAcc, true, true, kTileThreads>,
        (const void*)tile_kernel<double, double, false, true, kTileThreads>,
        (const void*)tile_kernel<double, double, true, false, kTileThreads>,
        (const void*)tile_kernel<float, MixedAcc, true, false, kTileThreads>,
        (const void*)tile_kernel<double, double, true, true, kTileThreadsDet>,
        (const void*)tile_kernel<float, MixedAcc, true, true, kTileThreadsDet>,
        (const void*)tile_kernel<double, double, false, true, kTileThreadsDet>,
        (const void*)tile_kernel<double, double, true, false, kTileThreadsDet>,
        (const void*)tile_kernel<float, MixedAcc, true, false, kTileThreadsDet>};
    hipError_t e = hipSuccess;
    for (const void* f : fns)
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return e;
}

// Uncondensed system, element part (one lane per element): the coupling blocks K_cf(a)
// (node a's row, the element's column; fourth column 0), K_fc(b) (the element's row, node b's
// column; fourth row 0) and K_ff (element diagonal, unit fourth diagonal) written to their
// unique positions, Dirichlet rows and columns zeroed; the element's rhs rows -R_f.
template <typename T>
__global__ __launch_bounds__(kBlock) void full_element_kernel(ElemArgs args, int n_nodes,
                                                              const int32_t* __restrict__ epos,
                                                              T* __restrict__ vals, double* __restrict__ rhs) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= args.n_elems) return;
    Elem E;
    if (!load_element(args, e, E)) {
        flag_element(args, 0, e);
        return;
    }
    const double nu = args.nu, inv_dt = E.transient ? args.inv_dt : 0.0;
    const int nid[4] = {E.t.x, E.t.y, E.t.z, E.t.w};
    uint32_t dm[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) dm[a] = args.dmask[nid[a]];
    const int32_t* ep = epos + 9 * (size_t)e;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        T Kcf[4][3];
        coarse_fine_block<T>(E, a, Kcf);
        T* dst = vals + (size_t)ep[a] * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool keep = !(dm[a] & (1u << r));
#pragma unroll
            for (int q = 0; q < 3; ++q) dst[4 * r + q] = keep ? Kcf[r][q] : T(0);
            dst[4 * r + 3] = T(0);
        }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        T Kfc[3][4];
        fine_coarse_block<T>(E, b, inv_dt, Kfc);
        T* dst = vals + (size_t)ep[4 + b] * 16;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[4 * i + q] = (dm[b] & (1u << q)) ? T(0) : Kfc[i][q];
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[12 + q] = T(0);
    }
    double Ki[3][3], Kff[3][3];
    fine_block_inverse(E, nu, Ki, Kff);
    T* dst = vals + (size_t)ep[8] * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[4 * i + q] = (i < 3 && q < 3) ? T(Kff[i][q]) : T(i == q ? 1 : 0);
    double Rf[3];
    fine_residual(E, nu, inv_dt, Rf);
    double* rr = rhs + 4 * ((size_t)n_nodes + e);
    rr[0] = -Rf[0];
    rr[1] = -Rf[1];
    rr[2] = -Rf[2];
    rr[3] = 0.0;
}

// Node-node blocks (condensed pattern) and node rhs rows into the uncondensed system.
template <typename T>
__global__ void full_copy_kernel(int64_t nb, int n4, const int32_t* __restrict__ cc, const T* __restrict__ src,
                                 T* __restrict__ dst, const double* __restrict__ rsrc, double* __restrict__ rdst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nb * 16) dst[(size_t)cc[i >> 4] * 16 + (i & 15)] = src[i];
    if (i < n4) rdst[i] = rsrc[i];
}

// u += dx (node rows), beta += dx (element rows, first three entries).
__global__ void full_update_kernel(int n_nodes, int n_elems, const double* __restrict__ dx, double* __restrict__ u,
                                   double* __restrict__ beta) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < 4 * (int64_t)n_nodes) u[i] += dx[i];
    if (i < 3 * (int64_t)n_elems) {
        const int64_t e = i / 3, q = i - 3 * e;
        beta[i] += dx[4 * ((int64_t)n_nodes + e) + q];
    }
}

int launch_full_assemble(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double nu,
                         double inv_dt, const double* body, void* vals, double* rhs, hipStream_t s) {
    ++c->elem_gen;                       // a new call number for the element flags
    ElemArgs a = make_args(c, u, u_prev, beta, nu, inv_dt, body);
    const int64_t nb16 = c->nb * 16;
    const int n4 = 4 * c->n_nodes;
    const int gcopy = (int)((std::max<int64_t>(nb16, n4) + kBlock - 1) / kBlock);
    if (c->prec == VMS_FP64) {
        launch_tiles<double, double, true, false>(c, a, tile_args(c), tile_lds_of(c, a), (double*)c->A, c->rhs,
                                                  nullptr, c->tile_part, s);
        full_element_kernel<double><<<grid_for(c->n_elems), kBlock, 0, s>>>(a, c->n_nodes, c->full_epos,
                                                                            (double*)vals, rhs);
        full_copy_kernel<double><<<gcopy, kBlock, 0, s>>>(c->nb, n4, c->full_cc, (const double*)c->A,
                                                          (double*)vals, c->rhs, rhs);
    } else {
        launch_tiles<float, MixedAcc, true, false>(c, a, tile_args(c), tile_lds_of(c, a), (float*)c->A, c->rhs,
                                                   nullptr, c->tile_part, s);
        full_element_kernel<float><<<grid_for(c->n_elems), kBlock, 0, s>>>(a, c->n_nodes, c->full_epos,
                                                                          (float*)vals, rhs);
        full_copy_kernel<float><<<gcopy, kBlock, 0, s>>>(c->nb, n4, c->full_cc, (const float*)c->A, (float*)vals,
                                                         c->rhs, rhs);
    }
    return check_hip(c, hipGetLastError(), "full assemble launch");
}

int launch_full_update(vms_ctx* c, const double* dx, double* u, double* beta, hipStream_t s) {
    const int64_t n = std::max<int64_t>(4 * (int64_t)c->n_nodes, 3 * (int64_t)c->n_elems);
    full_update_kernel<<<grid_for(n), kBlock, 0, s>>>(c->n_nodes, c->n_elems, dx, u, beta);
    return check_hip(c, hipGetLastError(), "full update launch");
}

// The condensed assembly with its scratch (element flags, per-tile norm partials) at the given
// device addresses: the context's own buffers, or the static scratch of the no-allocation entry.
static int launch_condense_in(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double nu,
                              double inv_dt, const double* body, void* A, double* rhs, double* rglob,
                              unsigned long long* eflags, double* tile_part, hipStream_t s) {
    const size_t es = elt_size(c);
    const double nn = c->n_nodes, ne = c->n_elems;
    ++c->elem_gen;                       // a new call number for the element flags
    ElemArgs a = make_args(c, u, u_prev, beta, nu, inv_dt, body);
    a.eflags = eflags;
    // algorithmic bytes: connectivity + beta per element; coordinates, state (and previous
    // velocity, body force) per node; block-CSR values and rhs written once (and the residual
    // rows, when asked for)
    const double alg = ne * (16.0 + 24.0) + nn * (24.0 + 32.0 + (a.u_prev ? 24.0 : 0.0) + (body ? 24.0 : 0.0)) +
                       (double)c->nb * 16 * es + 32.0 * nn * (rglob ? 2.0 : 1.0);
    PhaseScope ph(c, VMS_PH_CONDENSE, alg, s);
    if (c->prec == VMS_FP64)
        launch_tiles<double, double, true>(c, a, tile_args(c), tile_lds_of(c, a), (double*)A, rhs, rglob, tile_part, s);
    else
        launch_tiles<float, MixedAcc, true>(c, a, tile_args(c), tile_lds_of(c, a), (float*)A, rhs, rglob, tile_part, s);
    return check_hip(c, hipGetLastError(), "condense launch");
}

int launch_condense(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double nu,
                    double inv_dt, const double* body, void* A, double* rhs, double* rglob, hipStream_t s) {
    return launch_condense_in(c, u, u_prev, beta, nu, inv_dt, body, A, rhs, rglob, element_flags(c), c->tile_part,
                              s);
}

int launch_residual(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double nu,
                    double inv_dt, const double* body, double* rglob, hipStream_t s) {
    ++c->elem_gen;                       // a new call number for the element flags
    ElemArgs a = make_args(c, u, u_prev, beta, nu, inv_dt, body);
    {
        const double nn = c->n_nodes, ne = c->n_elems;
        PhaseScope ph(c, VMS_PH_RESIDUAL,
                      ne * 40.0 + nn * (56.0 + (a.u_prev ? 24.0 : 0.0) + (body ? 24.0 : 0.0)) +
                          (rglob ? 32.0 * nn : 0.0), s);
        launch_tiles<double, double, false>(c, a, tile_args(c), tile_lds_of(c, a), (double*)nullptr, nullptr, rglob,
                                            c->tile_part, s);
    }
    return check_hip(c, hipGetLastError(), "residual launch");
}

static int launch_norm_finalize_in(vms_ctx* c, const double* tile_part, double* out, hipStream_t s) {
    norm_finalize_kernel<<<1, kFinThreads, 0, s>>>(c->n_tiles, tile_part, out);
    return check_hip(c, hipGetLastError(), "norm launch");
}

int launch_norm_finalize(vms_ctx* c, double* out, hipStream_t s) {
    return launch_norm_finalize_in(c, c->tile_part, out, s);
}

// ---- scratch of the no-allocation entry point -----------------------------------------
// One static array per device (each GPU the library runs on holds its own copy until the
// process ends): the element flags, then the per-tile partial sums of the residual norm.
constexpr int kNoallocMaxTiles = 1 << 16;
constexpr size_t kNoallocFlagBytes = 256;
constexpr size_t kNoallocBytes = kNoallocFlagBytes + 2 * sizeof(double) * kNoallocMaxTiles;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::once_flag g_scratch_once[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (hipGetSymbolAddress, once per device, with
// that device current).  Host code uses only this address: the array's own name is a host-side
// stand-in, not a device address.
static int noalloc_scratch(vms_ctx* c, unsigned char** out) {
    const int dev = c->device;
    if (dev < 0 || dev >= kMaxDevices) return set_error(c, VMS_EINVAL, "no-allocation scratch: device index");
    std::call_once(g_scratch_once[dev], [dev]() {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        g_scratch_err[dev] = e;
        g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
        return check_hip(c, g_scratch_err[dev] != hipSuccess ? g_scratch_err[dev] : hipErrorInvalidSymbol,
                         "no-allocation scratch address");
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return VMS_OK;
}

int noalloc_scratch_init(vms_ctx* c) {
    unsigned char* p = nullptr;
    return noalloc_scratch(c, &p);
}

int check_element_flags(vms_ctx* c, hipStream_t s) {
    unsigned long long h[2];
    int rc = check_hip(c, hipMemcpyAsync(h, element_flags(c), sizeof h, hipMemcpyDeviceToHost, s), "flags");
    if (rc) return rc;
    if ((rc = check_hip(c, hipStreamSynchronize(s), "sync"))) return rc;
    // flags of the current call number only (flag_element)
    auto elem = [&](int k) -> long long {
        return (uint32_t)(h[k] >> 32) == c->elem_gen ? (long long)(0xFFFFFFFFull - (h[k] & 0xFFFFFFFFull)) : -1;
    };
    if (elem(0) >= 0) return set_error(c, VMS_EDEGENERATE, "element " + std::to_string(elem(0)) + " has det J <= 0");
    if (elem(1) >= 0) return set_error(c, VMS_ESINGULAR_KFF, "K_ff singular in element " + std::to_string(elem(1)));
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
    ++c->elem_gen;                       // a new call number for the element flags
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
                         bsr_vals, rhs, nullptr, s);
    if (rc) return rc;
    if (rnorm) return launch_norm_finalize(c, rnorm, s);
    return VMS_OK;
}

extern "C" int vms_condense_assemble_noalloc(vms_ctx* c, const double* u, const double* u_prev, const double* beta,
                                             double Re, double dt, const double* body, void* bsr_vals, double* rhs,
                                             double* rnorm, hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_condense_assemble_noalloc");
    if (rc) return rc;
    if (!bsr_vals || !rhs) return set_error(c, VMS_EINVAL, "vms_condense_assemble_noalloc: NULL output");
    if (c->n_tiles > kNoallocMaxTiles)
        return set_error(c, VMS_EINVAL, "vms_condense_assemble_noalloc: " + std::to_string(c->n_tiles) +
                                            " assembly tiles exceed the static scratch (" +
                                            std::to_string(kNoallocMaxTiles) + ")");
    unsigned char* base = nullptr;
    if ((rc = noalloc_scratch(c, &base))) return rc;
    unsigned long long* flags = reinterpret_cast<unsigned long long*>(base);
    double* part = reinterpret_cast<double*>(base + kNoallocFlagBytes);
    rc = launch_condense_in(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body,
                            bsr_vals, rhs, nullptr, flags, part, s);
    if (rc) return rc;
    if (rnorm) return launch_norm_finalize_in(c, part, rnorm, s);
    return VMS_OK;
}

extern "C" int vms_full_assemble(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double Re,
                                 double dt, const double* body, void* bsr_vals, double* rhs, double* rnorm,
                                 hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_full_assemble");
    if (rc) return rc;
    if (!c->full) return set_error(c, VMS_EINVAL, "vms_full_assemble: context created without full_system");
    if (!bsr_vals || !rhs) return set_error(c, VMS_EINVAL, "vms_full_assemble: NULL output");
    rc = launch_full_assemble(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body,
                              bsr_vals, rhs, s);
    if (rc) return rc;
    if (rnorm) return launch_norm_finalize(c, rnorm, s);
    return VMS_OK;
}

extern "C" int vms_residual(vms_ctx* c, const double* u, const double* u_prev, const double* beta, double Re,
                            double dt, const double* body, double* rglob, double* rnorm, hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_residual");
    if (rc) return rc;
    rc = launch_residual(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body, rglob, s);
    if (rc) return rc;
    if (rnorm) return launch_norm_finalize(c, rnorm, s);
    return VMS_OK;
}

extern "C" int vms_recover_update(vms_ctx* c, double* u, double* beta, const double* u_prev, double Re,
                                  double dt, const double* body, const double* du, hipStream_t s) {
    int rc = check_state_args(c, u, beta, Re, dt, u_prev, "vms_recover_update");
    if (rc) return rc;
    if (!du) return set_error(c, VMS_EINVAL, "vms_recover_update: NULL du");
    ++c->elem_gen;                       // a new call number for the element flags
    ElemArgs a = make_args(c, u, dt > 0 ? u_prev : nullptr, beta, 1.0 / Re, dt > 0 ? 1.0 / dt : 0.0, body);
    // beta is read and written by the same lane only, so the update is in place.
    {
        const double nn = c->n_nodes, ne = c->n_elems;
        PhaseScope ph(c, VMS_PH_RECOVER,
                      ne * (16.0 + 48.0) + nn * (56.0 + 32.0 + (a.u_prev ? 24.0 : 0.0) + (body ? 24.0 : 0.0)), s);
        recover_kernel<<<grid_for(c->n_elems), kBlock, 0, s>>>(a, du, beta);
    }
    update_kernel<<<grid_for(4 * (int64_t)c->n_nodes), kBlock, 0, s>>>(c->n_nodes, c->dmask, du, u);
    return check_hip(c, hipGetLastError(), "recover launch");
}
