/*
 * ORACLE -- test infrastructure only.  Only tests/, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.
 *
 * Element residual and consistent Newton tangent of the two-level
 * variational multiscale (VMS) weak form for linear tetrahedra with one
 * bubble per element, integrated by quadrature of the pointwise integrands.
 *
 *   Weak form (Section 3.2, coarse momentum / continuity / fine momentum):
 *     momentum rows, test function w (coarse  w = N_a e_i, or fine  w = b e_i):
 *        (w, (v.grad) v) + (grad w, 2 nu grad v) - (div w, p) - (w, f)
 *        [+ (w, (vbar - vbar_n) / dt) for transient runs, Section 4.1 Remark]
 *     continuity rows, test function q = N_a:
 *        -(q, div v)              (sign of the pressure residual, Section 4.1)
 *   with v = vbar + v',  vbar = sum_a N_a v_a,  v' = b beta  (Section 3.3),
 *   grad v' = beta (grad b)^T,  p = sum_a N_a p_a.  The traction term is zero
 *   (no workload prescribes a nonzero traction).
 *
 *   The transient term acts on the coarse velocity only, in the coarse and
 *   the fine rows alike: the fine scales are quasi-static (Section 4.1 Remark).
 *
 *   Tangent (Section 4.2, the 3x3-block Newton system): the derivative of each
 *   row's integrand in the direction of each of the 19 element unknowns
 *     d[(v.grad)v] = (dv.grad) v + (v.grad) dv,
 *   integrated with the same rule.  This is a pointwise linearisation,
 *   written independently of any closed-form integration.  With picard = 1 the
 *   advecting velocity is held at the current iterate (the fixed-point
 *   linearisation the introduction contrasts with Newton's): d[(v.grad)v] =
 *   (v.grad) dv only.
 *
 *   For tests of that tangent the advecting velocity of the residual can be
 *   taken from a separate state (u_adv, beta_adv; NULL: the state itself):
 *   the convective term is then (v_adv.grad) v, affine in the unknowns.
 *
 *   Bubble b = c * 256 l0 l1 l2 l3 (barycentric l_a; c = 1 normally; the
 *   paper leaves the bubble unspecified, see Section 3.3).
 *
 * Dof order inside an element: (v0x, v0y, v0z, p0, ..., v3x, v3y, v3z, p3,
 * beta_x, beta_y, beta_z).  Layouts (host, row-major, AoS):
 *   xyz [n_nodes][3], tets [n_elems][4], u [n_nodes][4], u_prev [n_nodes][4]
 *   or NULL (steady), beta [n_elems][3], body [n_nodes][3] or NULL,
 *   lam [nq][4], w [nq] (reference weights summing to 1/6),
 *   R [n_elems][19], K [n_elems][19][19] or NULL; u_adv [n_nodes][4] and
 *   beta_adv [n_elems][3] or NULL (both or neither).
 * Returns 0, or 1 + (index of the first element with det J <= 0).
 */
#include <stdint.h>
#include <string.h>

#define NDOF 19

static double tet_geometry(const double X[4][3], double g[4][3])
{
    double J[3][3];           /* J[i][k] = d x_i / d xi_k */
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            J[i][k] = X[k + 1][i] - X[0][i];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0))
        return det;
    double inv[3][3];         /* inv[k][i] = d xi_k / d x_i */
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int i = 0; i < 3; ++i) {
        g[1][i] = inv[0][i];
        g[2][i] = inv[1][i];
        g[3][i] = inv[2][i];
        g[0][i] = -(inv[0][i] + inv[1][i] + inv[2][i]);
    }
    return det;
}

static void element_one(const double X[4][3], const double U[4][4], const double Uprev[4][4],
                        const double Uadv[4][4], const double F[4][3], const double beta[3],
                        const double beta_adv[3], double nu, double inv_dt, double bscale, int picard,
                        int nq, const double* lam, const double* wq, double det, const double g[4][3],
                        double R[NDOF], double* K)
{
    memset(R, 0, sizeof(double) * NDOF);
    if (K) memset(K, 0, sizeof(double) * NDOF * NDOF);

    /* coarse velocity gradient (constant on the tet) */
    double Gbar[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Gbar[i][j] = 0.0;
            for (int a = 0; a < 4; ++a) Gbar[i][j] += U[a][i] * g[a][j];
        }

    for (int q = 0; q < nq; ++q) {
        const double* L = lam + 4 * q;
        const double dV = wq[q] * det;
        /* bubble and its gradient */
        double bub = bscale * 256.0 * L[0] * L[1] * L[2] * L[3];
        double db[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 4; ++a) {
            double prod = bscale * 256.0;
            for (int c = 0; c < 4; ++c) if (c != a) prod *= L[c];
            for (int i = 0; i < 3; ++i) db[i] += prod * g[a][i];
        }
        /* fields at the point */
        double vbar[3] = {0, 0, 0}, vprev[3] = {0, 0, 0}, f[3] = {0, 0, 0}, p = 0.0, vadv[3] = {0, 0, 0};
        for (int a = 0; a < 4; ++a) {
            for (int i = 0; i < 3; ++i) {
                vbar[i] += L[a] * U[a][i];
                vprev[i] += L[a] * Uprev[a][i];
                f[i] += L[a] * F[a][i];
                vadv[i] += L[a] * Uadv[a][i];
            }
            p += L[a] * U[a][3];
        }
        double v[3], va[3], G[3][3];
        for (int i = 0; i < 3; ++i) {
            v[i] = vbar[i] + bub * beta[i];
            va[i] = vadv[i] + bub * beta_adv[i];      /* advecting velocity */
            for (int j = 0; j < 3; ++j) G[i][j] = Gbar[i][j] + beta[i] * db[j];
        }
        double conv[3];
        for (int i = 0; i < 3; ++i)
            conv[i] = G[i][0] * va[0] + G[i][1] * va[1] + G[i][2] * va[2];
        double divv = G[0][0] + G[1][1] + G[2][2];

        /* test functions: momentum rows carry (value tw, gradient tg), continuity rows tq */
        double tw[NDOF][3], tg[NDOF][3][3], tq[NDOF];
        int mom[NDOF];
        memset(tw, 0, sizeof tw);
        memset(tg, 0, sizeof tg);
        memset(tq, 0, sizeof tq);
        for (int a = 0; a < 4; ++a) {
            for (int i = 0; i < 3; ++i) {
                int r = 4 * a + i;
                mom[r] = 1;
                tw[r][i] = L[a];
                for (int j = 0; j < 3; ++j) tg[r][i][j] = g[a][j];
            }
            mom[4 * a + 3] = 0;
            tq[4 * a + 3] = L[a];
        }
        for (int i = 0; i < 3; ++i) {
            int r = 16 + i;
            mom[r] = 1;
            tw[r][i] = bub;
            for (int j = 0; j < 3; ++j) tg[r][i][j] = db[j];
        }

        /* residual */
        double m[3];
        for (int i = 0; i < 3; ++i) m[i] = conv[i] + (vbar[i] - vprev[i]) * inv_dt - f[i];
        for (int r = 0; r < NDOF; ++r) {
            double val;
            if (mom[r]) {
                double visc = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) visc += tg[r][i][j] * G[i][j];
                double divw = tg[r][0][0] + tg[r][1][1] + tg[r][2][2];
                val = tw[r][0] * m[0] + tw[r][1] * m[1] + tw[r][2] * m[2]
                    + 2.0 * nu * visc - divw * p;
            } else {
                val = -tq[r] * divv;
            }
            R[r] += dV * val;
        }
        if (!K) continue;

        /* trial directions: full velocity dv, its coarse part dvb, gradient dG, pressure dp */
        double dv[NDOF][3], dvb[NDOF][3], dG[NDOF][3][3], dp[NDOF];
        memset(dv, 0, sizeof dv);
        memset(dvb, 0, sizeof dvb);
        memset(dG, 0, sizeof dG);
        memset(dp, 0, sizeof dp);
        for (int a = 0; a < 4; ++a) {
            for (int i = 0; i < 3; ++i) {
                int c = 4 * a + i;
                dv[c][i] = L[a];
                dvb[c][i] = L[a];
                for (int j = 0; j < 3; ++j) dG[c][i][j] = g[a][j];
            }
            dp[4 * a + 3] = L[a];
        }
        for (int i = 0; i < 3; ++i) {
            int c = 16 + i;
            dv[c][i] = bub;
            for (int j = 0; j < 3; ++j) dG[c][i][j] = db[j];
        }
        for (int c = 0; c < NDOF; ++c) {
            double dm[3];
            for (int i = 0; i < 3; ++i) {
                /* (v.grad) dv: the advected field; (dv.grad) v: the advecting one (Newton only) */
                dm[i] = dG[c][i][0] * va[0] + dG[c][i][1] * va[1] + dG[c][i][2] * va[2] + dvb[c][i] * inv_dt;
                if (!picard) dm[i] += G[i][0] * dv[c][0] + G[i][1] * dv[c][1] + G[i][2] * dv[c][2];
            }
            double ddiv = dG[c][0][0] + dG[c][1][1] + dG[c][2][2];
            for (int r = 0; r < NDOF; ++r) {
                double val;
                if (mom[r]) {
                    double visc = 0.0;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) visc += tg[r][i][j] * dG[c][i][j];
                    double divw = tg[r][0][0] + tg[r][1][1] + tg[r][2][2];
                    val = tw[r][0] * dm[0] + tw[r][1] * dm[1] + tw[r][2] * dm[2]
                        + 2.0 * nu * visc - divw * dp[c];
                } else {
                    val = -tq[r] * ddiv;
                }
                K[r * NDOF + c] += dV * val;
            }
        }
    }
}

int oracle_element(int64_t n_elems, const int32_t* tets, const double* xyz, const double* u,
                   const double* u_prev, const double* beta, const double* body, double nu,
                   double inv_dt, double bscale, int picard, const double* u_adv, const double* beta_adv,
                   int nq, const double* lam, const double* wq, double* R, double* K)
{
    int64_t first_bad = -1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_elems; ++e) {
        double X[4][3], U[4][4], Up[4][4], Ua[4][4], F[4][3], g[4][3];
        for (int a = 0; a < 4; ++a) {
            int64_t n = tets[4 * e + a];
            for (int i = 0; i < 3; ++i) {
                X[a][i] = xyz[3 * n + i];
                F[a][i] = body ? body[3 * n + i] : 0.0;
            }
            for (int i = 0; i < 4; ++i) {
                U[a][i] = u[4 * n + i];
                Up[a][i] = u_prev ? u_prev[4 * n + i] : 0.0;
                Ua[a][i] = u_adv ? u_adv[4 * n + i] : U[a][i];
            }
        }
        double det = tet_geometry(X, g);
        if (!(det > 0.0)) {
#pragma omp critical
            if (first_bad < 0 || e < first_bad) first_bad = e;
            continue;
        }
        element_one(X, U, Up, Ua, F, beta + 3 * e, beta_adv ? beta_adv + 3 * e : beta + 3 * e, nu,
                    u_prev ? inv_dt : 0.0, bscale, picard, nq, lam, wq, det, g, R + NDOF * e,
                    K ? K + (int64_t)NDOF * NDOF * e : NULL);
    }
    return first_bad < 0 ? 0 : (int)(1 + first_bad);
}
