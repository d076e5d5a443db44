// Deflated restarting for GMRES(m) (GMRES-DR, Morgan, SIAM J. Sci. Comput. 24 (2002)): the
// small dense algebra done on the host between two cycles.  Plain C++ (no HIP), so that it
// can be built and tested on its own.
//
// After a cycle with Arnoldi relation  B V_m = V_{m+1} Hbar  (Hbar (m+1) x m, upper Hessenberg
// but for the full leading block a deflated cycle starts with; B the preconditioned operator) and least-squares residual coefficients rc = c - Hbar y, the
// next cycle keeps the harmonic Ritz vectors of the k harmonic Ritz values of smallest modulus:
// eigenvectors g of  G = H_m + h^2 f e_m^T,  f = H_m^{-T} e_m,  h = Hbar(m, m-1).  With
// P = orth([g_1 .. g_k; 0], rc) ((m+1) x (k+1)), the new basis V_{k+1} = V_{m+1} P satisfies
// B V_k = V_{k+1} Hk,  Hk = P^T Hbar P(0:m, 0:k), and its last vector is the direction of the
// cycle's residual.  The Givens chain of the next cycle starts from the QR factors of Hk.
#include "deflate.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

// The routines below run between two GMRES cycles, with the GPU waiting: each is compiled
// twice, for CPUs with FMA (chosen at load time where the CPU has it; about 1.5x faster at
// m = 50) and for baseline x86-64.
#define VMS_HOST_CLONES __attribute__((target_clones("fma", "default")))

namespace vms {
namespace {

using cd = std::complex<double>;

// Complex product, quotient (Smith's method: R. L. Smith, Comm. ACM 5 (1962)) and squared
// modulus written out, without the special-value handling of the library's operators.
inline cd cmul(cd a, cd b) {
    return cd(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}
inline cd cdiv(cd a, cd b) {
    if (std::fabs(b.real()) >= std::fabs(b.imag())) {
        const double r = b.imag() / b.real(), d = b.real() + b.imag() * r;
        return cd((a.real() + a.imag() * r) / d, (a.imag() - a.real() * r) / d);
    }
    const double r = b.real() / b.imag(), d = b.imag() + b.real() * r;
    return cd((a.real() * r + a.imag()) / d, (a.imag() * r - a.real()) / d);
}
inline double mag2(cd a) { return a.real() * a.real() + a.imag() * a.imag(); }

// Solve A^T x = e_last for an m x m matrix A (column-major, leading dimension lda) by Gaussian
// elimination with partial pivoting: O(m^2) when A is upper Hessenberg (every cycle leaves H_m
// in that form), the dense elimination otherwise.  Returns false if A is singular.
VMS_HOST_CLONES bool solve_transposed_last(int m, const double* A, int lda, std::vector<double>& x) {
    bool hess = true;
    for (int c = 0; c < m && hess; ++c)
        for (int r = c + 2; r < m; ++r)
            if (A[(size_t)c * lda + r] != 0.0) {
                hess = false;
                break;
            }
    x.assign(m, 0.0);
    x[m - 1] = 1.0;
    if (hess) {
        // A = P L U by elimination with partial pivoting, which for an upper Hessenberg matrix
        // only ever exchanges rows c and c+1 and leaves one multiplier per column (L unit lower
        // bidiagonal).  Then A^T x = U^T L^T P^T x = e_last: U^T z = e_last forward, L^T w = z
        // backward with the exchanges undone in reverse order.
        std::vector<double> U((size_t)m * m);       // row-major copy of A
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) U[(size_t)r * m + c] = c + 1 >= r ? A[(size_t)c * lda + r] : 0.0;
        std::vector<double> mult(m, 0.0);
        std::vector<char> swapped(m, 0);
        for (int c = 0; c + 1 < m; ++c) {
            double* a = &U[(size_t)c * m];
            double* b = &U[(size_t)(c + 1) * m];
            if (std::fabs(b[c]) > std::fabs(a[c])) {
                for (int j = c; j < m; ++j) std::swap(a[j], b[j]);
                swapped[c] = 1;
            }
            if (!(std::fabs(a[c]) > 0.0)) return false;
            const double f = b[c] / a[c];
            mult[c] = f;
            b[c] = 0.0;
            if (f != 0.0)
                for (int j = c + 1; j < m; ++j) b[j] -= f * a[j];
        }
        if (!(std::fabs(U[(size_t)(m - 1) * m + m - 1]) > 0.0)) return false;
        // U^T z = e_last: z_c = (e_last[c] - sum_{r<c} U(r, c) z_r) / U(c, c)
        for (int c = 0; c < m; ++c) {
            double s = x[c];
            for (int r = 0; r < c; ++r) s -= U[(size_t)r * m + c] * x[r];
            x[c] = s / U[(size_t)c * m + c];
        }
        // L^T w = z (L has the multiplier of step c at row c+1, column c), then x = P w
        for (int c = m - 2; c >= 0; --c) {
            x[c] -= mult[c] * x[c + 1];
            if (swapped[c]) std::swap(x[c], x[c + 1]);
        }
        return true;
    }
    std::vector<double> M((size_t)m * m);           // M = A^T, row-major
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) M[(size_t)r * m + c] = A[(size_t)r * lda + c];
    for (int col = 0; col < m; ++col) {
        int piv = col;
        double best = std::fabs(M[(size_t)col * m + col]);
        for (int r = col + 1; r < m; ++r)
            if (std::fabs(M[(size_t)r * m + col]) > best) best = std::fabs(M[(size_t)r * m + col]), piv = r;
        if (!(best > 0.0)) return false;
        if (piv != col) {
            for (int c = 0; c < m; ++c) std::swap(M[(size_t)col * m + c], M[(size_t)piv * m + c]);
            std::swap(x[col], x[piv]);
        }
        for (int r = col + 1; r < m; ++r) {
            const double f = M[(size_t)r * m + col] / M[(size_t)col * m + col];
            if (f == 0.0) continue;
            for (int c = col; c < m; ++c) M[(size_t)r * m + c] -= f * M[(size_t)col * m + c];
            x[r] -= f * x[col];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        double s = x[r];
        for (int c = r + 1; c < m; ++c) s -= M[(size_t)r * m + c] * x[c];
        x[r] = s / M[(size_t)r * m + r];
    }
    return true;
}

// Reduction of a square matrix (n x n, row-major, in place) to upper Hessenberg form
// Z^T A Z by Householder reflections (Golub & Van Loan, Matrix Computations, Alg. 7.4.2); Z
// (row-major) is accumulated.  A column already zero below its subdiagonal is skipped, so a
// matrix that is Hessenberg except for a leading block costs reflections of that block only.
// Returns false when A was Hessenberg already (Z is then the identity and not formed).
VMS_HOST_CLONES bool reduce_to_hessenberg(int n, std::vector<double>& a, std::vector<double>& Z) {
    auto A = [&](int r, int c) -> double& { return a[(size_t)r * n + c]; };
    bool used = false;
    std::vector<double> v(n);
    for (int c = 0; c + 2 < n; ++c) {
        double below = 0.0;
        for (int r = c + 2; r < n; ++r) below += A(r, c) * A(r, c);
        if (below == 0.0) continue;
        if (!used) {
            Z.assign((size_t)n * n, 0.0);
            for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
            used = true;
        }
        const double x0 = A(c + 1, c);
        const double nrm = std::sqrt(x0 * x0 + below);
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        std::fill(v.begin(), v.end(), 0.0);
        v[c + 1] = x0 - alpha;
        for (int r = c + 2; r < n; ++r) v[r] = A(r, c);
        double vn = 0.0;
        for (int r = c + 1; r < n; ++r) vn += v[r] * v[r];
        const double f = 2.0 / vn;
        for (int cc = c; cc < n; ++cc) {                     // A <- (I - f v v^T) A
            double d = 0.0;
            for (int r = c + 1; r < n; ++r) d += v[r] * A(r, cc);
            d *= f;
            for (int r = c + 1; r < n; ++r) A(r, cc) -= d * v[r];
        }
        for (int r = 0; r < n; ++r) {                        // A <- A (I - f v v^T), Z likewise
            double d = 0.0, e = 0.0;
            for (int k = c + 1; k < n; ++k) {
                d += A(r, k) * v[k];
                e += Z[(size_t)r * n + k] * v[k];
            }
            d *= f;
            e *= f;
            for (int k = c + 1; k < n; ++k) {
                A(r, k) -= d * v[k];
                Z[(size_t)r * n + k] -= e * v[k];
            }
        }
        for (int r = c + 2; r < n; ++r) A(r, c) = 0.0;
    }
    return used;
}

// Eigenvalues of an upper Hessenberg matrix (n x n, row-major, destroyed) by the Francis
// double-shift QR iteration with deflation on negligible subdiagonal entries and exceptional
// shifts after 10 and 20 iterations without deflation (Golub & Van Loan, Matrix Computations,
// Sec. 7.5).  Returns false if an eigenvalue has not converged in 30 n iterations.
VMS_HOST_CLONES bool hessenberg_eigenvalues(int n, std::vector<double>& a, std::vector<cd>& ev) {
    auto A = [&](int r, int c) -> double& { return a[(size_t)r * n + c]; };
    ev.clear();
    double anorm = 0.0;
    for (int r = 0; r < n; ++r)
        for (int c = std::max(r - 1, 0); c < n; ++c) anorm += std::fabs(A(r, c));
    const double eps = 2.220446049250313e-16;
    int hi = n - 1;
    int its = 0, total = 0;
    double exshift = 0.0;
    while (hi >= 0) {
        // the active block ends at hi; find its start lo (a negligible subdiagonal above it)
        int lo = hi;
        while (lo > 0) {
            double s = std::fabs(A(lo - 1, lo - 1)) + std::fabs(A(lo, lo));
            if (s == 0.0) s = anorm;
            if (std::fabs(A(lo, lo - 1)) <= eps * s) {
                A(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {                                  // 1 x 1 block
            ev.emplace_back(A(hi, hi) + exshift, 0.0);
            --hi;
            its = 0;
            continue;
        }
        if (lo == hi - 1) {                              // 2 x 2 block
            const double p = A(hi - 1, hi - 1), q = A(hi - 1, hi), r = A(hi, hi - 1), s = A(hi, hi);
            const double tr = 0.5 * (p + s), det = p * s - q * r;
            const double disc = tr * tr - det;
            if (disc >= 0.0) {
                const double sq = std::sqrt(disc);
                const double l1 = tr + (tr >= 0.0 ? sq : -sq);
                const double l2 = l1 != 0.0 ? det / l1 : tr - (tr >= 0.0 ? sq : -sq);
                ev.emplace_back(l1 + exshift, 0.0);
                ev.emplace_back(l2 + exshift, 0.0);
            } else {
                const double im = std::sqrt(-disc);
                ev.emplace_back(tr + exshift, im);
                ev.emplace_back(tr + exshift, -im);
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (++total > 30 * n) return false;
        // shifts: the eigenvalues of the trailing 2 x 2 block (as their sum and product), or
        // exceptional ones
        double sum, prod;
        if (its == 10 || its == 20) {
            // the whole unreduced part (rows 0 .. hi) is shifted, so that every eigenvalue
            // found later takes exshift back
            const double t = std::fabs(A(hi, hi - 1)) + std::fabs(A(hi - 1, hi - 2));
            const double d = A(hi, hi);
            exshift += d;
            for (int i = 0; i <= hi; ++i) A(i, i) -= d;      // blocks above lo included
            sum = 1.5 * t;
            prod = t * t;
        } else {
            sum = A(hi - 1, hi - 1) + A(hi, hi);
            prod = A(hi - 1, hi - 1) * A(hi, hi) - A(hi - 1, hi) * A(hi, hi - 1);
        }
        ++its;
        // first column of (H - s1 I)(H - s2 I) restricted to the block
        double x = A(lo, lo) * A(lo, lo) + A(lo, lo + 1) * A(lo + 1, lo) - sum * A(lo, lo) + prod;
        double y = A(lo + 1, lo) * (A(lo, lo) + A(lo + 1, lo + 1) - sum);
        double z = A(lo + 1, lo) * A(lo + 2, lo + 1);
        // chase the bulge with 3 x 3 Householder reflectors, then a final 2 x 2 one
        for (int k = lo; k <= hi - 2; ++k) {
            const double nrm = std::sqrt(x * x + y * y + z * z);
            if (nrm > 0.0) {
                // reflector I - tau u u^T with u = (1, u1, u2): v = (x - alpha, y, z) scaled by
                // its first entry, and tau = 2 v0^2 / v^T v = -v0 / alpha, as v^T v = -2 alpha v0
                const double alpha = x >= 0.0 ? -nrm : nrm;
                const double v0 = x - alpha;
                const double iv = 1.0 / v0;
                const double u1 = y * iv, u2 = z * iv, tau = -v0 / alpha;
                // eigenvalues only: the transformations are applied inside the active block
                const int c0 = std::max(lo, k - 1);
                const int r1 = std::min(k + 3, hi);
                for (int c = c0; c <= hi; ++c) {                 // rows k..k+2 from the left
                    const double d = tau * (A(k, c) + u1 * A(k + 1, c) + u2 * A(k + 2, c));
                    A(k, c) -= d;
                    A(k + 1, c) -= d * u1;
                    A(k + 2, c) -= d * u2;
                }
                // columns k..k+2 from the right, bottom row first: rows k+1..k+3 of column k
                // hold the next reflector's vector, which can then be formed while the other
                // rows are still being updated
                for (int r = r1; r >= lo; --r) {
                    const double d = tau * (A(r, k) + A(r, k + 1) * u1 + A(r, k + 2) * u2);
                    A(r, k) -= d;
                    A(r, k + 1) -= d * u1;
                    A(r, k + 2) -= d * u2;
                }
            }
            x = A(k + 1, k);
            y = A(k + 2, k);
            if (k < hi - 2) z = A(k + 3, k);
        }
        {
            const int k = hi - 1;
            const double nrm = std::sqrt(x * x + y * y);
            if (nrm > 0.0) {
                const double alpha = x >= 0.0 ? -nrm : nrm;
                const double v0 = x - alpha;
                const double u1 = y / v0, tau = -v0 / alpha;
                for (int c = std::max(lo, k - 1); c <= hi; ++c) {
                    const double d = tau * (A(k, c) + u1 * A(k + 1, c));
                    A(k, c) -= d;
                    A(k + 1, c) -= d * u1;
                }
                for (int r = lo; r <= hi; ++r) {
                    const double d = tau * (A(r, k) + A(r, k + 1) * u1);
                    A(r, k) -= d;
                    A(r, k + 1) -= d * u1;
                }
            }
        }
        // the reflectors leave rounding below the subdiagonal; it is not part of the iteration.
        // A bulge reaches at most three rows below the diagonal, and the input is Hessenberg,
        // so the entries further down are exact zeros already
        for (int r = lo + 2; r <= hi; ++r) {
            A(r, r - 2) = 0.0;
            if (r - 3 >= lo) A(r, r - 3) = 0.0;
        }
    }
    return true;
}

// An eigenvector of the upper Hessenberg G (n x n, row-major) for the eigenvalue theta by
// inverse iteration: one solve with (G - theta I) from the vector of ones (theta comes from the
// QR iteration to rounding accuracy, so one step leaves an error of the order of rounding over
// the gap to the next eigenvalue).  Its LU with partial pivoting keeps the
// Hessenberg structure (each column has one entry below the diagonal, and the pivot is one of
// two rows), so a factorisation costs O(n^2).
VMS_HOST_CLONES void inverse_iteration(int n, const std::vector<double>& G, cd theta, std::vector<cd>& x) {
    std::vector<cd> M((size_t)n * n);
    double gnorm = 0.0;
    for (int r = 0; r < n; ++r)
        for (int c = std::max(r - 1, 0); c < n; ++c) {
            M[(size_t)r * n + c] = G[(size_t)r * n + c];
            gnorm = std::max(gnorm, std::fabs(G[(size_t)r * n + c]));
        }
    for (int i = 0; i < n; ++i) M[(size_t)i * n + i] -= theta;
    const double tiny = 1e-14 * std::max(gnorm, 1e-300);
    std::vector<char> swapped(n, 0);
    std::vector<cd> mult(n, cd(0.0));
    for (int col = 0; col + 1 < n; ++col) {
        cd* a = &M[(size_t)col * n];
        cd* b = &M[(size_t)(col + 1) * n];
        if (mag2(b[col]) > mag2(a[col])) {
            for (int c = col; c < n; ++c) std::swap(a[c], b[c]);
            swapped[col] = 1;
        }
        if (mag2(a[col]) < tiny * tiny) a[col] = tiny;               // theta is an exact eigenvalue
        const cd f = cdiv(b[col], a[col]);
        mult[col] = f;
        b[col] = 0.0;
        if (f != cd(0.0))
            for (int c = col + 1; c < n; ++c) b[c] -= cmul(f, a[c]);
    }
    if (mag2(M[(size_t)(n - 1) * n + n - 1]) < tiny * tiny) M[(size_t)(n - 1) * n + n - 1] = tiny;
    x.assign(n, cd(1.0, 0.0));
    for (int pass = 0; pass < 1; ++pass) {
        for (int col = 0; col + 1 < n; ++col) {
            if (swapped[col]) std::swap(x[col], x[col + 1]);
            x[col + 1] -= cmul(mult[col], x[col]);
        }
        for (int r = n - 1; r >= 0; --r) {
            cd s = x[r];
            const cd* row = &M[(size_t)r * n];
            for (int c = r + 1; c < n; ++c) s -= cmul(row[c], x[c]);
            x[r] = cdiv(s, row[r]);
        }
        double nrm = 0.0;
        for (const cd& v : x) nrm += mag2(v);
        nrm = std::sqrt(nrm);
        for (cd& v : x) v = cd(v.real() / nrm, v.imag() / nrm);
    }
}

// Orthonormalises column `col` of P ((rows) x (cols), column-major, ld = rows) against columns
// 0 .. col-1 (modified Gram-Schmidt, two passes).  Returns its norm before normalisation
// relative to its initial norm (0 if it vanished).
double orthonormalize_column(int rows, std::vector<double>& P, int col) {
    double* v = &P[(size_t)col * rows];
    double n0 = 0.0;
    for (int i = 0; i < rows; ++i) n0 += v[i] * v[i];
    n0 = std::sqrt(n0);
    if (!(n0 > 0.0)) return 0.0;
    for (int pass = 0; pass < 2; ++pass)
        for (int c = 0; c < col; ++c) {
            const double* q = &P[(size_t)c * rows];
            double d = 0.0;
            for (int i = 0; i < rows; ++i) d += q[i] * v[i];
            for (int i = 0; i < rows; ++i) v[i] -= d * q[i];
        }
    double n1 = 0.0;
    for (int i = 0; i < rows; ++i) n1 += v[i] * v[i];
    n1 = std::sqrt(n1);
    if (!(n1 > 1e-10 * n0)) return 0.0;
    for (int i = 0; i < rows; ++i) v[i] /= n1;
    return n1 / n0;
}

}  // namespace

VMS_HOST_CLONES int dr_setup(int m, int k, const double* Hbar, int ldh, const double* rc, DrSetup* out) {
    out->kk = 0;
    if (m < 2 || k < 1 || k >= m) return 0;
    // G = H_m + h^2 f e_m^T (row-major), f = H_m^{-T} e_m
    std::vector<double> f;
    if (!solve_transposed_last(m, Hbar, ldh, f)) return 0;
    const double h = Hbar[(size_t)(m - 1) * ldh + m];
    std::vector<double> G((size_t)m * m);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) G[(size_t)r * m + c] = Hbar[(size_t)c * ldh + r];
    for (int r = 0; r < m; ++r) G[(size_t)r * m + (m - 1)] += h * h * f[r];
    // after a deflated cycle H_m has a full leading block: back to Hessenberg form first
    std::vector<double> Z;
    const bool reduced = reduce_to_hessenberg(m, G, Z);
    std::vector<double> work = G;
    std::vector<cd> ev;
    if (!hessenberg_eigenvalues(m, work, ev)) return 0;
    std::sort(ev.begin(), ev.end(), [](const cd& a, const cd& b) {
        const double aa = std::abs(a), bb = std::abs(b);
        if (aa != bb) return aa < bb;
        return a.imag() > b.imag();
    });
    // the k smallest, a complex pair counted whole (its real and imaginary parts)
    const int rows = m + 1;
    std::vector<double> P;
    P.reserve((size_t)(k + 2) * rows);
    std::vector<cd> x;
    int taken = 0;
    for (size_t i = 0; i < ev.size() && taken < k; ++i) {
        const cd t = ev[i];
        if (t.imag() < 0.0) continue;                    // the pair is taken at its upper member
        inverse_iteration(m, G, t, x);
        if (reduced) {                                   // an eigenvector of G is Z x
            std::vector<cd> zx(m, cd(0.0));
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) zx[r] += Z[(size_t)r * m + c] * x[c];
            x.swap(zx);
        }
        const int parts = t.imag() > 0.0 ? 2 : 1;
        for (int p = 0; p < parts; ++p) {
            const int col = (int)(P.size() / rows);
            P.resize(P.size() + rows, 0.0);
            for (int r = 0; r < m; ++r) P[(size_t)col * rows + r] = p == 0 ? x[r].real() : x[r].imag();
            if (orthonormalize_column(rows, P, col) == 0.0) P.resize(P.size() - rows);   // dependent: dropped
            else ++taken;
        }
    }
    const int kk = (int)(P.size() / rows);
    if (kk < 1 || kk + 1 > m) return 0;
    // the residual direction last
    P.resize(P.size() + rows);
    for (int r = 0; r < rows; ++r) P[(size_t)kk * rows + r] = rc[r];
    if (orthonormalize_column(rows, P, kk) == 0.0) return 0;
    // Hk = P^T Hbar P(0:m, 0:kk)  ((kk+1) x kk, column-major)
    std::vector<double> HP((size_t)rows * kk, 0.0);               // Hbar P(0:m, 0:kk)
    for (int c = 0; c < kk; ++c)
        for (int l = 0; l < m; ++l) {
            const double p = P[(size_t)c * rows + l];
            if (p == 0.0) continue;
            const double* hl = &Hbar[(size_t)l * ldh];
            for (int r = 0; r < rows; ++r) HP[(size_t)c * rows + r] += hl[r] * p;
        }
    std::vector<double> Hk((size_t)(kk + 1) * kk, 0.0);
    for (int c = 0; c < kk; ++c)
        for (int r = 0; r <= kk; ++r) {
            double s = 0.0;
            for (int l = 0; l < rows; ++l) s += P[(size_t)r * rows + l] * HP[(size_t)c * rows + l];
            Hk[(size_t)c * (kk + 1) + r] = s;
        }
    // A Hessenberg basis of the kept space: with U orthogonal (kk x kk), P_k U spans the same
    // space and diag(U^T, 1) Hk U is its matrix.  U is chosen so that this matrix is upper
    // Hessenberg (the kept space is a Krylov space), which keeps the next cycle's Hbar, and so
    // its harmonic Ritz problem, in Hessenberg form.  Writing Hk = [T; h^T]: reduce T^T to
    // Hessenberg form W^T T^T W with W e_1 along h (a reflection onto h, then the Householder
    // reduction, which fixes e_1); U is W with its columns reversed.
    {
        const int nr = kk + 1;
        std::vector<double> hv(kk);
        double hn = 0.0;
        for (int c = 0; c < kk; ++c) {
            hv[c] = Hk[(size_t)c * nr + kk];
            hn += hv[c] * hv[c];
        }
        hn = std::sqrt(hn);
        std::vector<double> W((size_t)kk * kk, 0.0);          // row-major
        for (int i = 0; i < kk; ++i) W[(size_t)i * kk + i] = 1.0;
        if (hn > 0.0) {                                       // W0 = I - 2 v v^T / v^T v, W0 e_1 = h / alpha
            std::vector<double> v = hv;
            const double alpha = hv[0] >= 0.0 ? -hn : hn;
            v[0] -= alpha;
            double vn = 0.0;
            for (double e : v) vn += e * e;
            if (vn > 0.0)
                for (int i = 0; i < kk; ++i)
                    for (int j = 0; j < kk; ++j) W[(size_t)i * kk + j] -= 2.0 * v[i] * v[j] / vn;
        }
        // A = W0^T T^T W0 (row-major), T(r, c) = Hk[c * nr + r]
        std::vector<double> TW((size_t)kk * kk, 0.0), A((size_t)kk * kk, 0.0);
        for (int i = 0; i < kk; ++i)                          // TW = T^T W0
            for (int j = 0; j < kk; ++j) {
                double s = 0.0;
                for (int l = 0; l < kk; ++l) s += Hk[(size_t)i * nr + l] * W[(size_t)l * kk + j];
                TW[(size_t)i * kk + j] = s;
            }
        for (int i = 0; i < kk; ++i)
            for (int j = 0; j < kk; ++j) {
                double s = 0.0;
                for (int l = 0; l < kk; ++l) s += W[(size_t)l * kk + i] * TW[(size_t)l * kk + j];
                A[(size_t)i * kk + j] = s;
            }
        std::vector<double> Z;
        if (reduce_to_hessenberg(kk, A, Z)) {                 // W = W0 Z
            std::vector<double> WZ((size_t)kk * kk, 0.0);
            for (int i = 0; i < kk; ++i)
                for (int j = 0; j < kk; ++j) {
                    double s = 0.0;
                    for (int l = 0; l < kk; ++l) s += W[(size_t)i * kk + l] * Z[(size_t)l * kk + j];
                    WZ[(size_t)i * kk + j] = s;
                }
            W.swap(WZ);
        }
        auto U = [&](int i, int c) { return W[(size_t)i * kk + (kk - 1 - c)]; };
        // P_k <- P_k U
        std::vector<double> Pk((size_t)rows * kk, 0.0);
        for (int c = 0; c < kk; ++c)
            for (int l = 0; l < kk; ++l) {
                const double u = U(l, c);
                for (int r = 0; r < rows; ++r) Pk[(size_t)c * rows + r] += P[(size_t)l * rows + r] * u;
            }
        std::copy(Pk.begin(), Pk.end(), P.begin());
        // Hk <- diag(U^T, 1) Hk U, rounding below the subdiagonal cleared
        std::vector<double> HU((size_t)nr * kk, 0.0);
        for (int c = 0; c < kk; ++c)
            for (int l = 0; l < kk; ++l) {
                const double u = U(l, c);
                for (int r = 0; r < nr; ++r) HU[(size_t)c * nr + r] += Hk[(size_t)l * nr + r] * u;
            }
        for (int c = 0; c < kk; ++c)
            for (int r = 0; r < nr; ++r) {
                double s = 0.0;
                if (r == kk) {
                    s = HU[(size_t)c * nr + kk];
                } else {
                    for (int l = 0; l < kk; ++l) s += U(l, r) * HU[(size_t)c * nr + l];
                }
                Hk[(size_t)c * nr + r] = r > c + 1 ? 0.0 : s;
            }
    }
    out->kk = kk;
    out->Hk = Hk;
    out->P.assign(P.begin(), P.end());
    // QR of Hk by Householder reflections: Qt = Q^T ((kk+1) x (kk+1), column-major), R (kk x kk)
    const int nr = kk + 1;
    std::vector<double> R = out->Hk;                               // (kk+1) x kk, column-major
    std::vector<double> Qt((size_t)nr * nr, 0.0);
    for (int i = 0; i < nr; ++i) Qt[(size_t)i * nr + i] = 1.0;
    for (int c = 0; c < kk; ++c) {
        double nrm = 0.0;
        for (int r = c; r < nr; ++r) nrm += R[(size_t)c * nr + r] * R[(size_t)c * nr + r];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) continue;
        const double x0 = R[(size_t)c * nr + c];
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        std::vector<double> v(nr, 0.0);
        v[c] = x0 - alpha;
        for (int r = c + 1; r < nr; ++r) v[r] = R[(size_t)c * nr + r];
        double vn = 0.0;
        for (int r = c; r < nr; ++r) vn += v[r] * v[r];
        if (!(vn > 0.0)) continue;
        for (int cc = c; cc < kk; ++cc) {
            double d = 0.0;
            for (int r = c; r < nr; ++r) d += v[r] * R[(size_t)cc * nr + r];
            d *= 2.0 / vn;
            for (int r = c; r < nr; ++r) R[(size_t)cc * nr + r] -= d * v[r];
        }
        for (int cc = 0; cc < nr; ++cc) {                         // Qt <- (I - 2 v v^T / vn) Qt
            double d = 0.0;
            for (int r = c; r < nr; ++r) d += v[r] * Qt[(size_t)cc * nr + r];
            d *= 2.0 / vn;
            for (int r = c; r < nr; ++r) Qt[(size_t)cc * nr + r] -= d * v[r];
        }
    }
    out->Qt = Qt;
    out->R.assign((size_t)kk * kk, 0.0);
    for (int c = 0; c < kk; ++c)
        for (int r = 0; r <= c; ++r) out->R[(size_t)c * kk + r] = R[(size_t)c * nr + r];
    return kk;
}

}  // namespace vms
