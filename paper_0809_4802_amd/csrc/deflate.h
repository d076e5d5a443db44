// Deflated restarting of GMRES(m): host-side dense algebra between two cycles (deflate.cpp).
#pragma once

#include <vector>

namespace vms {

struct DrSetup {
    int kk = 0;                 // kept harmonic Ritz vectors (k, or k + 1 to keep a complex pair whole)
    std::vector<double> P;      // (m+1) x (kk+1), column-major: the new basis is V_{m+1} P, its last
                                // vector the direction of the cycle's residual
    std::vector<double> Hk;     // (kk+1) x kk, column-major: B V_kk = V_{kk+1} Hk
    std::vector<double> Qt;     // (kk+1) x (kk+1), column-major: Q^T of Hk = Q [R; 0]
    std::vector<double> R;      // kk x kk, column-major, upper triangular
};

// Hbar: the cycle's (m+1) x m Hessenberg matrix, column-major with leading dimension ldh;
// rc: the (m+1) least-squares residual coefficients c - Hbar y.  Keeps the harmonic Ritz
// vectors of the k harmonic Ritz values of smallest modulus.  Returns kk (0: nothing kept --
// a singular H_m, an eigenvalue iteration that did not converge, or a residual inside the
// kept space).
int dr_setup(int m, int k, const double* Hbar, int ldh, const double* rc, DrSetup* out);

}  // namespace vms
