"""ORACLE (test infrastructure): restarted GMRES with deflated restarting, plain FP64, CPU.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may import this module.
It shares no code with the GPU library.

Deflated restarting is not part of the paper's method: the paper solves the condensed system
with restarted GMRES (Section 6), and the library offers deflated restarting as an option of
that solver.  The reference here is GMRES-DR as R. B. Morgan defines it (SIAM J. Sci. Comput.
24 (2002) 20-37): after a cycle with Arnoldi relation (A M) V_m = V_{m+1} Hbar, keep the
harmonic Ritz vectors of the k harmonic Ritz values of smallest modulus, i.e. eigenvectors g of
H_m + h^2 f e_m^T with f = H_m^{-T} e_m and h = Hbar(m, m-1); together with the cycle's
least-squares residual coefficients they span a space P on which (A M) V_{m+1} P_k =
V_{m+1} P Hk with Hk = P^T Hbar P_k.  The next cycle starts from that block and extends it by
Arnoldi steps.

Like the library, every cycle restarts from the true residual r = b - A x: the part of r
outside the kept vectors (two Gram-Schmidt passes) is the next basis vector, and r's
coefficients in the kept basis form the cycle's least-squares right-hand side.  A cycle that
stopped on its residual estimate, or ran fewer than `restart` steps, is followed by a plain
restart.  The dense algebra is numpy's: eig for the harmonic Ritz problem, QR for the kept
basis, lstsq for the cycle's least-squares problem after every step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class GmresDrResult:
    x: np.ndarray
    iters: int               # Arnoldi steps (products with A M), over all cycles
    restarts: int            # cycles
    true_rel_res: float
    converged: bool
    theta: np.ndarray        # harmonic Ritz values kept at the last deflated restart (empty if none)


def harmonic_ritz(H, m, k):
    """The harmonic Ritz pairs of a cycle's (m+1) x m matrix Hbar for the k values of smallest
    modulus (Morgan 2002): eigenpairs of H_m + h^2 H_m^{-T} e_m e_m^T.  A complex pair is kept
    whole (its real and imaginary parts), so k + 1 vectors may come back.  Returns (theta, Y),
    Y real [m, kk]."""
    Hm = H[:m, :m]
    h = H[m, m - 1]
    em = np.zeros(m)
    em[-1] = 1.0
    f = np.linalg.solve(Hm.T, em)
    G = Hm + h * h * np.outer(f, em)
    th, Z = np.linalg.eig(G)
    # by modulus; of a conjugate pair the member with positive imaginary part first
    order = sorted(range(m), key=lambda i: (abs(th[i]), -th[i].imag))
    cols, vals = [], []
    for i in order:
        if len(cols) >= k:
            break
        if th[i].imag < 0:
            continue
        if th[i].imag > 0:
            cols += [Z[:, i].real, Z[:, i].imag]
            vals += [th[i], np.conj(th[i])]
        else:
            cols.append(Z[:, i].real)
            vals.append(th[i].real)
    return np.array(vals), np.array(cols).T


def gmres_dr(A, b, restart=50, k=10, max_iters=10000, rtol=1e-12, Minv_blocks=None):
    """GMRES-DR(restart, k), right preconditioned by the block-diagonal M (blocks [n/4, 4, 4],
    or the identity): solves A M y = b, x = M y.  Success iff ||b - A x|| <= rtol ||b||,
    recomputed at every restart.  k = 0 is plain restarted GMRES."""
    n = b.size
    m = restart
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return GmresDrResult(x, 0, 0, 0.0, True, np.zeros(0))

    def M(v):
        if Minv_blocks is None:
            return v
        return np.einsum("nij,nj->ni", Minv_blocks, v.reshape(-1, 4)).ravel()

    iters = restarts = 0
    kept = None                      # (W [n, kk] orthonormal, Hk [kk+1, kk]) for the next cycle
    theta = np.zeros(0)
    tol = rtol * bn
    while True:
        r = b - A @ x
        rn = np.linalg.norm(r)
        if rn <= tol:
            return GmresDrResult(x, iters, restarts, rn / bn, True, theta)
        if iters >= max_iters:
            return GmresDrResult(x, iters, restarts, rn / bn, False, theta)
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        c = np.zeros(m + 1)
        u = r / rn
        if kept is not None:
            W, Hk = kept
            kk = W.shape[1]
            V[:, :kk] = W
            H[:kk + 1, :kk] = Hk
            s = W.T @ u
            u = u - W @ s
            s2 = W.T @ u
            u = u - W @ s2
            s = s + s2
            rho = np.linalg.norm(u)
            V[:, kk] = u / rho
            c[:kk] = rn * s
            c[kk] = rn * rho
        else:
            kk = 0
            V[:, 0] = u
            c[0] = rn
        stopped = False
        jend = kk
        if kk > 0:
            # the kept block alone may already meet the tolerance
            y = np.linalg.lstsq(H[:kk + 1, :kk], c[:kk + 1], rcond=None)[0]
            stopped = np.linalg.norm(c[:kk + 1] - H[:kk + 1, :kk] @ y) <= tol
        for j in range(kk, kk + min(m - kk, max_iters - iters) if not stopped else kk):
            w = A @ M(V[:, j])
            for _ in range(2):       # classical Gram-Schmidt, two passes
                hv = V[:, :j + 1].T @ w
                w = w - V[:, :j + 1] @ hv
                H[:j + 1, j] += hv
            H[j + 1, j] = np.linalg.norm(w)
            iters += 1
            jend = j + 1
            if H[j + 1, j] > 0:
                V[:, j + 1] = w / H[j + 1, j]
            y = np.linalg.lstsq(H[:j + 2, :j + 1], c[:j + 2], rcond=None)[0]
            est = np.linalg.norm(c[:j + 2] - H[:j + 2, :j + 1] @ y)
            if est <= tol or H[j + 1, j] == 0.0:
                stopped = True
                break
        y = np.linalg.lstsq(H[:jend + 1, :jend], c[:jend + 1], rcond=None)[0]
        x = x + M(V[:, :jend] @ y)
        restarts += 1
        kept = None
        if k > 0 and not stopped and jend == m:
            theta, Y = harmonic_ritz(H, m, k)
            nk = Y.shape[1]
            rc = c - H @ y
            Pm = np.zeros((m + 1, nk + 1))
            Pm[:m, :nk] = Y
            Pm[:, nk] = rc
            P, _ = np.linalg.qr(Pm)
            if P[:, nk] @ rc < 0:
                P[:, nk] = -P[:, nk]         # the last basis vector points along the residual
            kept = (V @ P[:, :nk], P.T @ H @ P[:m, :nk])
