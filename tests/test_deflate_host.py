"""Host algebra of deflated restarting (csrc/deflate.cpp), built with g++ on its own and
checked against numpy (not gpu).

For the (m+1) x m Hessenberg matrix Hbar of a cycle and its least-squares residual
coefficients rc (orthogonal to the range of Hbar, so parallel to every harmonic Ritz
residual), the kept
space must be spanned by the eigenvectors of G = H_m + h^2 H_m^{-T} e_m e_m^T (numpy.linalg.eig)
for the k harmonic Ritz values of smallest modulus; those vectors close under Hbar
(Hbar P_k = P_{k+1} Hk, the property deflated restarting rests on); P is orthonormal with the
residual direction last; Qt Hk = [R; 0] with R upper triangular."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0809_4802_amd", "csrc")
SHIM = r"""
#include "deflate.h"
#include <algorithm>
extern "C" int dr_setup_c(int m, int k, const double* H, int ldh, const double* rc, double* P, double* Hk,
                          double* Qt, double* R) {
    vms::DrSetup s;
    const int kk = vms::dr_setup(m, k, H, ldh, rc, &s);
    if (kk == 0) return 0;
    std::copy(s.P.begin(), s.P.end(), P);
    std::copy(s.Hk.begin(), s.Hk.end(), Hk);
    std::copy(s.Qt.begin(), s.Qt.end(), Qt);
    std::copy(s.R.begin(), s.R.end(), R);
    return kk;
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("deflate")
    shim = d / "shim.cpp"
    shim.write_text(SHIM)
    so = d / "libdeflate_check.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(shim),
                           os.path.join(CSRC, "deflate.cpp"), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    L.dr_setup_c.restype = ctypes.c_int
    return L


def _call(L, H, rc, k):
    m = H.shape[1]
    ldh = m + 3                                          # padded leading dimension
    Hc = np.zeros((m, ldh))
    Hc[:, :m + 1] = H.T                                  # column-major storage
    P = np.zeros((k + 2) * (m + 1))
    Hk = np.zeros((k + 2) * (k + 1))
    Qt = np.zeros((k + 2) ** 2)
    R = np.zeros((k + 1) ** 2)
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    kk = L.dr_setup_c(m, k, ptr(Hc), ldh, ptr(np.ascontiguousarray(rc)), ptr(P), ptr(Hk), ptr(Qt), ptr(R))
    P = P[:(kk + 1) * (m + 1)].reshape(kk + 1, m + 1).T
    Hk = Hk[:(kk + 1) * kk].reshape(kk, kk + 1).T
    Qt = Qt[:(kk + 1) ** 2].reshape(kk + 1, kk + 1).T
    R = R[:kk * kk].reshape(kk, kk).T
    return kk, P, Hk, Qt, R


def _hessenberg(m, seed, shift=0.0, j0=0):
    """A random (m+1) x m Hessenberg matrix; with j0 > 0 its leading (j0+1) x j0 block is full,
    as after a deflated restart that kept j0 vectors."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m + 1, m)) / np.sqrt(m)
    H = np.triu(A, -1)
    H[:j0 + 1, :j0] = A[:j0 + 1, :j0]
    H[np.arange(1, m + 1), np.arange(m)] = np.abs(H[np.arange(1, m + 1), np.arange(m)]) + 0.1
    H[:m] += shift * np.eye(m)
    # rc is a least-squares residual c - Hbar y, orthogonal to the range of Hbar, as in GMRES
    c = rng.standard_normal(m + 1)
    y = np.linalg.lstsq(H, c, rcond=None)[0]
    return H, c - H @ y


@pytest.mark.parametrize("m,k,seed,shift,j0", [(50, 10, 1, 0.0, 0), (50, 10, 2, 0.3, 0), (30, 5, 3, 1.0, 0),
                                               (64, 16, 4, 0.0, 0), (50, 10, 5, 0.0, 11), (40, 8, 6, 0.5, 9),
                                               (64, 32, 7, 0.0, 33)])
def test_kept_space_is_the_smallest_harmonic_ritz_vectors(lib, m, k, seed, shift, j0):
    H, rc = _hessenberg(m, seed, shift, j0)
    _check_kept_space(lib, H, rc, k)


def test_small_subdiagonals(lib):
    """Subdiagonal entries spread over six decades, as near a breakdown of the Arnoldi process.
    H_m is then ill-conditioned.  Every harmonic Ritz residual is parallel to the left null
    vector (-h f; 1) of Hbar, so closure holds only as far as that vector, computed from
    f = H_m^{-T} e_m, and the given rc agree: to about cond(H_m) times the rounding unit.  The
    span of the kept vectors is still checked tightly against numpy."""
    m, k = 50, 10
    H, _ = _hessenberg(m, 8)
    rng = np.random.default_rng(9)
    H[np.arange(1, m + 1), np.arange(m)] *= 10.0 ** rng.uniform(-6.0, 0.0, m)
    c = rng.standard_normal(m + 1)
    rc = c - H @ np.linalg.lstsq(H, c, rcond=None)[0]
    cond = np.linalg.cond(H[:m])
    assert cond > 1e10
    _check_kept_space(lib, H, rc, k, closure_rtol=100 * cond * np.finfo(float).eps)


def _check_kept_space(lib, H, rc, k, closure_rtol=1e-10):
    m = H.shape[1]
    kk, P, Hk, Qt, R = _call(lib, H, rc, k)
    assert kk in (k, k + 1)
    # P orthonormal, the first kk columns with a zero last row, the last one the residual direction
    assert np.allclose(P.T @ P, np.eye(kk + 1), atol=1e-12)
    assert np.abs(P[m, :kk]).max() == 0.0
    r_perp = rc - P[:, :kk] @ (P[:, :kk].T @ rc)
    assert np.allclose(P[:, kk], r_perp / np.linalg.norm(r_perp), atol=1e-12)
    # the kept basis is a Krylov one: Hk is upper Hessenberg
    assert np.abs(np.tril(Hk, -2)).max() == 0.0
    # closure: Hbar P_k stays inside span(P) and Hk is its matrix
    HP = H @ P[:m, :kk]
    assert np.allclose(HP, P @ Hk, atol=closure_rtol * np.abs(HP).max())
    # the span is numpy's eigenvectors of G for the kk harmonic Ritz values of smallest modulus
    Hm, h = H[:m], H[m, m - 1]
    f = np.linalg.solve(Hm.T, np.eye(m)[-1])
    G = Hm + h * h * np.outer(f, np.eye(m)[-1])
    th, W = np.linalg.eig(G)
    sel = np.argsort(np.abs(th))[:kk]
    Wr = np.concatenate([W[:, sel].real, W[:, sel].imag], axis=1)
    Q = P[:m, :kk]
    resid = Wr - Q @ (Q.T @ Wr)
    assert np.linalg.norm(resid) <= 1e-8 * np.linalg.norm(Wr), np.linalg.norm(resid)
    # QR of Hk
    assert np.allclose(Qt @ Qt.T, np.eye(kk + 1), atol=1e-12)
    QH = Qt @ Hk
    assert np.allclose(QH[:kk], R, atol=1e-12 * np.abs(Hk).max()) and np.abs(QH[kk]).max() <= 1e-12 * np.abs(Hk).max()
    assert np.allclose(R, np.triu(R))


def test_singular_leading_block_keeps_nothing(lib):
    m = 8
    H = np.zeros((m + 1, m))
    H[np.arange(1, m + 1), np.arange(m)] = 1.0          # H_m is singular (zero first row)
    kk, *_ = _call(lib, H, np.ones(m + 1), 3)
    assert kk == 0


# ---- the Francis double-shift QR itself (eigenvalues of an upper Hessenberg matrix) ----------
EIG_SHIM = r"""
#include "deflate.cpp"
extern "C" int hess_eig_c(int n, const double* a, double* re, double* im) {
    std::vector<double> w(a, a + (size_t)n * n);
    std::vector<std::complex<double>> ev;
    if (!vms::hessenberg_eigenvalues(n, w, ev)) return 0;
    for (int i = 0; i < (int)ev.size(); ++i) {
        re[i] = ev[i].real();
        im[i] = ev[i].imag();
    }
    return (int)ev.size();
}
"""


@pytest.fixture(scope="module")
def eig_lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("hess_eig")
    shim = d / "eig_shim.cpp"
    shim.write_text(EIG_SHIM)
    so = d / "libhess_eig.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(shim), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    L.hess_eig_c.restype = ctypes.c_int
    return L


def _eig(L, H):
    n = H.shape[0]
    a = np.ascontiguousarray(H, dtype=np.float64)         # row-major, as the routine takes it
    re, im = np.zeros(n), np.zeros(n)
    ptr = lambda v: v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    got = L.hess_eig_c(n, ptr(a), ptr(re), ptr(im))
    assert got == n
    return re + 1j * im


def _same_spectrum(ev, ref, tol):
    """Each computed eigenvalue matched to a distinct reference one (greedy on distance)."""
    ref = list(ref)
    for z in ev:
        k = int(np.argmin([abs(z - r) for r in ref]))
        assert abs(z - ref[k]) <= tol, (z, ref[k])
        ref.pop(k)


def test_cyclic_shift_needs_the_exceptional_shifts(eig_lib):
    """The cyclic permutation (ones below the diagonal, one in the corner) is orthogonal with its
    eigenvalues the n-th roots of unity, all of modulus 1: the standard double shifts leave it
    unchanged, and only the exceptional shifts move the iteration."""
    for n in (3, 8, 10, 13):
        C = np.zeros((n, n))
        C[np.arange(1, n), np.arange(n - 1)] = 1.0
        C[0, n - 1] = 1.0
        ev = _eig(eig_lib, C)
        _same_spectrum(ev, np.exp(2j * np.pi * np.arange(n) / n), 1e-10)


def test_prescribed_spectrum_with_pairs_and_repeats(eig_lib):
    """A Hessenberg matrix similar to a block-diagonal one with chosen eigenvalues: real ones
    (one repeated), complex pairs, and values of equal modulus."""
    import scipy.linalg as sl
    rng = np.random.default_rng(21)
    real = [0.5, -1.25, 2.0, 2.0, 3.5, -0.75]
    pairs = [(1.0, 2.0), (-0.5, 0.75), (0.0, 3.0), (2.0, 0.0001)]
    blocks = [np.array([[x]]) for x in real] + [np.array([[a, b], [-b, a]]) for a, b in pairs]
    T = sl.block_diag(*blocks)
    n = T.shape[0]
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    H = sl.hessenberg(Q @ T @ Q.T)
    ref = real + [complex(a, s * b) for a, b in pairs for s in (1, -1)]
    _same_spectrum(_eig(eig_lib, H), ref, 1e-8 * np.abs(ref).max())


def test_split_and_small_matrices(eig_lib):
    """A zero subdiagonal entry splits the problem; 1x1 and 2x2 blocks are solved directly."""
    rng = np.random.default_rng(5)
    H = np.triu(rng.standard_normal((9, 9)), -1)
    H[4, 3] = 0.0
    _same_spectrum(_eig(eig_lib, H), np.linalg.eigvals(H), 1e-10 * np.abs(H).max() * 9)
    _same_spectrum(_eig(eig_lib, np.array([[2.5]])), [2.5], 0.0)
    for M in (np.array([[1.0, 2.0], [-3.0, 1.0]]), np.array([[4.0, 1.0], [2.0, 3.0]])):
        _same_spectrum(_eig(eig_lib, M), np.linalg.eigvals(M), 1e-13)
