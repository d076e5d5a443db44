"""ORACLE (test infrastructure): Newton-Schur method, plain FP64, CPU.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library.

Steps, in the paper's order:
  element residual / tangent         Section 4.1-4.2   (element.c, quadrature)
  element Schur condensation         Section 5, Eq. (SchurUpdate) and the
                                     assembled blocks K_vv, K_vp, K_pv, K_pp, R_1, R_2
  assembly + Dirichlet elimination   Section 5 (assembly operator), Section 6
  linear solve                       Section 6 (Krylov solver; here also direct)
  fine-scale recovery                Section 5 (increment of the fine scales)
  Newton update                      Section 4.2 (update of vbar, p, v')
  brute-force full Newton            Section 4.2, Eq. (NewtonUpdate2), all
                                     4 n_nodes + 3 n_elems unknowns at once
Conventions: u [n_nodes, 4] = (vx, vy, vz, p), beta [n_elems, 3]; the global
coarse dof of (node, c) is 4 node + c; nu = 1 / Re; K Delta = -R.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import element_residual_tangent


# ----------------------------------------------------------------------------- condensation
def condense(R, K):
    """Element Schur complement of the fine scales (Section 5).

    K* = K_cc - K_cf K_ff^-1 K_fc   (16 x 16: the four condensed blocks)
    R* = R_cp - K_cf K_ff^-1 R_f    (16: the condensed residuals R_1, R_2)
    K_ff^-1 is applied by LU with partial pivoting (numpy.linalg.solve).
    """
    Kcc = K[:, :16, :16]
    Kcf = K[:, :16, 16:]
    Kfc = K[:, 16:, :16]
    Kff = K[:, 16:, 16:]
    W = np.linalg.solve(Kff, Kfc)                              # K_ff^-1 K_fc
    z = np.linalg.solve(Kff, R[:, 16:, None])[..., 0]          # K_ff^-1 R_f
    Kstar = Kcc - Kcf @ W
    Rstar = R[:, :16] - np.einsum("eij,ej->ei", Kcf, z)
    return Kstar, Rstar


def recover_fine(R, K, du_e):
    """Fine-scale increment dbeta = K_ff^-1 (-R_f - K_fc du_e) (Section 5).

    K_fc holds both dR_f/dvbar and dR_f/dp, so du_e is the element's
    16-vector of coarse increments (velocity and pressure)."""
    Kfc = K[:, 16:, :16]
    Kff = K[:, 16:, 16:]
    rhs = -R[:, 16:] - np.einsum("eij,ej->ei", Kfc, du_e)
    return np.linalg.solve(Kff, rhs[..., None])[..., 0]


# ----------------------------------------------------------------------------- assembly
def element_coarse_dofs(tets):
    """[E, 16] global coarse dof ids in element dof order."""
    return (4 * tets[:, :, None].astype(np.int64) + np.arange(4)[None, None, :]).reshape(-1, 16)


def assemble_vector(tets, n_nodes, Re16):
    """Sum element 16-vectors into a global [4 n_nodes] vector (element order)."""
    out = np.zeros(4 * n_nodes)
    np.add.at(out, element_coarse_dofs(tets).ravel(), Re16.ravel())
    return out


def assemble_matrix(tets, n_nodes, Ke16, dirichlet_dofs):
    """Assemble element 16x16 blocks into CSR with Dirichlet rows and columns
    replaced by the identity (elimination with a unit diagonal)."""
    dofs = element_coarse_dofs(tets)
    rows = np.repeat(dofs, 16, axis=1).ravel()
    cols = np.tile(dofs, (1, 16)).ravel()
    vals = Ke16.reshape(Ke16.shape[0], -1).ravel().copy()
    is_d = np.zeros(4 * n_nodes, dtype=bool)
    is_d[dirichlet_dofs] = True
    vals[is_d[rows] | is_d[cols]] = 0.0
    n = 4 * n_nodes
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    diag = np.zeros(n)
    diag[dirichlet_dofs] = 1.0
    return (A + sp.diags(diag)).tocsr()


def free_mask(n_nodes, dirichlet_dofs):
    m = np.ones(4 * n_nodes, dtype=bool)
    m[dirichlet_dofs] = False
    return m


def residual_norm(tets, n_nodes, R, dirichlet_dofs):
    """FP64 Newton residual norm: ||[R_c; R_p] on free dofs, R_f on every element||_2.

    The paper stops Newton when the residual is below a tolerance
    (Section 4.2) without naming the norm; this is the reading used."""
    rc = assemble_vector(tets, n_nodes, R[:, :16])
    fm = free_mask(n_nodes, dirichlet_dofs)
    return float(np.sqrt(np.sum(rc[fm] ** 2) + np.sum(R[:, 16:] ** 2)))


@dataclass
class Problem:
    """Everything that defines one nonlinear solve on a mesh."""
    xyz: np.ndarray
    tets: np.ndarray
    dirichlet_dofs: np.ndarray
    nu: float
    dt: float = 0.0
    u_prev: np.ndarray | None = None
    body: np.ndarray | None = None
    picard: bool = False        # fixed-point tangent (advecting velocity held) instead of Newton's

    @property
    def n_nodes(self):
        return self.xyz.shape[0]

    @property
    def n_elems(self):
        return self.tets.shape[0]

    def element(self, u, beta, with_tangent=True):
        return element_residual_tangent(self.xyz, self.tets, u, beta, self.nu, self.dt,
                                        self.u_prev, self.body, with_tangent=with_tangent, picard=self.picard)


def condensed_system(prob: Problem, u, beta):
    """(A, b, R, K): assembled condensed tangent with Dirichlet elimination,
    rhs b = -R* (zero at Dirichlet dofs), and the element R, K."""
    R, K = prob.element(u, beta)
    Kstar, Rstar = condense(R, K)
    A = assemble_matrix(prob.tets, prob.n_nodes, Kstar, prob.dirichlet_dofs)
    b = -assemble_vector(prob.tets, prob.n_nodes, Rstar)
    b[prob.dirichlet_dofs] = 0.0
    return A, b, R, K


# ----------------------------------------------------------------------------- linear solves
def solve_direct(A, b):
    """Sparse LU (SuperLU via scipy) of the assembled system."""
    return spla.spsolve(A.tocsc(), b)


def block_jacobi_inverse(A, n_nodes):
    """Inverses of the 4x4 diagonal blocks [n_nodes, 4, 4]."""
    D = np.zeros((n_nodes, 4, 4))
    Acoo = A.tocoo()
    same = (Acoo.row // 4) == (Acoo.col // 4)
    r, c, v = Acoo.row[same], Acoo.col[same], Acoo.data[same]
    np.add.at(D, (r // 4, r % 4, c % 4), v)
    return np.linalg.inv(D)


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    restarts: int
    true_rel_res: float
    converged: bool


def gmres(A, b, x0=None, restart=50, max_iters=10000, rtol=1e-12, Minv_blocks=None):
    """Restarted GMRES(m), right preconditioned, modified Gram-Schmidt and
    Givens rotations (textbook form).  Success iff the true relative
    residual ||b - A x|| / ||b|| <= rtol, recomputed at every restart.

    Minv_blocks [n_nodes, 4, 4]: block-Jacobi (or other block-diagonal)
    preconditioner M; the iteration solves A M y = b, x = x0 + M y."""
    n = b.size
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return GmresResult(np.zeros(n), 0, 0, 0.0, True)

    def M(v):
        if Minv_blocks is None:
            return v
        return np.einsum("nij,nj->ni", Minv_blocks, v.reshape(-1, 4)).ravel()

    iters = 0
    restarts = 0
    while True:
        r = b - A @ x
        rn = np.linalg.norm(r)
        if rn <= rtol * bn:
            return GmresResult(x, iters, restarts, rn / bn, True)
        if iters >= max_iters:
            return GmresResult(x, iters, restarts, rn / bn, False)
        m = min(restart, max_iters - iters)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = rn
        V[0] = r / rn
        k = 0
        for j in range(m):
            w = A @ M(V[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            iters += 1
            if abs(g[j + 1]) <= rtol * bn:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + M(V[:k].T @ y)
        restarts += 1


# ----------------------------------------------------------------------------- Newton
@dataclass
class NewtonLog:
    rnorms: list = field(default_factory=list)
    lin_iters: list = field(default_factory=list)


def newton_schur_step(prob: Problem, u, beta, linear="direct", rtol=1e-12, restart=50,
                      max_iters=20000):
    """One Newton-Schur iteration.  Returns (u_new, beta_new, rnorm_before, info)."""
    A, b, R, K = condensed_system(prob, u, beta)
    rn = residual_norm(prob.tets, prob.n_nodes, R, prob.dirichlet_dofs)
    info = {}
    if linear == "direct":
        du = solve_direct(A, b)
    else:
        res = gmres(A, b, restart=restart, rtol=rtol, max_iters=max_iters,
                    Minv_blocks=block_jacobi_inverse(A, prob.n_nodes))
        if not res.converged:
            raise RuntimeError(f"GMRES did not converge ({res.iters} its, {res.true_rel_res:.2e})")
        du = res.x
        info["gmres"] = res
    du[prob.dirichlet_dofs] = 0.0
    du_e = du[element_coarse_dofs(prob.tets)]
    dbeta = recover_fine(R, K, du_e)
    return u + du.reshape(-1, 4), beta + dbeta, rn, info


def residual_norm_at(prob: Problem, u, beta):
    R, _ = prob.element(u, beta, with_tangent=False)
    return residual_norm(prob.tets, prob.n_nodes, R, prob.dirichlet_dofs)


def newton_solve(prob: Problem, u, beta, tol=1e-10, max_newton=30, **kw):
    """Newton-Schur loop until ||R_k|| <= tol ||R_0||.  Returns (u, beta, log)."""
    log = NewtonLog()
    r0 = None
    for _ in range(max_newton):
        rn = residual_norm_at(prob, u, beta)
        log.rnorms.append(rn)
        if r0 is None:
            r0 = rn
        if rn <= tol * r0 or rn == 0.0:
            return u, beta, log
        u, beta, _, info = newton_schur_step(prob, u, beta, **kw)
        if "gmres" in info:
            log.lin_iters.append(info["gmres"].iters)
    rn = residual_norm_at(prob, u, beta)
    log.rnorms.append(rn)
    if rn > tol * r0:
        raise RuntimeError(f"Newton did not converge: {log.rnorms}")
    return u, beta, log


def full_system(prob: Problem, u, beta):
    """The uncondensed Newton system of Eq. NewtonUpdate2 (Section 4.2): the 19x19 element
    Jacobians assembled over all 4 n_nodes + 3 n_elems unknowns (coarse dofs first, then the
    fine dofs of element e at 4 n_nodes + 3 e + i), Dirichlet rows and columns replaced by
    the identity.  Returns (A [csc], rhs = -R with zeros at Dirichlet dofs)."""
    R, K = prob.element(u, beta)
    nn, ne = prob.n_nodes, prob.n_elems
    nc = 4 * nn
    n = nc + 3 * ne
    dofs = np.concatenate([element_coarse_dofs(prob.tets),
                           nc + 3 * np.arange(ne)[:, None] + np.arange(3)[None, :]], axis=1)
    rows = np.repeat(dofs, 19, axis=1).ravel()
    cols = np.tile(dofs, (1, 19)).ravel()
    vals = K.reshape(ne, -1).ravel().copy()
    is_d = np.zeros(n, dtype=bool)
    is_d[prob.dirichlet_dofs] = True
    vals[is_d[rows] | is_d[cols]] = 0.0
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    diag = np.zeros(n)
    diag[prob.dirichlet_dofs] = 1.0
    A = (A + sp.diags(diag)).tocsc()
    rhs = np.zeros(n)
    np.add.at(rhs, dofs.ravel(), -R.ravel())
    rhs[prob.dirichlet_dofs] = 0.0
    return A, rhs


def full_newton_step(prob: Problem, u, beta):
    """Brute-force Newton step on the uncondensed system (Eq. NewtonUpdate2), solved by
    sparse LU."""
    A, rhs = full_system(prob, u, beta)
    d = spla.spsolve(A, rhs)
    nc = 4 * prob.n_nodes
    return u + d[:nc].reshape(-1, 4), beta + d[nc:].reshape(-1, 3)
