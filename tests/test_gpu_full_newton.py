"""Uncondensed Newton-Raphson on the GPU (Section 4.2, Eq. NewtonUpdate2), through the C ABI.

The uncondensed system is laid out over n_nodes + n_elems block rows (node dofs, then the
three fine dofs of each element and one unused slot); the oracle numbers the fine dofs of
element e at 4 n_nodes + 3 e + i.  Tolerances: FP64 1e-12 on the assembled matrix and rhs,
mixed 1e-5; one FP64 Newton-Raphson step against the oracle's brute-force step (sparse LU)
and against the Newton-Schur step, which reaches the same iterate (block elimination is
exact algebra, Section 5).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import vms as O
from workloads import kuhn_box, jitter_interior, cavity_mesh, cavity_bc, apply_dirichlet, boundary_nodes
from tests.gpu_common import DEV, to_dev, random_state, rel_fro

pytestmark = pytest.mark.gpu


def _mesh():
    m = jitter_interior(kuhn_box((3, 4, 5), (0, 0, 0), (1.0, 1.2, 1.4)), 0.2, 5)
    bnd = np.nonzero(boundary_nodes(m.tets, m.n_nodes))[0]
    dofs = np.unique(np.concatenate([(4 * bnd[:, None] + np.arange(3)).ravel(), [3]])).astype(np.int32)
    return m, dofs


def _context(B, m, dofs, precision):
    return B.Context(to_dev(m.xyz), to_dev(m.tets.astype(np.int32)), to_dev(dofs), precision=precision,
                     full_system=True)


def _to_oracle_layout(ctx, vals, rhs, m):
    """scipy CSR over the oracle's 4 n_nodes + 3 n_elems dofs, the rhs in the same order, and the
    entries of the unused slots (which must be an identity)."""
    rowptr, colidx = ctx.full_pattern()
    nr = ctx.full_rows
    v = vals.detach().double().cpu().numpy().reshape(-1, 4, 4)
    brow = np.repeat(np.arange(nr), np.diff(rowptr))
    rows = (4 * brow[:, None, None] + np.arange(4)[None, :, None]).repeat(4, axis=2).ravel()
    cols = (4 * colidx[:, None, None] + np.arange(4)[None, None, :]).repeat(4, axis=1).ravel()
    nn = m.n_nodes
    perm = np.full(4 * nr, -1, dtype=np.int64)
    perm[:4 * nn] = np.arange(4 * nn)
    e = np.arange(m.n_elems)
    for q in range(3):
        perm[4 * (nn + e) + q] = 4 * nn + 3 * e + q
    keep = (perm[rows] >= 0) & (perm[cols] >= 0)
    n = 4 * nn + 3 * m.n_elems
    A = sp.csr_matrix((v.ravel()[keep], (perm[rows[keep]], perm[cols[keep]])), shape=(n, n))
    dummy = sp.csr_matrix((v.ravel()[~keep], (rows[~keep], cols[~keep])), shape=(4 * nr, 4 * nr))
    r = rhs.cpu().numpy().ravel()
    b = np.zeros(n)
    b[perm[perm >= 0]] = r[perm >= 0]
    return A, b, dummy, r[perm < 0]


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_full_assemble_matches_oracle(vms_lib, precision, tol):
    B = vms_lib
    m, dofs = _mesh()
    ctx = _context(B, m, dofs, precision)
    assert ctx.full_rows == m.n_nodes + m.n_elems
    u, up, beta, body = random_state(m, 21)
    Re, dt = 40.0, 0.05
    vals, rhs, rn = B.vms_full_assemble(ctx, to_dev(u), to_dev(beta), Re, dt, to_dev(up), to_dev(body))
    torch.cuda.synchronize()
    A, b, dummy, rdummy = _to_oracle_layout(ctx, vals, rhs, m)
    prob = O.Problem(m.xyz, m.tets, dofs, nu=1.0 / Re, dt=dt, u_prev=up, body=body)
    A_o, b_o = O.full_system(prob, u, beta)
    assert sp.linalg.norm(A - A_o) <= tol * sp.linalg.norm(A_o)
    assert np.linalg.norm(b - b_o) <= 1e-12 * np.linalg.norm(b_o)      # residual rows are FP64 in both paths
    d = dummy.tocoo()
    nz = d.data != 0.0
    assert np.all(d.row[nz] == d.col[nz]) and np.all(d.data[nz] == 1.0) and nz.sum() == m.n_elems
    assert np.all(rdummy == 0.0)
    assert abs(rn.item() - O.residual_norm_at(prob, u, beta)) <= 1e-12 * rn.item()


def test_full_newton_step_matches_oracle_and_schur(vms_lib):
    B = vms_lib
    m, dofs = _mesh()
    u, up, beta, body = random_state(m, 22, beta_scale=0.05, vel_scale=0.5)
    u.ravel()[dofs] = 0.3
    Re, dt = 30.0, 0.1
    lin = B.solve_opts(rtol=1e-12, max_iters=40000)
    ctx = _context(B, m, dofs, B.VMS_FP64)
    ud, bd = to_dev(u), to_dev(beta)
    info = B.vms_full_newton_step(ctx, ud, bd, Re, dt, to_dev(up), to_dev(body), lin)
    assert info.lin.true_rel_res <= 1e-12
    prob = O.Problem(m.xyz, m.tets, dofs, nu=1.0 / Re, dt=dt, u_prev=up, body=body)
    u_o, b_o = O.full_newton_step(prob, u, beta)
    assert rel_fro(ud.cpu().numpy(), u_o) <= 1e-10
    assert rel_fro(bd.cpu().numpy(), b_o) <= 1e-9
    # the Newton-Schur step from the same state reaches the same iterate
    us, bs = to_dev(u), to_dev(beta)
    B.vms_newton_step(ctx, us, bs, Re, dt, to_dev(up), to_dev(body), lin)
    assert rel_fro(ud.cpu().numpy(), us.cpu().numpy()) <= 1e-10
    assert rel_fro(bd.cpu().numpy(), bs.cpu().numpy()) <= 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_full_newton_converges_to_the_schur_solution(vms_lib, precision):
    """Cavity 4^3, Re 100: Newton-Raphson on the uncondensed system reaches the residual
    tolerance (by the oracle's residual) and the same solution as Newton-Schur."""
    B = vms_lib
    m = cavity_mesh(4)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    ctx = _context(B, m, bc.dofs, precision)
    Re, tol = 100.0, (1e-10 if precision == 0 else 1e-8)
    lin = B.solve_opts(rtol=tol / 10, max_iters=40000)
    solutions = []
    for step in (B.vms_full_newton_step, B.vms_newton_step):
        ud = to_dev(u)
        bd = torch.zeros((m.n_elems, 3), dtype=torch.float64, device=DEV)
        r0 = None
        for _ in range(15):
            info = step(ctx, ud, bd, Re, 0.0, None, None, lin)
            r0 = info.rnorm_before if r0 is None else r0
            if info.rnorm_after <= tol * r0:
                break
        prob = O.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / Re)
        assert O.residual_norm_at(prob, ud.cpu().numpy(), bd.cpu().numpy()) <= 1.01 * tol * r0
        solutions.append(ud.cpu().numpy())
    assert rel_fro(solutions[0], solutions[1]) <= (1e-8 if precision == 0 else 1e-5)


def test_full_newton_inexact_cavity16_iterations(vms_lib):
    """Cavity 16^3, Re 100, inexact Newton (forcing terms) to 1e-8: Newton-Raphson and
    Newton-Schur take the same number of Newton steps and comparable GMRES iterations.  The
    near-singular constant-pressure mode needs the coarse correction in both systems; without
    it restarted GMRES on the uncondensed system stalls near convergence."""
    from paper_0809_4802_amd import driver
    B = vms_lib
    m = cavity_mesh(16)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    ctx = _context(B, m, bc.dofs, B.VMS_FP64)
    out = {}
    for method in ("full", "schur"):
        ud = to_dev(u)
        bd = torch.zeros((m.n_elems, 3), dtype=torch.float64, device=DEV)
        r = driver.newton_solve(ctx, ud, bd, 100.0, tol=1e-8, lin=B.solve_opts(rtol=1e-9, max_iters=20000),
                                forcing="ew", method=method)
        out[method] = (r, ud.cpu().numpy())
    (rf, uf), (rs, us) = out["full"], out["schur"]
    it_f = sum(d["iters"] for d in rf.lin)
    it_s = sum(d["iters"] for d in rs.lin)
    print(f"cavity16 Re 100: Newton-Raphson {len(rf.rnorms) - 1} steps {it_f} GMRES iterations {rf.seconds:.3f} s; "
          f"Newton-Schur {len(rs.lin)} steps {it_s} iterations {rs.seconds:.3f} s")
    assert len(rf.lin) == len(rs.lin)
    assert it_f <= 1.5 * it_s
    assert rel_fro(uf, us) <= 1e-6
