"""Pins of the learned block-Jacobi oracle (not gpu).

  * central differences of the loss                          -> the gradient
  * a zero output layer gives P_i = D_i^-1 exactly             -> the wiring
  * loss of the exact block-diagonal inverse on a block-diagonal A is 0
  * Adam's first step moves every weight by lr (bias correction)
"""
import numpy as np
import scipy.sparse as sp

from oracle import vms
from oracle import learned_pc as lp
from workloads import cavity_mesh, cavity_bc, apply_dirichlet


def _system(re=50.0):
    m = cavity_mesh(3)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    prob = vms.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / re)
    A, b, _, _ = vms.condensed_system(prob, u, np.zeros((m.n_elems, 3)))
    return m, bc, A, b


def test_gradient_matches_central_differences():
    m, bc, A, b = _system()
    x, D = lp.features(A, m.n_nodes, bc.dofs)
    mask = lp.dirichlet_mask(m.n_nodes, bc.dofs)
    rng = np.random.default_rng(0)
    w = lp.init_weights(1)
    w[lp.N_HID * lp.N_IN + lp.N_HID:] = 0.02 * rng.standard_normal(lp.N_OUT * lp.N_HID + lp.N_OUT)
    rs = [b] + [rng.standard_normal(b.size) for _ in range(2)]
    for r in rs:
        r[bc.dofs] = 0.0
    _, g = lp.loss_and_grad(w, A, x, D, mask, rs)
    idx = rng.choice(w.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (lp.loss_and_grad(wp, A, x, D, mask, rs)[0]
              - lp.loss_and_grad(wm, A, x, D, mask, rs)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max()), i


def test_zero_output_layer_is_block_jacobi():
    m, bc, A, b = _system()
    x, D = lp.features(A, m.n_nodes, bc.dofs)
    mask = lp.dirichlet_mask(m.n_nodes, bc.dofs)
    P = lp.preconditioner_blocks(lp.init_weights(1), x, D, mask)
    assert np.allclose(P, vms.block_jacobi_inverse(A, m.n_nodes), rtol=1e-12, atol=1e-14)
    assert x.shape == (m.n_nodes, lp.N_IN) and np.isfinite(x).all()
    # Dirichlet flags and unit Dirichlet rows
    flags = x[:, 21:25].ravel()
    assert np.array_equal(np.nonzero(flags)[0], np.sort(bc.dofs))


def test_exact_inverse_gives_zero_loss():
    rng = np.random.default_rng(4)
    n = 6
    blocks = rng.standard_normal((n, 4, 4)) + 4 * np.eye(4)
    A = sp.block_diag(list(blocks)).tocsr()
    x, D = lp.features(A, n, np.array([], dtype=np.int64))
    mask = lp.dirichlet_mask(n, np.array([], dtype=np.int64))
    rs = [rng.standard_normal(4 * n)]
    loss, g = lp.loss_and_grad(lp.init_weights(1), A, x, D, mask, rs)
    assert loss < 1e-28 and np.abs(g).max() < 1e-12


def test_adam_first_step():
    rng = np.random.default_rng(2)
    w = rng.standard_normal(10)
    g = rng.standard_normal(10)
    w1, m, v = lp.adam_step(w, g, np.zeros(10), np.zeros(10), 1, lr=0.01)
    assert np.allclose(w - w1, 0.01 * np.sign(g), rtol=1e-6)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
