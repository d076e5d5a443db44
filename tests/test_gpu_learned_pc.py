"""Learned block-Jacobi correction: GPU kernels (through the C ABI) against the FP64 oracle.

The oracle functions are fed the GPU-assembled matrix (converted to scipy) so that
only the learned-preconditioner arithmetic is compared.  FP32 kernels: features and
blocks to 1e-5, loss and gradient to 1e-3 (norm-wise), Adam to 1e-5.
"""
import numpy as np
import pytest
import torch

from oracle import learned_pc as LP
from oracle import vms as O
from workloads import cavity_mesh, cavity_bc, apply_dirichlet
from tests.gpu_common import DEV, to_dev, make_context, bsr_to_csr, rel_fro

pytestmark = pytest.mark.gpu


def _system(B, precision, n=5, re=50.0):
    m = cavity_mesh(n)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    ctx = make_context(B, m, bc.dofs, precision)
    A_g, b_g, _ = B.vms_condense_assemble(ctx, to_dev(u), to_dev(np.zeros((m.n_elems, 3))), re)
    torch.cuda.synchronize()
    return m, bc, ctx, A_g, b_g, bsr_to_csr(ctx, A_g)


def _weights(seed, out_scale=0.05):
    rng = np.random.default_rng(seed)
    w = LP.init_weights(1)
    n_out = LP.N_OUT * LP.N_HID + LP.N_OUT
    w[-n_out:] = out_scale * rng.standard_normal(n_out)
    return w


@pytest.mark.parametrize("precision", [0, 1])
def test_features_and_blocks(vms_lib, precision):
    B = vms_lib
    m, bc, ctx, A_g, b_g, A = _system(B, precision)
    feats = B.vms_pc_features(ctx, A_g).cpu().numpy()
    x_o, D = LP.features(A, m.n_nodes, bc.dofs)
    assert rel_fro(feats, x_o) <= 1e-5
    P_bj = B.vms_pc_blocks(ctx, A_g, None).cpu().numpy().reshape(-1, 4, 4)
    assert rel_fro(P_bj, O.block_jacobi_inverse(A, m.n_nodes)) <= 1e-5
    w = _weights(3)
    P = B.vms_pc_blocks(ctx, A_g, to_dev(w.astype(np.float32))).cpu().numpy().reshape(-1, 4, 4)
    P_o = LP.preconditioner_blocks(w.astype(np.float32).astype(np.float64), x_o, D,
                                   LP.dirichlet_mask(m.n_nodes, bc.dofs))
    assert rel_fro(P, P_o) <= 1e-5


def test_loss_gradient_and_adam(vms_lib):
    B = vms_lib
    m, bc, ctx, A_g, b_g, A = _system(B, B.VMS_FP64)
    rng = np.random.default_rng(7)
    rs = [b_g.cpu().numpy().ravel()] + [rng.standard_normal(4 * m.n_nodes) for _ in range(2)]
    for r in rs:
        r[bc.dofs] = 0.0
    rs32 = np.stack(rs).astype(np.float32)
    w = _weights(4)
    w32 = w.astype(np.float32)
    wd = to_dev(w32)
    grad = torch.zeros(B.PC_NWEIGHTS, dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    B.vms_pc_train_step(ctx, A_g, to_dev(rs32.reshape(3, -1, 4)), wd, None, 0, 0.0, grad, loss)
    x_o, D = LP.features(A, m.n_nodes, bc.dofs)
    mask = LP.dirichlet_mask(m.n_nodes, bc.dofs)
    L_o, g_o = LP.loss_and_grad(w32.astype(np.float64), A, x_o, D, mask,
                                [r.astype(np.float64) for r in rs32])
    assert abs(loss.item() - L_o) <= 1e-4 * L_o
    assert rel_fro(grad.cpu().numpy(), g_o) <= 1e-3
    assert np.array_equal(wd.cpu().numpy(), w32)          # lr = 0: no update
    # one Adam step
    state = torch.zeros(2 * B.PC_NWEIGHTS, dtype=torch.float32, device=DEV)
    B.vms_pc_train_step(ctx, A_g, to_dev(rs32.reshape(3, -1, 4)), wd, state, 1, 1e-3, grad, loss)
    w_new, _, _ = LP.adam_step(w32.astype(np.float64), grad.cpu().numpy().astype(np.float64),
                               np.zeros_like(w), np.zeros_like(w), 1, lr=1e-3)
    assert np.max(np.abs(wd.cpu().numpy() - w_new)) <= 1e-5


def test_training_lowers_the_loss_and_gmres_uses_it(vms_lib):
    from paper_0809_4802_amd import learned
    B = vms_lib
    m, bc, ctx, A_g, b_g, A = _system(B, B.VMS_MIXED, n=6, re=100.0)
    samples = learned.collect_samples(ctx, A_g, b_g, n_samples=8, cycle_iters=20)
    assert samples.shape[0] >= 2
    w, hist = learned.train(ctx, [(A_g, samples)], steps=60, lr=3e-3, batch=4, seed=1)
    assert hist[-1] < hist[0]
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A_g, b_g, x, B.solve_opts(rtol=1e-9, pc=B.VMS_PC_LEARNED, pc_weights=w,
                                                                max_iters=20000))
    assert rc == 0 and info.true_rel_res <= 1e-9 and info.fell_back_to_bj == 0
    bad = w.clone()
    bad[-1] = float("nan")
    x2 = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A_g, b_g, x2, B.solve_opts(rtol=1e-9, pc=B.VMS_PC_LEARNED, pc_weights=bad,
                                                                 max_iters=20000))
    assert rc == 0 and info.fell_back_to_bj == 1 and info.true_rel_res <= 1e-9


def test_restart_residual_logging(vms_lib):
    B = vms_lib
    m, bc, ctx, A_g, b_g, A = _system(B, B.VMS_FP64)
    log = torch.zeros((4, m.n_nodes, 4), dtype=torch.float32, device=DEV)
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A_g, b_g, x, B.solve_opts(restart=10, rtol=1e-12, max_iters=25,
                                                                log_residuals=log), allow_noconv=True)
    assert info.logged >= 3
    first = log[0].cpu().numpy().ravel()
    assert rel_fro(first, b_g.cpu().numpy().ravel()) <= 1e-6       # x0 = 0: r0 = b


def test_trained_correction_gains_over_block_jacobi(vms_lib):
    """Trained on the Newton systems of one cavity 16^3 solve at Re 100 (checkpoints selected on
    its last system), evaluated on Newton systems at Re 150 it never saw: GMRES(50) iterations
    to 1e-6 with the learned blocks against plain block-Jacobi."""
    from paper_0809_4802_amd import learned, driver
    B = vms_lib
    m = cavity_mesh(16)
    bc = cavity_bc(m)
    u0 = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u0, bc)
    ctx = make_context(B, m, bc.dofs, B.VMS_MIXED)
    data, _ = learned.collect_newton_data(ctx, to_dev(u0), to_dev(np.zeros((m.n_elems, 3))), 100.0,
                                          lin=B.solve_opts(restart=50, rtol=1e-4, max_iters=40000), per_step=32)
    assert len(data) >= 3
    val = [(A, S[0].contiguous()) for A, S in data[-1:]]
    w, report = learned.train_validated(ctx, data[:-1], val, steps=200, lr=3e-4)
    assert w is not None, report
    # held-out systems: the first two Newton systems at Re 150
    u = to_dev(u0)
    beta = torch.zeros((m.n_elems, 3), dtype=torch.float64, device=DEV)
    tests = []
    for _ in range(2):
        A, b, _ = B.vms_condense_assemble(ctx, u, beta, 150.0)
        tests.append((A.clone(), b.clone()))
        B.vms_newton_step(ctx, u, beta, 150.0, 0.0, None, None, B.solve_opts(rtol=1e-6, max_iters=40000))
    it_bj = sum(learned.gmres_iterations(ctx, A, b, None, rtol=1e-6) for A, b in tests)
    it_ln = sum(learned.gmres_iterations(ctx, A, b, w, rtol=1e-6) for A, b in tests)
    print(f"learned correction: validation {report['val_iters_bj']} -> {report['val_iters_selected']} iterations; "
          f"held-out Re 150 systems: block-Jacobi {it_bj}, learned {it_ln} ({it_ln / it_bj:.2f}x)")
    assert it_ln < 0.9 * it_bj
