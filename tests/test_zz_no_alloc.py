"""The no-allocation entry point vms_condense_assemble_noalloc against vms_condense_assemble.

Two calls in a row on one GPU, the second on a smaller mesh (fewer assembly tiles), in both
precisions: the condensed tangent, rhs and residual norm of the two entry points must agree to
the tolerances of the method (FP64 1e-12, mixed 1e-5 on the tangent; the rhs and the norm are
FP64 in both).  The LDS accumulation order of the assembly is not fixed, so the comparison is
norm-wise.
"""
import numpy as np
import pytest
import torch

from workloads import cavity_mesh, cavity_bc, apply_dirichlet
from tests.gpu_common import DEV, make_context, to_dev

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = a.double()
    b = b.double()
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_condense_assemble(vms_lib, precision):
    B = vms_lib
    tol = 1e-12 if precision == B.VMS_FP64 else 1e-5
    for n, seed in ((16, 3), (6, 4)):           # the second call has the smaller input
        m = cavity_mesh(n)
        bc = cavity_bc(m)
        rng = np.random.default_rng(seed)
        u = rng.standard_normal((m.n_nodes, 4))
        apply_dirichlet(u, bc)
        up = u + 0.05 * rng.standard_normal(u.shape)
        beta = 0.05 * rng.standard_normal((m.n_elems, 3))
        ctx = make_context(B, m, bc.dofs, precision)
        ud, upd, bd = to_dev(u), to_dev(up), to_dev(beta)
        A0, r0, n0 = B.vms_condense_assemble(ctx, ud, bd, 200.0, 0.02, upd)
        A1 = ctx.new_bsr()
        r1 = ctx.new_vec()
        n1 = torch.zeros(1, dtype=torch.float64, device=DEV)
        B.vms_condense_assemble_noalloc(ctx, ud, bd, 200.0, A1, r1, n1, 0.02, upd)
        torch.cuda.synchronize()
        ea, er = _rel(A1, A0), _rel(r1, r0)
        en = abs(float(n1.item()) - float(n0.item())) / float(n0.item())
        print(f"cavity {n}^3 precision {precision}: tangent {ea:.2e}, rhs {er:.2e}, norm {en:.2e}")
        assert ea <= tol and er <= 1e-12 and en <= 1e-12
        ctx.close()
