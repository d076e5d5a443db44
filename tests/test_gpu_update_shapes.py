"""The Gram-Schmidt update's row split across XCDs, through the C ABI (gpu).

The update launch splits the vector rows in eighths, one per XCD: the rows the dots launch
formed there when the dots have a multiple of 8 chunks (8 or 16 chunks below 131,072 nodes, 64
from there on), even eighths otherwise; FP32 vectors and meshes from 131,072 nodes on take two
rows per thread.  Cavity boxes sized to land on each case and on both sides of the 131,072-node
threshold carry a random system on their block pattern (no Dirichlet dofs; diagonal blocks
4 I plus noise, every other block noise of row norm about 3), whose GMRES converges in a few
restart cycles at any size, so that every mesh exercises full Arnoldi columns: the solve must
reach its tolerance, checked with the true residual recomputed on the host from the stored
matrix (scipy, FP64)."""
import numpy as np
import pytest
import torch

from workloads.mesh import kuhn_box
from tests.gpu_common import DEV, bsr_to_csr, make_context, to_dev

pytestmark = pytest.mark.gpu


def _chunks(n_nodes):
    return 64 if n_nodes >= 131072 else max(1, min(16, (n_nodes + 255) // 256))


@pytest.mark.parametrize("dims,chunks", [((11, 11, 11), 7), ((12, 12, 11), 8), ((12, 12, 12), 9),
                                         ((15, 15, 15), 16), ((50, 50, 49), 16), ((50, 50, 50), 64)])
@pytest.mark.parametrize("precision", [0, 1])
def test_gmres_reaches_its_tolerance_for_every_row_split(vms_lib, dims, chunks, precision):
    B = vms_lib
    m = kuhn_box(dims, (0, 0, 0), (1, 1, 1), name="box")
    assert _chunks(m.n_nodes) == chunks
    print(f"update row split: box {dims}, {m.n_nodes} nodes, {chunks} dot chunks, precision {precision}",
          flush=True)
    ctx = make_context(B, m, np.zeros(0, np.int32), precision)     # no Dirichlet dofs: a plain system
    rowptr, colidx, diagpos = ctx.bsr_pattern()
    rng = np.random.default_rng(sum(dims) + 100 * precision)
    vals = 1.5 * rng.standard_normal((ctx.nb, 4, 4)) / np.sqrt(15.0)
    vals[diagpos] = 4.0 * np.eye(4) + 0.3 * rng.standard_normal((m.n_nodes, 4, 4))
    A = torch.from_numpy(vals.reshape(ctx.nb, 16)).to(DEV).to(ctx.dtype).contiguous()
    rhs = to_dev(rng.standard_normal((m.n_nodes, 4)))
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=30, rtol=1e-10, max_iters=2000))
    Am = bsr_to_csr(ctx, A)
    b = rhs.cpu().numpy().ravel()
    rel = np.linalg.norm(b - Am @ x.cpu().numpy().ravel()) / np.linalg.norm(b)
    print(f"  rc {rc}, steps {info.iters}, cycles {info.restarts}, true residual {rel:.2e}")
    assert rc == B.VMS_OK and info.true_rel_res <= 1e-10 and info.iters > 30
    assert rel <= 1.01e-10
