"""Pins of the oracle's element residual and tangent (not gpu).

What fixes each result, independently of the oracle's own code:
  * central finite differences of the residual           -> the tangent
  * a closed-form integration of the same weak form, written here from
    the bubble moments (exact integrals of barycentric monomials)  -> every
    residual and tangent term, including the fine-scale convective ones
  * patch test: a linear divergence-free velocity, a linear pressure and
    the matching body force make the discrete residual vanish    -> signs of
    the convective, viscous, pressure and body terms
  * bubble-scale invariance of K*, R* (b -> c b, beta -> beta / c)
  * Stokes limit: the condensed pressure block equals the MINI element's
    -B^2 / (2 nu Kb) g_a . g_b (textbook static condensation of the bubble)
  * continuity rows sum to -|T| div(vbar) per element
"""
import numpy as np
import pytest

from oracle.element import element_residual_tangent
from oracle.vms import condense, assemble_vector, free_mask
from workloads import jittered_cube, boundary_nodes


def random_state(mesh, seed, beta_scale=0.3):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((mesh.n_nodes, 4))
    up = rng.standard_normal((mesh.n_nodes, 4))
    beta = beta_scale * rng.standard_normal((mesh.n_elems, 3))
    f = rng.standard_normal((mesh.n_nodes, 3))
    return u, up, beta, f


@pytest.fixture(scope="module")
def small_mesh():
    return jittered_cube(2, seed=7, amp=0.2)


def test_tangent_matches_central_differences(small_mesh):
    m = small_mesh
    u, up, beta, f = random_state(m, 1)
    nu, dt = 0.23, 0.05
    sel = [0, 5, 17, 30, 47]
    tets = m.tets[sel]
    _, K = element_residual_tangent(m.xyz, tets, u, beta[sel], nu, dt, up, f)
    h = 1e-6
    for k, e in enumerate(sel):
        for c in range(19):
            def res(s):
                uu, bb = u.copy(), beta[e:e + 1].copy()
                if c < 16:
                    uu[m.tets[e, c // 4], c % 4] += s
                else:
                    bb[0, c - 16] += s
                return element_residual_tangent(m.xyz, m.tets[e:e + 1], uu, bb, nu, dt, up, f,
                                                with_tangent=False)[0][0]
            fd = (res(h) - res(-h)) / (2 * h)
            assert np.max(np.abs(fd - K[k, :, c])) <= 1e-7 * np.max(np.abs(K[k])), (e, c)


# ---------------------------------------------------------------------------- closed form
def closed_form(X, U, Up, F, beta, nu, inv_dt):
    """Exact integration of the weak form on one tet via bubble moments."""
    J = (X[1:] - X[0]).T
    inv = np.linalg.inv(J)
    g = np.vstack([-inv.sum(axis=0), inv])
    vol = np.linalg.det(J) / 6.0
    I3 = np.eye(3)
    M = vol * (np.ones((4, 4)) + np.eye(4)) / 20.0
    B1, B, C = 8 * vol / 105, 32 * vol / 105, 8192 * vol / 51975
    Kb = 4096 / 945 * vol * np.sum(g * g)
    v, p = U[:, :3], U[:, 3]
    dv = v - Up[:, :3]
    G = v.T @ g
    th = np.trace(G)
    gp = g.T @ p
    V = M @ v
    Wv = B1 * v.sum(axis=0)
    R = np.zeros(19)
    K = np.zeros((19, 19))
    for a in range(4):
        R[4 * a:4 * a + 3] = (G @ V[a] + B1 * G @ beta - (g[a] @ Wv + th * B1) * beta
                              - 0.5 * C * (beta @ g[a]) * beta + 2 * nu * vol * G @ g[a]
                              - vol / 4 * p.sum() * g[a] - M[a] @ F + inv_dt * M[a] @ dv)
        R[4 * a + 3] = -th * vol / 4 + B * (beta @ g[a])
    R[16:] = (G @ Wv + C * (G - 0.5 * th * I3) @ beta + 2 * nu * Kb * beta + B * gp
              - B1 * F.sum(axis=0) + inv_dt * B1 * dv.sum(axis=0))
    for a in range(4):
        for b in range(4):
            s = g[b] @ V[a] + M[a, b] * inv_dt + 2 * nu * vol * g[a] @ g[b] + B1 * g[b] @ beta
            K[4 * a:4 * a + 3, 4 * b:4 * b + 3] = (s * I3 + M[a, b] * G
                                                   - np.outer(beta, B1 * g[a] + B1 * g[b]))
            K[4 * a:4 * a + 3, 4 * b + 3] = -vol / 4 * g[a]
            K[4 * a + 3, 4 * b:4 * b + 3] = -vol / 4 * g[b]
        K[4 * a:4 * a + 3, 16:] = (B1 * G - (g[a] @ Wv + th * B1) * I3
                                   - 0.5 * C * ((beta @ g[a]) * I3 + np.outer(beta, g[a])))
        K[4 * a + 3, 16:] = B * g[a]
        K[16:, 4 * a:4 * a + 3] = ((g[a] @ Wv) * I3 + B1 * G
                                   + C * ((g[a] @ beta) * I3 - 0.5 * np.outer(beta, g[a]))
                                   + B1 * inv_dt * I3)
        K[16:, 4 * a + 3] = B * g[a]
    K[16:, 16:] = C * (G - 0.5 * th * I3) + 2 * nu * Kb * I3
    return R, K


@pytest.mark.parametrize("transient", [False, True])
def test_matches_closed_form(small_mesh, transient):
    m = small_mesh
    u, up, beta, f = random_state(m, 2)
    nu, dt = 0.017, (0.01 if transient else 0.0)
    R, K = element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f)
    for e in range(m.n_elems):
        t = m.tets[e]
        Rc, Kc = closed_form(m.xyz[t], u[t], up[t], f[t], beta[e], nu, 1.0 / dt if transient else 0.0)
        assert np.max(np.abs(R[e] - Rc)) <= 1e-12 * np.max(np.abs(Rc))
        assert np.max(np.abs(K[e] - Kc)) <= 1e-12 * np.max(np.abs(Kc))


def test_patch_linear_solution_is_exact():
    m = jittered_cube(3, seed=11)
    rng = np.random.default_rng(5)
    Ag = rng.standard_normal((3, 3))
    Ag -= np.trace(Ag) / 3 * np.eye(3)                  # divergence free
    c = rng.standard_normal(3)
    q = rng.standard_normal(3)
    v = m.xyz @ Ag.T + c
    u = np.concatenate([v, (m.xyz @ q + 0.4)[:, None]], axis=1)
    f = v @ Ag.T + q                                    # (v.grad)v + grad p, linear
    beta = np.zeros((m.n_elems, 3))
    R, _ = element_residual_tangent(m.xyz, m.tets, u, beta, 0.31, 0.1, u, f, with_tangent=False)
    rc = assemble_vector(m.tets, m.n_nodes, R[:, :16]).reshape(-1, 4)
    interior = ~boundary_nodes(m.tets, m.n_nodes)
    scale = np.max(np.abs(R))
    assert np.max(np.abs(rc[interior])) <= 1e-12 * scale
    assert np.max(np.abs(rc[:, 3])) <= 1e-12 * scale    # every continuity row
    assert np.max(np.abs(R[:, 16:])) <= 1e-12 * scale   # every fine-scale row
    # a wrong sign on the pressure would leave a visible residual
    u_bad = u.copy()
    u_bad[:, 3] *= -1
    Rb, _ = element_residual_tangent(m.xyz, m.tets, u_bad, beta, 0.31, 0.1, u, f, with_tangent=False)
    rb = assemble_vector(m.tets, m.n_nodes, Rb[:, :16]).reshape(-1, 4)
    assert np.max(np.abs(rb[interior])) > 1e-3 * scale


def test_bubble_scale_invariance(small_mesh):
    m = small_mesh
    u, up, beta, f = random_state(m, 3)
    nu, dt = 0.05, 0.02
    R1, K1 = element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f, bubble_scale=1.0)
    R2, K2 = element_residual_tangent(m.xyz, m.tets, u, beta / 3.7, nu, dt, up, f,
                                      bubble_scale=3.7)
    Ks1, Rs1 = condense(R1, K1)
    Ks2, Rs2 = condense(R2, K2)
    assert np.max(np.abs(Ks1 - Ks2)) <= 1e-13 * np.max(np.abs(Ks1))
    assert np.max(np.abs(Rs1 - Rs2)) <= 1e-13 * np.max(np.abs(Rs1))


def test_stokes_limit_is_mini_condensation(small_mesh):
    m = small_mesh
    nu = 0.7
    u = np.zeros((m.n_nodes, 4))
    beta = np.zeros((m.n_elems, 3))
    R, K = element_residual_tangent(m.xyz, m.tets, u, beta, nu)
    Ks, _ = condense(R, K)
    for e in range(m.n_elems):
        X = m.xyz[m.tets[e]]
        J = (X[1:] - X[0]).T
        inv = np.linalg.inv(J)
        g = np.vstack([-inv.sum(axis=0), inv])
        vol = np.linalg.det(J) / 6
        B = 32 * vol / 105
        Kb = 4096 / 945 * vol * np.sum(g * g)
        kpp = -B * B / (2 * nu * Kb) * (g @ g.T)
        got = Ks[e][3::4, 3::4]
        assert np.allclose(got, kpp, rtol=1e-12, atol=1e-14 * np.abs(kpp).max())
        # viscous coarse/fine coupling vanishes for linear tets
        assert np.max(np.abs(K[e][:16, 16:][np.arange(16) % 4 != 3])) <= 1e-13 * np.abs(K[e]).max()
        # velocity-velocity block is untouched by the condensation in this limit
        vel = np.arange(16) % 4 != 3
        assert np.allclose(Ks[e][np.ix_(vel, vel)], K[e][:16, :16][np.ix_(vel, vel)], atol=1e-14)


def test_continuity_rows_sum_to_minus_divergence(small_mesh):
    m = small_mesh
    u, up, beta, f = random_state(m, 4)
    R, _ = element_residual_tangent(m.xyz, m.tets, u, beta, 0.1, with_tangent=False)
    for e in range(m.n_elems):
        X = m.xyz[m.tets[e]]
        J = (X[1:] - X[0]).T
        inv = np.linalg.inv(J)
        g = np.vstack([-inv.sum(axis=0), inv])
        vol = np.linalg.det(J) / 6
        div = np.trace(u[m.tets[e], :3].T @ g)
        assert np.isclose(R[e][3:16:4].sum(), -vol * div, rtol=1e-12, atol=1e-14)


def test_degenerate_element_is_reported():
    m = jittered_cube(2, seed=1)
    xyz = m.xyz.copy()
    t = m.tets[3]
    xyz[t[3]] = xyz[t[0]]           # collapse a vertex onto another
    with pytest.raises(ValueError, match="degenerate"):
        element_residual_tangent(xyz, m.tets, np.zeros((m.n_nodes, 4)),
                                 np.zeros((m.n_elems, 3)), 1.0)
