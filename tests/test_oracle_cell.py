"""Pins of the oracle's cell operators: internal force (eq. internalloadvec), tangent
(Sec. 3.1.4, eq. fullquadraturerule), energy, and the stencil snapshot layout.

Each check uses something other than the oracle itself: closed forms for homogeneous
deformation, the divergence theorem, central finite differences, invariances, and the
textbook small-strain Q1 stiffness (Voigt B-matrix form, exact Gauss integration).
"""
import numpy as np
import pytest

import lattice as L


def _cell(dim, nel, seed=0, kind="hole", amp=0.02):
    rng = np.random.default_rng(seed)
    if dim == 2:
        ex, ey = np.meshgrid(np.arange(nel), np.arange(nel), indexing="xy")
        cen = np.stack([(ex.ravel() + 0.5) / nel, (ey.ravel() + 0.5) / nel], 1)
        keep = (np.linalg.norm(cen - 0.5, axis=1) > 0.3).astype(np.uint8)
    else:
        keep = (rng.random(nel ** 3) < 0.7).astype(np.uint8)
    nloc = (nel + 1) ** dim
    u = amp * rng.standard_normal((nloc, dim))
    return keep, u


def _node_coords(dim, nel):
    nn = nel + 1
    a = np.arange(nn ** dim)
    X = np.zeros((a.size, dim))
    for ax in range(dim):
        X[:, ax] = (a % nn) / nel
        a = a // nn
    return X


def _active(dim, nel, keep):
    nn = nel + 1
    act = np.zeros(nn ** dim, bool)
    for e in np.nonzero(keep)[0]:
        ie = [(e // nel ** ax) % nel for ax in range(dim)]
        for c in range(2 ** dim):
            a = sum((ie[ax] + ((c >> ax) & 1)) * nn ** ax for ax in range(dim))
            act[a] = True
    return act


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_homogeneous_energy_closed_form(orc, dim, nel):
    # u = (F - I) X: every Gauss point sees F, so Pi = W(F) * n_kept * h^d.
    keep, _ = _cell(dim, nel, seed=1)
    rng = np.random.default_rng(3)
    Fd = np.eye(dim) + 0.1 * rng.standard_normal((dim, dim))
    X = _node_coords(dim, nel)
    u = X @ (Fd - np.eye(dim)).T
    mu, lam = 1.3, 6.0
    r = orc.cell_eval(dim, nel, keep, u, mu, lam)
    F3 = np.eye(3); F3[:dim, :dim] = Fd
    J = np.linalg.det(F3)
    W = 0.5 * mu * (np.sum(F3 ** 2) - 3) - mu * np.log(J) + 0.5 * lam * np.log(J) ** 2
    assert abs(r["energy"] - W * keep.sum() / nel ** dim) < 1e-14 * abs(W) * keep.sum()


def test_homogeneous_force_divergence_theorem(orc):
    # For homogeneous F, f_a = P . (boundary integral of N_a n): zero at interior nodes,
    # P n h at a node in the middle of a straight boundary edge (2D).
    dim, nel = 2, 8
    keep = np.ones(nel * nel, np.uint8)
    Fd = np.array([[1.05, 0.02], [-0.01, 0.93]])
    X = _node_coords(dim, nel)
    u = X @ (Fd - np.eye(2)).T
    r = orc.cell_eval(dim, nel, keep, u, 1.0, 10.0)
    _, P, _ = orc.neo_hooke(np.block([[Fd, np.zeros((2, 1))], [np.zeros((1, 2)), np.ones((1, 1))]]), 1.0, 10.0)
    P = P[:2, :2]
    f = r["f"].reshape(nel + 1, nel + 1, 2)          # [iy][ix][i]
    h = 1.0 / nel
    assert np.abs(f[1:-1, 1:-1]).max() < 1e-14
    # right edge ix = nel (outward normal +x), interior of the edge
    tol = 1e-13 * np.abs(P).max() * h
    np.testing.assert_allclose(f[3, nel], P @ np.array([1.0, 0.0]) * h, rtol=0, atol=tol)
    # bottom edge iy = 0 (normal -y)
    np.testing.assert_allclose(f[0, 4], P @ np.array([0.0, -1.0]) * h, rtol=0, atol=tol)


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_zero_displacement_zero_force(orc, dim, nel):
    keep, u = _cell(dim, nel)
    r = orc.cell_eval(dim, nel, keep, np.zeros_like(u), 1.0, 5.0)
    assert r["energy"] == 0.0
    assert np.abs(r["f"]).max() == 0.0


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_force_is_energy_gradient_and_tangent_is_force_jacobian(orc, dim, nel):
    keep, u = _cell(dim, nel, seed=5)
    mu, lam = 1.0, 5.0
    r = orc.cell_eval(dim, nel, keep, u, mu, lam, dense=True)
    act = _active(dim, nel, keep)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(u.shape) * act[:, None]
    h = 1e-6
    rp = orc.cell_eval(dim, nel, keep, u + h * v, mu, lam)
    rm = orc.cell_eval(dim, nel, keep, u - h * v, mu, lam)
    dE = (rp["energy"] - rm["energy"]) / (2 * h)
    assert abs(dE - np.sum(r["f"] * v)) <= 1e-7 * abs(dE)
    Kv = r["K"] @ v.ravel()
    fd = ((rp["f"] - rm["f"]) / (2 * h)).ravel()
    assert np.linalg.norm(Kv - fd) <= 1e-7 * np.linalg.norm(Kv)


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_tangent_symmetric_and_translations_in_kernel(orc, dim, nel):
    keep, u = _cell(dim, nel, seed=9, amp=0.05)
    r = orc.cell_eval(dim, nel, keep, u, 1.0, 5.0, dense=True)
    K = r["K"]
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    act = _active(dim, nel, keep)
    for ax in range(dim):
        t = np.zeros(u.shape); t[act, ax] = 1.0
        assert np.abs(K @ t.ravel()).max() <= 1e-13 * np.abs(K).max()


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_rotations_in_kernel_at_reference(orc, dim, nel):
    keep, u = _cell(dim, nel)
    r = orc.cell_eval(dim, nel, keep, np.zeros_like(u), 1.0, 5.0, dense=True)
    K = r["K"]
    X = _node_coords(dim, nel)
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for (p, q) in pairs:
        w = np.zeros_like(u)
        w[:, p] = -X[:, q]; w[:, q] = X[:, p]
        assert np.abs(K @ w.ravel()).max() <= 1e-13 * np.abs(K).max()


def test_frame_invariance(orc):
    # x -> Q x (rigid rotation of the deformed configuration): energy unchanged, f -> Q f.
    dim, nel = 2, 6
    keep, u = _cell(dim, nel, seed=11, amp=0.05)
    X = _node_coords(dim, nel)
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    x = X + u
    u2 = x @ Q.T - X
    r1 = orc.cell_eval(dim, nel, keep, u, 1.0, 10.0)
    r2 = orc.cell_eval(dim, nel, keep, u2, 1.0, 10.0)
    assert abs(r1["energy"] - r2["energy"]) <= 1e-12 * abs(r1["energy"])
    np.testing.assert_allclose(r2["f"], r1["f"] @ Q.T, atol=1e-12 * np.abs(r1["f"]).max())


def _textbook_q1_stiffness(dim, h, mu, lam):
    """Small-strain Q1 element stiffness K = int B^T D B over the element (Voigt B-matrix form,
    isotropic Hooke D), integrated with a 4-point Gauss-Legendre rule per axis, which is exact
    for this polynomial integrand."""
    xg, wg = np.polynomial.legendre.leggauss(4)
    xg = 0.5 * h * (xg + 1.0); wg = 0.5 * h * wg
    nstr = 3 if dim == 2 else 6
    D = np.zeros((nstr, nstr))
    D[:dim, :dim] = lam
    for i in range(dim):
        D[i, i] += 2 * mu
    for k in range(dim, nstr):
        D[k, k] = mu
    nc = 2 ** dim
    K = np.zeros((dim * nc, dim * nc))
    import itertools
    for idx in itertools.product(range(4), repeat=dim):
        x = np.array([xg[i] for i in idx]); w = np.prod([wg[i] for i in idx])
        B = np.zeros((nstr, dim * nc))
        for a in range(nc):
            bits = [(a >> ax) & 1 for ax in range(dim)]
            g = np.zeros(dim)
            for ax in range(dim):
                v = 1.0
                for bx in range(dim):
                    if bx == ax:
                        v *= (1.0 / h) if bits[bx] else (-1.0 / h)
                    else:
                        v *= (x[bx] / h) if bits[bx] else (1 - x[bx] / h)
                g[ax] = v
            if dim == 2:
                B[0, 2 * a] = g[0]; B[1, 2 * a + 1] = g[1]; B[2, 2 * a] = g[1]; B[2, 2 * a + 1] = g[0]
            else:
                for ax in range(3):
                    B[ax, 3 * a + ax] = g[ax]
                B[3, 3 * a + 1] = g[2]; B[3, 3 * a + 2] = g[1]
                B[4, 3 * a + 0] = g[2]; B[4, 3 * a + 2] = g[0]
                B[5, 3 * a + 0] = g[1]; B[5, 3 * a + 1] = g[0]
        K += w * B.T @ D @ B
    return K


@pytest.mark.parametrize("dim", [2, 3])
def test_reference_tangent_is_textbook_linear_elasticity(orc, dim):
    # At u = 0 the tangent reduces to isotropic Hooke (ln 1 = 0, sigma = 0): one element equals
    # the classical small-strain Q1 stiffness (plane strain in 2D).
    nel = 1
    mu, lam = 1.0, 10.0 if dim == 2 else 5.0
    keep = np.ones(1, np.uint8)
    r = orc.cell_eval(dim, nel, keep, np.zeros((2 ** dim, dim)), mu, lam, dense=True)
    Kt = _textbook_q1_stiffness(dim, 1.0, mu, lam)
    np.testing.assert_allclose(r["K"], Kt, atol=1e-13 * np.abs(Kt).max())


def test_stencil_matches_dense(orc):
    dim, nel = 2, 5
    keep, u = _cell(dim, nel, seed=13)
    r = orc.cell_eval(dim, nel, keep, u, 1.0, 10.0, dense=True)
    nn = nel + 1
    st = r["stencil"].reshape(nn ** 2, 9, 2, 2)
    K = r["K"]
    for a in range(nn ** 2):
        ia = (a % nn, a // nn)
        for o in range(9):
            ib = (ia[0] + o % 3 - 1, ia[1] + o // 3 - 1)
            if not (0 <= ib[0] < nn and 0 <= ib[1] < nn):
                assert np.all(st[a, o] == 0)
                continue
            b = ib[0] + nn * ib[1]
            np.testing.assert_array_equal(st[a, o], K[2 * a:2 * a + 2, 2 * b:2 * b + 2])


def test_inverted_element_flagged(orc):
    dim, nel = 2, 4
    keep = np.ones(nel * nel, np.uint8)
    X = _node_coords(dim, nel)
    u = np.zeros_like(X)
    u[:, 0] = -2.0 * X[:, 0]                          # F_xx = -1 -> J < 0
    r = orc.cell_eval(dim, nel, keep, u, 1.0, 1.0)
    assert r["status"] == orc.E_INVERTED


def test_workload_cells_converge_under_fd(orc):
    # a cell of the 4x4 hole workload: tangent-vs-residual FD at h = 1e-6
    cfg = L.config(0)
    keep = L.make_keep(cfg)
    l2g, nact, g2bg = orc.dofmap(2, cfg.ncell, cfg.nel, keep)
    uloc = orc.gather_local(L.make_displacement(cfg)[g2bg], l2g)
    c = 5
    r = orc.cell_eval(2, cfg.nel, keep[c], uloc[c], 1.0, 10.0, dense=True)
    v = np.random.default_rng(1).standard_normal(uloc[c].shape) * (l2g[c] >= 0)[:, None]
    h = 1e-6
    fp = orc.cell_eval(2, cfg.nel, keep[c], uloc[c] + h * v, 1.0, 10.0)["f"]
    fm = orc.cell_eval(2, cfg.nel, keep[c], uloc[c] - h * v, 1.0, 10.0)["f"]
    Kv = r["K"] @ v.ravel()
    assert np.linalg.norm(Kv - ((fp - fm) / (2 * h)).ravel()) <= 1e-7 * np.linalg.norm(Kv)


# ---------------------------------------------------------------------------------------------
# One-point (reduced) quadrature, the snapshot rule with fewer points per direction of
# eq. (snapshots): one point at the element centre with weight 1 (times h^d).  Pinned without
# the oracle's own formulas: the weight by closed forms that hold for any point, the point by
# the textbook centroid B-matrix stiffness and by the centroid stress written out here, the
# tangent's consistency by finite differences of the one-point force, and the rank deficiency
# (hourglass modes) that every one-point Q1 element has.
def _centroid_grads(dim, h):
    """g_c = grad_X N_c at the element centre: the axis factor is -+1/h, the others 1/2."""
    nc = 2 ** dim
    g = np.zeros((nc, dim))
    for c in range(nc):
        for ax in range(dim):
            g[c, ax] = (1.0 if (c >> ax) & 1 else -1.0) / h * 0.5 ** (dim - 1)
    return g


def _piola(F3, mu, lam):
    Fit = np.linalg.inv(F3).T
    lnJ = np.log(np.linalg.det(F3))
    return mu * (F3 - Fit) + lam * lnJ * Fit


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_reduced_rule_homogeneous_energy_closed_form(orc, dim, nel):
    # homogeneous F: the one point sees F, so Pi = W(F) n_kept h^d -- fixes the weight (1)
    keep, _ = _cell(dim, nel, seed=21)
    rng = np.random.default_rng(23)
    Fd = np.eye(dim) + 0.1 * rng.standard_normal((dim, dim))
    u = _node_coords(dim, nel) @ (Fd - np.eye(dim)).T
    mu, lam = 0.9, 4.0
    r = orc.cell_eval(dim, nel, keep, u, mu, lam, rule=orc.RULE_REDUCED)
    F3 = np.eye(3); F3[:dim, :dim] = Fd
    J = np.linalg.det(F3)
    W = 0.5 * mu * (np.sum(F3 ** 2) - 3) - mu * np.log(J) + 0.5 * lam * np.log(J) ** 2
    assert abs(r["energy"] - W * keep.sum() / nel ** dim) < 1e-14 * abs(W) * keep.sum()


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_reduced_rule_affine_force_equals_full_rule(orc, dim, nel):
    # affine u: P is constant and the corner gradients are linear in the other coordinates, so
    # one centre point integrates P g_a exactly -- equal to the 2^d-point force
    keep, _ = _cell(dim, nel, seed=25)
    rng = np.random.default_rng(27)
    Fd = np.eye(dim) + 0.08 * rng.standard_normal((dim, dim))
    u = _node_coords(dim, nel) @ (Fd - np.eye(dim)).T + 0.01
    r1 = orc.cell_eval(dim, nel, keep, u, 1.0, 5.0, rule=orc.RULE_REDUCED)
    r2 = orc.cell_eval(dim, nel, keep, u, 1.0, 5.0, rule=orc.RULE_FULL)
    np.testing.assert_allclose(r1["f"], r2["f"], rtol=0, atol=1e-13 * np.abs(r2["f"]).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_reduced_rule_reference_tangent_is_centroid_B_matrix(orc, dim):
    # u = 0: one-point stiffness = h^d B(centroid)^T D B(centroid), D isotropic Hooke
    nel = 1
    h = 1.0
    mu, lam = 1.0, 10.0 if dim == 2 else 5.0
    r = orc.cell_eval(dim, nel, np.ones(1, np.uint8), np.zeros((2 ** dim, dim)), mu, lam, rule=orc.RULE_REDUCED,
                      dense=True)
    g = _centroid_grads(dim, h)
    nstr = 3 if dim == 2 else 6
    D = np.zeros((nstr, nstr))
    D[:dim, :dim] = lam
    for i in range(dim):
        D[i, i] += 2 * mu
    for k in range(dim, nstr):
        D[k, k] = mu
    B = np.zeros((nstr, dim * 2 ** dim))
    for a in range(2 ** dim):
        if dim == 2:
            B[0, 2 * a] = g[a, 0]; B[1, 2 * a + 1] = g[a, 1]; B[2, 2 * a] = g[a, 1]; B[2, 2 * a + 1] = g[a, 0]
        else:
            for ax in range(3):
                B[ax, 3 * a + ax] = g[a, ax]
            B[3, 3 * a + 1] = g[a, 2]; B[3, 3 * a + 2] = g[a, 1]
            B[4, 3 * a + 0] = g[a, 2]; B[4, 3 * a + 2] = g[a, 0]
            B[5, 3 * a + 0] = g[a, 1]; B[5, 3 * a + 1] = g[a, 0]
    Kt = h ** dim * B.T @ D @ B
    np.testing.assert_allclose(r["K"], Kt, atol=1e-13 * np.abs(Kt).max())
    # one point leaves the hourglass modes in the kernel: rank = (3 or 6) strain components
    sv = np.linalg.svd(r["K"], compute_uv=False)
    assert int(np.sum(sv > 1e-12 * sv[0])) == nstr


@pytest.mark.parametrize("dim", [2, 3])
def test_reduced_rule_force_is_centroid_stress(orc, dim):
    # one element, non-affine u: f_c = h^d P(F(centroid)) g_c(centroid)
    nel = 1
    h = 1.0
    rng = np.random.default_rng(29)
    u = 0.05 * rng.standard_normal((2 ** dim, dim))
    mu, lam = 1.2, 3.0
    r = orc.cell_eval(dim, nel, np.ones(1, np.uint8), u, mu, lam, rule=orc.RULE_REDUCED)
    g = _centroid_grads(dim, h)
    F3 = np.eye(3)
    F3[:dim, :dim] += u.T @ g
    P = _piola(F3, mu, lam)[:dim, :dim]
    f = h ** dim * g @ P.T                      # f[c, i] = sum_J P_iJ g_cJ
    np.testing.assert_allclose(r["f"], f, rtol=0, atol=1e-14 * np.abs(f).max())


@pytest.mark.parametrize("dim,nel", [(2, 5), (3, 3)])
def test_reduced_rule_tangent_is_force_jacobian(orc, dim, nel):
    keep, u = _cell(dim, nel, seed=31)
    mu, lam = 1.0, 5.0
    R = orc.RULE_REDUCED
    r = orc.cell_eval(dim, nel, keep, u, mu, lam, rule=R, dense=True)
    act = _active(dim, nel, keep)
    v = np.random.default_rng(33).standard_normal(u.shape) * act[:, None]
    h = 1e-6
    fp = orc.cell_eval(dim, nel, keep, u + h * v, mu, lam, rule=R)["f"]
    fm = orc.cell_eval(dim, nel, keep, u - h * v, mu, lam, rule=R)["f"]
    Kv = r["K"] @ v.ravel()
    assert np.linalg.norm(Kv - ((fp - fm) / (2 * h)).ravel()) <= 1e-7 * np.linalg.norm(Kv)
    # and the one-point tangent is not the full-rule one (the rule is really in use)
    rf = orc.cell_eval(dim, nel, keep, u, mu, lam, rule=orc.RULE_FULL, dense=True)
    assert np.linalg.norm(rf["K"] - r["K"]) > 1e-3 * np.linalg.norm(rf["K"])
