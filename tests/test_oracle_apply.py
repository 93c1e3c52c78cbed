"""Pins of the oracle's operator applies: the plain per-cell apply against explicit dense
matrices, and the ROM apply of eq. (romstiffnessmatrix) against its special cases."""
import numpy as np
import pytest

import lattice as L


@pytest.fixture(scope="module")
def hole(orc):
    cfg = L.config(0)
    keep = L.make_keep(cfg)
    l2g, nact, g2bg = orc.dofmap(2, cfg.ncell, cfg.nel, keep)
    uloc = orc.gather_local(L.make_displacement(cfg)[g2bg], l2g)
    mu, lam = L.make_material(cfg)
    ev = orc.cells_eval(2, cfg.nel, keep, uloc, mu, lam)
    X = L.make_rhs(cfg)
    return dict(cfg=cfg, keep=keep, l2g=l2g, uloc=uloc, mu=mu, lam=lam, T=ev["T"], X=X)


def _dense(orc, h, c):
    cfg = h["cfg"]
    return orc.cell_eval(2, cfg.nel, h["keep"][c], h["uloc"][c], h["mu"][c], h["lam"][c], dense=True)["K"]


def test_plain_apply_is_dense_product(orc, hole):
    cfg = hole["cfg"]
    Y = orc.plain_apply(2, cfg.nel, hole["T"], hole["l2g"], hole["X"])
    YT = orc.plain_apply(2, cfg.nel, hole["T"], hole["l2g"], hole["X"], transpose=True)
    for c in (0, 7, 15):
        K = _dense(orc, hole, c)
        m = np.repeat(hole["l2g"][c] >= 0, 2)
        x = hole["X"][c].reshape(-1, cfg.m) * m[:, None]
        y = (K @ x) * m[:, None]
        yt = (K.T @ x) * m[:, None]
        np.testing.assert_allclose(Y[c].reshape(-1, cfg.m), y, rtol=0, atol=1e-13 * np.abs(y).max())
        np.testing.assert_allclose(YT[c].reshape(-1, cfg.m), yt, rtol=0, atol=1e-13 * np.abs(y).max())


def test_combo_with_identity_alpha_is_plain(orc, hole):
    cfg = hole["cfg"]
    Ns = cfg.n_cells
    alpha = np.eye(Ns)
    Yc = orc.combo_apply(2, cfg.nel, hole["T"], alpha, hole["l2g"], hole["X"])
    Yp = orc.plain_apply(2, cfg.nel, hole["T"], hole["l2g"], hole["X"])
    np.testing.assert_array_equal(Yc, Yp)


def test_principal_cells_reproduce_themselves(orc, hole):
    cfg = hole["cfg"]
    g = orc.greedy(hole["T"], cfg.tol, cfg.cap)
    nr = g["n_r"]
    Kp = hole["T"][g["S"][:nr]]
    Yc = orc.combo_apply(2, cfg.nel, Kp, g["alpha"], hole["l2g"], hole["X"])
    Yp = orc.plain_apply(2, cfg.nel, hole["T"], hole["l2g"], hole["X"])
    for s in g["S"][:nr]:
        assert np.linalg.norm(Yc[s] - Yp[s]) <= 1e-12 * np.linalg.norm(Yp[s])
    # the ROM error is controlled by the greedy tolerance (snapshots are the full-rule tangents)
    rel = np.linalg.norm(Yc - Yp) / np.linalg.norm(Yp)
    assert rel < 1e-6


def test_combo_symmetry_and_linearity(orc, hole):
    cfg = hole["cfg"]
    rng = np.random.default_rng(1)
    nr = 5
    Kp = hole["T"][[1, 4, 9, 12, 14]]
    alpha = rng.standard_normal((cfg.n_cells, nr))
    X1 = hole["X"]
    X2 = L.make_rhs(cfg, stream=1)
    Y1 = orc.combo_apply(2, cfg.nel, Kp, alpha, hole["l2g"], X1)
    Y2 = orc.combo_apply(2, cfg.nel, Kp, alpha, hole["l2g"], X2)
    m = (hole["l2g"] >= 0)[:, :, None, None]
    lhs = np.sum(Y1 * X2 * m); rhs = np.sum(X1 * m * Y2)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(Y1 ** 2) * np.sum(X2 ** 2))
    Y12 = orc.combo_apply(2, cfg.nel, Kp, alpha, hole["l2g"], 2.0 * X1 - 3.0 * X2)
    np.testing.assert_allclose(Y12, 2.0 * Y1 - 3.0 * Y2, atol=1e-12 * np.abs(Y1).max())
    a2 = rng.standard_normal(alpha.shape)
    Ya = orc.combo_apply(2, cfg.nel, Kp, alpha + a2, hole["l2g"], X1)
    Yb = orc.combo_apply(2, cfg.nel, Kp, a2, hole["l2g"], X1)
    np.testing.assert_allclose(Ya, Y1 + Yb, atol=1e-12 * np.abs(Ya).max())


def test_combo_forms_are_alpha_derivatives(orc, hole):
    cfg = hole["cfg"]
    Kp = hole["T"][[0, 3, 5]]
    Ybar = L.make_rhs(cfg, stream=2)
    G = orc.combo_forms(2, cfg.nel, Kp, 4, hole["l2g"], hole["X"], Ybar)
    m = (hole["l2g"] >= 0)[:, :, None, None]
    for k in range(3):
        a = np.zeros((cfg.n_cells, 3)); a[:, k] = 1.0
        Yk = orc.combo_apply(2, cfg.nel, Kp, a, hole["l2g"], hole["X"])
        np.testing.assert_allclose(G[:, k], np.sum((Ybar * m * Yk).reshape(cfg.n_cells, -1), axis=1), rtol=1e-12)
    assert np.all(G[:, 3] == 0)
