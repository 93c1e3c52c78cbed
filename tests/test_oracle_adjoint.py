"""Pins of the oracle's adjoint pieces (reverse mode of the residual and of the ROM apply
with respect to the applied vectors and the per-cell Lame parameters, the principal set
frozen).  Checked by central finite differences and by the closed-form scaling law that
holds when lam is a fixed multiple of mu (then every tangent is mu_i times a mu-free
tangent, the greedy selection is unchanged and Ktilde_i scales with mu_i alone)."""
import numpy as np
import pytest

import lattice as L


def test_alpha_ls_adjoint_fd(orc):
    rng = np.random.default_rng(0)
    Ns, n, nr = 7, 40, 3
    T = rng.standard_normal((Ns, n))
    S = [1, 4, 5]
    abar = rng.standard_normal((Ns, nr))

    def alpha_of(Tall):
        TS = Tall[S].T
        return np.linalg.lstsq(TS, Tall.T, rcond=None)[0].T

    alpha = alpha_of(T)
    tbar, TbarS = orc.alpha_ls_adjoint(T[S].T, T, alpha, abar)
    # total cotangent of every snapshot: as data (tbar) plus, for principals, as a basis column
    grad = tbar.copy()
    for k, s in enumerate(S):
        grad[s] += TbarS[:, k]
    dT = rng.standard_normal(T.shape)
    h = 1e-6
    fd = (np.sum(abar * alpha_of(T + h * dT)) - np.sum(abar * alpha_of(T - h * dT))) / (2 * h)
    assert abs(fd - np.sum(grad * dT)) <= 1e-7 * abs(fd)


def test_residual_linear_in_lame_and_adjoint(orc):
    cfg = L.config(3).with_sub((2, 2, 1))
    keep = L.make_keep(cfg)
    l2g, _, g2bg = orc.dofmap(3, cfg.ncell_eff, cfg.nel, keep)
    uloc = orc.gather_local(L.make_displacement(cfg)[g2bg], l2g)
    mu, lam = L.make_material(cfg)
    Ns = cfg.n_cells
    r = orc.cells_eval(3, cfg.nel, keep, uloc, mu, lam)
    rm = orc.cells_eval(3, cfg.nel, keep, uloc, np.ones(Ns), np.zeros(Ns))
    rl = orc.cells_eval(3, cfg.nel, keep, uloc, np.zeros(Ns), np.ones(Ns))
    f_lin = mu[:, None, None] * rm["f"] + lam[:, None, None] * rl["f"]
    np.testing.assert_allclose(r["f"], f_lin, atol=1e-13 * np.abs(r["f"]).max())
    T_lin = mu[:, None] * rm["T"] + lam[:, None] * rl["T"]
    np.testing.assert_allclose(r["T"], T_lin, atol=1e-13 * np.abs(r["T"]).max())
    # reverse mode of phi = <w, f(u)>: ubar_i = K_i^T w_i, mubar_i = <w_i, f_i^mu>; check by FD
    rng = np.random.default_rng(2)
    w = rng.standard_normal(uloc.shape) * (l2g >= 0)[:, :, None]
    c = 1
    ub = orc.stencil_apply(3, cfg.nel, r["T"][c], l2g[c], w[c][:, :, None], transpose=True)[:, :, 0]
    v = rng.standard_normal(uloc[c].shape) * (l2g[c] >= 0)[:, None]
    h = 1e-6
    fp = orc.cell_eval(3, cfg.nel, keep[c], uloc[c] + h * v, mu[c], lam[c])["f"]
    fm = orc.cell_eval(3, cfg.nel, keep[c], uloc[c] - h * v, mu[c], lam[c])["f"]
    fd = np.sum(w[c] * (fp - fm)) / (2 * h)
    assert abs(fd - np.sum(ub * v)) <= 1e-7 * abs(fd)
    fp = orc.cell_eval(3, cfg.nel, keep[c], uloc[c], mu[c] + h, lam[c])["f"]
    fm = orc.cell_eval(3, cfg.nel, keep[c], uloc[c], mu[c] - h, lam[c])["f"]
    fd = np.sum(w[c] * (fp - fm)) / (2 * h)
    assert abs(fd - np.sum(w[c] * rm["f"][c])) <= 1e-7 * abs(fd)


@pytest.fixture(scope="module")
def logmu(orc):
    """A 2x2x1 slice of the log-uniform-mu BCC lattice (lam = 5 mu), m = 1."""
    cfg = L.config(3).with_sub((2, 2, 1))
    keep = L.make_keep(cfg)
    l2g, _, g2bg = orc.dofmap(3, cfg.ncell_eff, cfg.nel, keep)
    uloc = orc.gather_local(L.make_displacement(cfg)[g2bg], l2g)
    mu, lam = L.make_material(cfg)
    X = L.make_rhs(cfg, m=1)
    return dict(cfg=cfg, keep=keep, l2g=l2g, uloc=uloc, mu=mu, lam=lam, X=X)


def _objective(orc, d, mu, lam, S=None, tol=1e-8, cap=4):
    """J = sum_i X_i^T Ktilde_i X_i with Ktilde from the greedy (S frozen when given)."""
    cfg = d["cfg"]
    T = orc.cells_eval(3, cfg.nel, d["keep"], d["uloc"], mu, lam, want_f=False, want_energy=False)["T"]
    if S is None:
        g = orc.greedy(T, tol, cap)
        S = list(g["S"][:g["n_r"]])
    alpha = np.linalg.lstsq(T[S].T, T.T, rcond=None)[0].T
    Y = orc.combo_apply(3, cfg.nel, T[S], alpha, d["l2g"], d["X"])
    return float(np.sum(Y * d["X"])), S, T, alpha


def _gradient(orc, d, S, T, alpha):
    """Reverse mode assembled from oracle pieces: direct dependence through the principal
    tangents plus the dependence through alpha (least squares, S frozen)."""
    cfg = d["cfg"]
    Ns = cfg.n_cells
    ones, zeros = np.ones(Ns), np.zeros(Ns)
    Tm = orc.cells_eval(3, cfg.nel, d["keep"], d["uloc"], ones, zeros, want_f=False, want_energy=False)["T"]
    Tl = orc.cells_eval(3, cfg.nel, d["keep"], d["uloc"], zeros, ones, want_f=False, want_energy=False)["T"]
    nr = len(S)
    Ybar = d["X"]                                            # J = <X, Y(X)>
    abar = orc.combo_forms(3, cfg.nel, T[S], nr, d["l2g"], d["X"], Ybar)
    Gm = orc.combo_forms(3, cfg.nel, Tm[S], nr, d["l2g"], d["X"], Ybar)
    Gl = orc.combo_forms(3, cfg.nel, Tl[S], nr, d["l2g"], d["X"], Ybar)
    mubar = np.zeros(Ns); lambar = np.zeros(Ns)
    for k, s in enumerate(S):
        mubar[s] += np.sum(alpha[:, k] * Gm[:, k])
        lambar[s] += np.sum(alpha[:, k] * Gl[:, k])
    tbar, TbarS = orc.alpha_ls_adjoint(T[S].T, T, alpha, abar)
    mubar += np.sum(tbar * Tm, axis=1)
    lambar += np.sum(tbar * Tl, axis=1)
    for k, s in enumerate(S):
        mubar[s] += TbarS[:, k] @ Tm[s]
        lambar[s] += TbarS[:, k] @ Tl[s]
    return mubar, lambar


def test_combo_gradient_fd_and_scaling_law(orc, logmu):
    d = logmu
    J, S, T, alpha = _objective(orc, d, d["mu"], d["lam"])
    mubar, lambar = _gradient(orc, d, S, T, alpha)
    g = mubar + 5.0 * lambar                                   # lam = 5 mu
    # scaling law: Ktilde_i = mu_i * (mu-free ROM tangent), so dJ/dmu_i = J_i / mu_i
    Y = orc.combo_apply(3, d["cfg"].nel, T[S], alpha, d["l2g"], d["X"])
    Ji = np.sum((Y * d["X"]).reshape(d["cfg"].n_cells, -1), axis=1)
    np.testing.assert_allclose(g, Ji / d["mu"], rtol=1e-7)
    # central finite differences, h = 1e-6, S frozen
    h = 1e-6
    for c in range(d["cfg"].n_cells):
        mp = d["mu"].copy(); mp[c] += h
        mm = d["mu"].copy(); mm[c] -= h
        Jp = _objective(orc, d, mp, 5 * mp, S=S)[0]
        Jm = _objective(orc, d, mm, 5 * mm, S=S)[0]
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g[c]) <= 1e-6 * abs(fd)
