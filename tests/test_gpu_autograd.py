"""torch.autograd through the hand-written adjoints.

LatCombo (ROM apply): compliance-type objective J = <X, Y(X)> on the log-uniform-mu BCC
lattice (lam = 5 mu, one right-hand side); dJ/dmu against (i) the closed-form scaling law
dJ/dmu_i = J_i / mu_i (every tangent is mu_i times a mu-free tangent, so the ROM tangent
scales with mu_i alone), (ii) the oracle's gradient assembled from its own pieces, and
(iii) central finite differences (h = 1e-6, principal set frozen) on the oracle.
LatResidual: gradients of <v, r(u)> in u, mu, lam against central finite differences of the
GPU residual itself and the oracle's adjoint.
"""
import numpy as np
import pytest
import torch

import lattice as L
import oracle as O
from gpu_common import Case, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def logmu():
    return Case(L.config(3).with_sub((3, 3, 2)), m=1)


def test_combo_lame_gradient(logmu):
    from paper_2603_10741_amd import autograd as AG
    c = logmu
    P, cfg = c.P, c.cfg
    st = AG.build_rom_state(P, c.ug, c.mu_t, c.lam_t, cfg.tol)
    X, Xp = c.rhs(m=1)
    mu = c.mu_t.clone().requires_grad_(True)
    lam = 5.0 * mu
    Y = AG.rom_apply(Xp, mu, lam, st, 1)
    J = torch.sum(Y * Xp)
    J.backward()
    g = mu.grad.cpu().numpy()
    # (i) scaling law
    Ji = np.sum((c.unpack(Y.detach(), 1) * c.masked(X)).reshape(cfg.n_cells, -1), axis=1)
    np.testing.assert_allclose(g, Ji / c.mu, rtol=1e-8, atol=1e-12 * np.abs(Ji / c.mu).max())
    # (ii) the oracle's gradient from its own pieces (same principal cells)
    S = st.S.cpu().numpy()[:st.n_r]
    T = c.orc["T"]
    alpha = np.linalg.lstsq(T[S].T, T.T, rcond=None)[0].T
    Ns = cfg.n_cells
    Tm = O.cells_eval(3, cfg.nel, c.keep, c.uloc, np.ones(Ns), np.zeros(Ns), want_f=False, want_energy=False)["T"]
    Tl = O.cells_eval(3, cfg.nel, c.keep, c.uloc, np.zeros(Ns), np.ones(Ns), want_f=False, want_energy=False)["T"]
    nr = len(S)
    abar = O.combo_forms(3, cfg.nel, T[S], nr, c.l2g, X, X)
    Gm = O.combo_forms(3, cfg.nel, Tm[S], nr, c.l2g, X, X)
    Gl = O.combo_forms(3, cfg.nel, Tl[S], nr, c.l2g, X, X)
    mub = np.zeros(Ns); lamb = np.zeros(Ns)
    for k, s in enumerate(S):
        mub[s] += np.sum(alpha[:, k] * Gm[:, k]); lamb[s] += np.sum(alpha[:, k] * Gl[:, k])
    tbar, TbarS = O.alpha_ls_adjoint(T[S].T, T, alpha, abar)
    mub += np.sum(tbar * Tm, axis=1); lamb += np.sum(tbar * Tl, axis=1)
    for k, s in enumerate(S):
        mub[s] += TbarS[:, k] @ Tm[s]; lamb[s] += TbarS[:, k] @ Tl[s]
    go = mub + 5.0 * lamb
    assert rel(g, go) <= 1e-8
    # (iii) central finite differences on the oracle, principal set frozen
    h = 1e-6
    for cell in (0, 7, 13):
        vals = []
        for sgn in (1, -1):
            mu2 = c.mu.copy(); mu2[cell] += sgn * h
            T2 = O.cells_eval(3, cfg.nel, c.keep, c.uloc, mu2, 5 * mu2, want_f=False, want_energy=False)["T"]
            a2 = np.linalg.lstsq(T2[S].T, T2.T, rcond=None)[0].T
            Y2 = O.combo_apply(3, cfg.nel, T2[S], a2, c.l2g, X)
            vals.append(np.sum(Y2 * c.masked(X)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[cell]) <= 1e-6 * abs(fd)


@pytest.mark.timeout(600)
def test_combo_lame_gradient_full_lattice():
    # the full 8^3 log-uniform-mu lattice (512 cells, 12^3 hexes, cap 64): dJ/dmu of J = <X, Y(X)>
    # against the scaling law on every cell, the oracle's assembled gradient on every cell, and
    # central differences (h = 1e-6, principal set frozen) on two ordinary cells and one principal
    from paper_2603_10741_amd import autograd as AG
    c = Case(L.config(3), m=1)
    P, cfg = c.P, c.cfg
    st = AG.build_rom_state(P, c.ug, c.mu_t, c.lam_t, cfg.tol)
    X, Xp = c.rhs(m=1)
    mu = c.mu_t.clone().requires_grad_(True)
    Y = AG.rom_apply(Xp, mu, 5.0 * mu, st, 1)
    J = torch.sum(Y * Xp)
    J.backward()
    g = mu.grad.cpu().numpy()
    Ns = cfg.n_cells
    Xm = c.masked(X)
    Ji = np.sum((c.unpack(Y.detach(), 1) * Xm).reshape(Ns, -1), axis=1)
    np.testing.assert_allclose(g, Ji / c.mu, rtol=1e-8, atol=1e-12 * np.abs(Ji / c.mu).max())
    S = st.S.cpu().numpy()[:st.n_r]
    T = c.orc["T"]
    alpha = np.linalg.lstsq(T[S].T, T.T, rcond=None)[0].T
    Tm = O.cells_eval(3, cfg.nel, c.keep, c.uloc, np.ones(Ns), np.zeros(Ns), want_f=False, want_energy=False)["T"]
    Tl = O.cells_eval(3, cfg.nel, c.keep, c.uloc, np.zeros(Ns), np.ones(Ns), want_f=False, want_energy=False)["T"]
    nr = len(S)
    abar = O.combo_forms(3, cfg.nel, T[S], nr, c.l2g, X, X)
    Gm = O.combo_forms(3, cfg.nel, Tm[S], nr, c.l2g, X, X)
    Gl = O.combo_forms(3, cfg.nel, Tl[S], nr, c.l2g, X, X)
    mub = np.zeros(Ns); lamb = np.zeros(Ns)
    for k, s_ in enumerate(S):
        mub[s_] += np.sum(alpha[:, k] * Gm[:, k]); lamb[s_] += np.sum(alpha[:, k] * Gl[:, k])
    tbar, TbarS = O.alpha_ls_adjoint(T[S].T, T, alpha, abar)
    mub += np.sum(tbar * Tm, axis=1); lamb += np.sum(tbar * Tl, axis=1)
    for k, s_ in enumerate(S):
        mub[s_] += TbarS[:, k] @ Tm[s_]; lamb[s_] += TbarS[:, k] @ Tl[s_]
    go = mub + 5.0 * lamb
    assert rel(g, go) <= 1e-8
    del Tm, Tl
    h = 1e-6
    ordinary = [int(x) for x in np.setdiff1d(np.arange(Ns), S)[[3, 200]]]
    for cell in ordinary + [int(S[1])]:
        vals = []
        for sgn in (1, -1):
            mu2 = c.mu.copy(); mu2[cell] += sgn * h
            T2 = T.copy()
            T2[cell] = O.cell_eval(3, cfg.nel, c.keep[cell], c.uloc[cell], mu2[cell], 5 * mu2[cell])["stencil"]
            if cell in S:
                a2 = np.linalg.lstsq(T2[S].T, T2.T, rcond=None)[0].T
                Y2 = O.combo_apply(3, cfg.nel, T2[S], a2, c.l2g, X)
                vals.append(np.sum(Y2 * Xm))
            else:
                a2 = np.linalg.lstsq(T2[S].T, T2[cell], rcond=None)[0]
                Y2 = O.combo_apply(3, cfg.nel, T2[S], a2[None, :], c.l2g[[cell]], X[[cell]])
                vals.append(np.sum(Y2 * Xm[[cell]]))
        fd = (vals[0] - vals[1]) / (2 * h)
        print(f"[autograd] full 8^3 cell {cell} (principal {cell in S}): fd {fd:.6e} gpu {g[cell]:.6e}", flush=True)
        assert abs(fd - g[cell]) <= 1e-6 * abs(fd)


def test_combo_input_gradient_is_transpose(logmu):
    from paper_2603_10741_amd import autograd as AG
    c = logmu
    st = AG.build_rom_state(c.P, c.ug, c.mu_t, c.lam_t, c.cfg.tol, for_adjoint=False)
    X, Xp = c.rhs(m=1)
    Yb, Ybp = c.rhs(stream=3, m=1)
    Xv = Xp.clone().requires_grad_(True)
    Y = AG.rom_apply(Xv, c.mu_t, c.lam_t, st, 1)
    torch.sum(Y * Ybp).backward()
    Xb = c.unpack(Xv.grad, 1)
    S = st.S.cpu().numpy()[:st.n_r]
    Xbo = O.combo_apply(3, c.nel, c.orc["T"][S], st.alpha.cpu().numpy(), c.l2g, Yb, transpose=True)
    assert rel(Xb, Xbo) <= 1e-10


def test_residual_gradients(logmu):
    from paper_2603_10741_amd import autograd as AG
    c = logmu
    P = c.P
    rng = np.random.default_rng(4)
    v = torch.from_numpy(rng.standard_normal((P.nglobal, 3))).to(c.dev)
    u = c.ug.clone().requires_grad_(True)
    mu = c.mu_t.clone().requires_grad_(True)
    lam = c.lam_t.clone().requires_grad_(True)
    r = AG.residual(u, mu, lam, P)
    torch.sum(r * v).backward()
    # oracle adjoint: ubar = sum_s A^s K_s^T A^{sT} v
    w = O.gather_local(v.cpu().numpy(), c.l2g)
    ub = np.zeros_like(w)
    for cell in range(c.cfg.n_cells):
        ub[cell] = O.stencil_apply(3, c.nel, c.orc["T"][cell], c.l2g[cell], w[cell][:, :, None], transpose=True)[:, :, 0]
    ubo = O.assemble(ub, c.l2g, P.nglobal)
    assert rel(u.grad.cpu().numpy(), ubo) <= 1e-10
    # central differences of the GPU residual itself (h = 1e-6)
    h = 1e-6
    d = torch.from_numpy(rng.standard_normal((P.nglobal, 3))).to(c.dev)
    with torch.no_grad():
        fp = torch.sum(AG.residual(c.ug + h * d, c.mu_t, c.lam_t, P) * v).item()
        fm = torch.sum(AG.residual(c.ug - h * d, c.mu_t, c.lam_t, P) * v).item()
    fd = (fp - fm) / (2 * h)
    assert abs(fd - torch.sum(u.grad * d).item()) <= 1e-6 * abs(fd)
    for cell in (2, 11):
        e = torch.zeros_like(c.mu_t); e[cell] = h
        with torch.no_grad():
            fdm = (torch.sum(AG.residual(c.ug, c.mu_t + e, c.lam_t, P) * v).item()
                   - torch.sum(AG.residual(c.ug, c.mu_t - e, c.lam_t, P) * v).item()) / (2 * h)
            fdl = (torch.sum(AG.residual(c.ug, c.mu_t, c.lam_t + e, P) * v).item()
                   - torch.sum(AG.residual(c.ug, c.mu_t, c.lam_t - e, P) * v).item()) / (2 * h)
        assert abs(fdm - mu.grad[cell].item()) <= 1e-6 * max(abs(fdm), 1e-12)
        assert abs(fdl - lam.grad[cell].item()) <= 1e-6 * max(abs(fdl), 1e-12)
