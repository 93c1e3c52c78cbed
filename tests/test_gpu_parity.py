"""GPU parity: every C-ABI entry point against the FP64 oracle on the same seeded inputs.

Bars: DOF maps and principal-cell indices bit-exact; the greedy fed with the oracle's
snapshots bit-exact in every output (same fixed arithmetic order on both sides); FP64
operator applies within 1e-10 relative (Frobenius); tangents/residuals within 1e-12 of the
largest entry (only rounding order and the log implementation differ)."""
import numpy as np
import pytest
import torch

import lattice as L
import oracle as O
from gpu_common import Case, rel

pytestmark = pytest.mark.gpu

CASES = {
    "hole4": lambda: L.config(0),
    "hole32": lambda: L.config(1),
    "bcc_sub": lambda: L.config(2).with_sub((3, 3, 2)),
    "mixed_sub": lambda: L.config(4).with_sub((2, 2, 2)),
    "logmu_sub": lambda: L.config(3).with_sub((2, 2, 2)),
    # cells of more than 16 elements per edge: the per-node 3D tangent kernel instead of the
    # node-line sweep (whose kept-element masks hold 4 x 16 slots)
    "bcc_n18_sub": lambda: L.config(2).with_(nel=18).with_sub((2, 2, 1)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    return Case(CASES[request.param]())


def test_dofmap_bit_exact(case):
    np.testing.assert_array_equal(case.l2g_gpu.cpu().numpy(), case.l2g)
    np.testing.assert_array_equal(case.nact_gpu.cpu().numpy(), case.nact)
    np.testing.assert_array_equal(case.g2bg_gpu.cpu().numpy(), case.g2bg)
    perm = case.perm.cpu().numpy()
    cells = perm[perm >= 0]
    assert sorted(cells.tolist()) == list(range(case.cfg.n_cells))


def test_residual_energy_snapshot(case):
    P = case.P
    P.reset_status()
    r = P.residual_tangent(case.ug, case.mu_t, case.lam_t, f=True, energy=True, snap=True, plain=True)
    P.check_status()
    o = case.orc
    f = case.canon_field(r["f"], case.dim)
    T = case.canon_T(r["snap"])
    scale_f = np.abs(o["f"]).max()
    assert np.abs(f - o["f"]).max() <= 1e-12 * scale_f
    np.testing.assert_allclose(r["energy"].cpu().numpy(), o["energy"], rtol=1e-12, atol=1e-15)
    assert np.abs(T - o["T"]).max() <= 1e-12 * np.abs(o["T"]).max()
    Kc = P.plain_ops_to_canon(r["plain"]).cpu().numpy()
    assert np.abs(Kc - o["T"]).max() <= 1e-12 * np.abs(o["T"]).max()
    # assembled residual r = sum_s A^s f^s
    rg = P.assemble(r["f"], case.dim)[: P.nglobal * case.dim].cpu().numpy().reshape(-1, case.dim)
    ro = O.assemble(o["f"], case.l2g, P.nglobal)
    assert np.abs(rg - ro).max() <= 1e-12 * scale_f


def test_residual_only_path(case):
    # force and energy without the tangent (element-centric colour passes) against the oracle and
    # against the tangent kernel's own force
    P = case.P
    P.reset_status()
    r1 = P.residual_tangent(case.ug, case.mu_t, case.lam_t, f=True, energy=True, snap=False, plain=False)
    r2 = P.residual_tangent(case.ug, case.mu_t, case.lam_t, f=True, energy=True, snap=True, plain=False)
    P.check_status()
    o = case.orc
    f1 = case.canon_field(r1["f"], case.dim)
    f2 = case.canon_field(r2["f"], case.dim)
    scale = np.abs(o["f"]).max()
    assert np.abs(f1 - o["f"]).max() <= 1e-12 * scale
    assert np.abs(f1 - f2).max() <= 1e-12 * scale
    np.testing.assert_allclose(r1["energy"].cpu().numpy(), o["energy"], rtol=1e-12, atol=1e-15)


def test_greedy_cross_fed_bit_exact(case):
    """GPU greedy on the oracle's snapshots reproduces the oracle bit for bit."""
    P, cfg = case.P, case.cfg
    T = case.orc["T"]
    T_cil = case.to_cil_T(T)
    P.reset_status()
    g = P.select_principal(T_cil, cfg.tol, keep_Z=True)
    go = O.greedy(T, cfg.tol, cfg.cap, keep_Z=True)
    code, _ = P.check_status()
    n_r = int(g["n_r"].item())
    assert n_r == go["n_r"]
    assert (code == 7) == (go["status"] == O.W_CAP)
    np.testing.assert_array_equal(g["S"].cpu().numpy(), go["S"])
    np.testing.assert_array_equal(g["nu"].cpu().numpy(), go["nu"])
    np.testing.assert_array_equal(g["beta"].cpu().numpy(), go["beta"])
    np.testing.assert_array_equal(g["R"].cpu().numpy(), go["R"])
    np.testing.assert_array_equal(g["alpha"].cpu().numpy(), go["alpha"])
    np.testing.assert_array_equal(g["Z"].cpu().numpy(), go["Z"])
    assert g["achieved"].item() == go["achieved"]
    np.testing.assert_array_equal(case.canon_T(T_cil), go["Delta"])


@pytest.mark.parametrize("cap", [1, 5, 8, 13])
def test_greedy_lagged_residuals(case, cap):
    """The greedy writes its residuals back every 8 iterations and replays the pending updates in
    between; stopping at a cap that is not a multiple of 8 leaves pending updates that the exit
    applies.  Every output, the residual Delta included, must still be the oracle's bit for bit."""
    P, cfg = case.P, case.cfg
    cap = min(cap, P.cap)
    T = case.orc["T"]
    T_cil = case.to_cil_T(T)
    P.reset_status()
    g = P.select_principal(T_cil, cfg.tol, cap=cap, keep_Z=True)
    go = O.greedy(T, cfg.tol, cap, keep_Z=True)
    P.check_status()
    n_r = int(g["n_r"].item())
    assert n_r == go["n_r"]
    np.testing.assert_array_equal(g["S"].cpu().numpy()[:cap], go["S"][:cap])
    np.testing.assert_array_equal(g["beta"].cpu().numpy()[:, :cap], go["beta"][:, :cap])
    np.testing.assert_array_equal(g["alpha"].cpu().numpy()[:, :cap], go["alpha"][:, :cap])
    np.testing.assert_array_equal(g["Z"].cpu().numpy()[:cap], go["Z"][:cap])
    assert g["achieved"].item() == go["achieved"]
    np.testing.assert_array_equal(case.canon_T(T_cil), go["Delta"])


@pytest.mark.parametrize("cap", [5, 13])
def test_greedy_lagged_rows(case, cap):
    """The greedy on the leading rows only (the sampled-entry entry point), stopped between
    write-backs: the ring of basis rows is then strided by the row count.  The outputs are the
    oracle's greedy on those rows bit for bit, Z is zero past them, and the rows past them are
    left as they were."""
    P, cfg = case.P, case.cfg
    cap = min(cap, P.cap)
    T = case.orc["T"]
    rows = P.nsnap // 3 + 7
    T_cil = case.to_cil_T(T)
    P.reset_status()
    g = P.select_principal(T_cil, cfg.tol, cap=cap, keep_Z=True, rows=rows)
    go = O.greedy(np.ascontiguousarray(T[:, :rows]), cfg.tol, cap, keep_Z=True)
    P.check_status()
    assert int(g["n_r"].item()) == go["n_r"]
    np.testing.assert_array_equal(g["S"].cpu().numpy()[:cap], go["S"][:cap])
    np.testing.assert_array_equal(g["beta"].cpu().numpy()[:, :cap], go["beta"][:, :cap])
    np.testing.assert_array_equal(g["alpha"].cpu().numpy()[:, :cap], go["alpha"][:, :cap])
    Z = g["Z"].cpu().numpy()
    np.testing.assert_array_equal(Z[:cap, :rows], go["Z"][:cap])
    assert not Z[:, rows:].any()
    assert g["achieved"].item() == go["achieved"]
    D = case.canon_T(T_cil)
    np.testing.assert_array_equal(D[:, :rows], go["Delta"])
    np.testing.assert_array_equal(D[:, rows:], T[:, rows:])


def test_greedy_end_to_end(case):
    """GPU snapshots -> GPU greedy vs oracle snapshots -> oracle greedy: the same principal cells
    unless the arg-max margin at the diverging step is below the snapshots' rounding level."""
    P, cfg = case.P, case.cfg
    r = P.residual_tangent(case.ug, case.mu_t, case.lam_t, f=False, energy=False, snap=True)
    g = P.select_principal(r["snap"], cfg.tol, keep_Z=False)
    go = O.greedy(case.orc["T"], cfg.tol, cfg.cap, keep_Z=False)
    S, So = g["S"].cpu().numpy(), go["S"]
    n_r = int(g["n_r"].item())
    if n_r == go["n_r"] and np.array_equal(S, So):
        return
    # find the first divergence and check that it is a near-tie in the oracle's own arithmetic
    k = int(np.nonzero(S != So)[0][0]) if n_r == go["n_r"] else min(n_r, go["n_r"])
    pre = O.greedy(case.orc["T"], cfg.tol, k, keep_Z=False) if k > 0 else None
    D = pre["Delta"] if pre is not None else case.orc["T"] / np.linalg.norm(case.orc["T"], axis=1, keepdims=True)
    m = np.sort(np.abs(D).max(axis=1))[::-1]
    print(f"[greedy] {cfg.name}: principal cells differ at step {k}, margin {(m[0]-m[1])/m[0]:.3e}", flush=True)
    assert (m[0] - m[1]) <= 1e-12 * m[0], f"principal cells differ at step {k} with margin {(m[0]-m[1])/m[0]:.3e}"


def test_applies(case):
    P, cfg = case.P, case.cfg
    o = case.orc
    go = O.greedy(o["T"], cfg.tol, cfg.cap, keep_Z=False)
    n_r = go["n_r"]
    S_t = torch.from_numpy(go["S"]).to(case.dev)
    alpha_t = torch.from_numpy(go["alpha"]).to(case.dev)
    ops = P.principal_ops(case.ug, case.mu_t, case.lam_t, S_t, n_r, parts=True)
    # principal stack vs the oracle's principal stencils
    Kst = ops["K"].cpu().numpy().reshape(P.nloc, P.E, P.cap)
    Kp = o["T"][go["S"][:n_r]]
    for k in range(n_r):
        assert np.abs(Kst[:, :, k].ravel() - Kp[k]).max() <= 1e-12 * np.abs(Kp).max()
    assert np.all(Kst[:, :, n_r:] == 0)
    X, Xp = case.rhs()
    Y = case.unpack(P.apply_combo(ops["K"], n_r, alpha_t, Xp, case.m))
    Yo = O.combo_apply(case.dim, case.nel, Kp, go["alpha"], case.l2g, X)
    assert rel(Y, Yo) <= 1e-10
    YT = case.unpack(P.apply_combo(ops["K"], n_r, alpha_t, Xp, case.m, transpose=True))
    YTo = O.combo_apply(case.dim, case.nel, Kp, go["alpha"], case.l2g, X, transpose=True)
    assert rel(YT, YTo) <= 1e-10
    r = P.residual_tangent(case.ug, case.mu_t, case.lam_t, f=False, energy=False, snap=False, plain=True)
    Yp = case.unpack(P.apply_plain(r["plain"], Xp, case.m))
    Ypo = O.plain_apply(case.dim, case.nel, o["T"], case.l2g, X)
    assert rel(Yp, Ypo) <= 1e-10
    # outputs vanish at DOFs a cell does not own; round trip of the packed layout
    assert np.all(Y[case.l2g < 0] == 0)
    np.testing.assert_array_equal(case.unpack(Xp), case.masked(X))
    # element by element (no entry is allowed to hide behind the global norm) and per cell
    for a, b in ((Y, Yo), (YT, YTo), (Yp, Ypo)):
        assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    for c in range(0, case.cfg.n_cells, max(1, case.cfg.n_cells // 16)):
        assert rel(Y[c], Yo[c]) <= 1e-9


def test_combo_adjoint_forms_and_lame(case):
    _check_combo_adjoint(case)


@pytest.mark.parametrize("mk", [lambda: L.config(2).with_sub((4, 4, 3)), lambda: L.config(1).with_sub((6, 6))],
                         ids=["bcc_48", "hole_36"])
def test_combo_adjoint_wide_basis(mk):
    # N_r in (32, 64]: the widest contraction tiles of the adjoint forms
    case = Case(mk().with_(tol=1e-13, cap=64))
    assert _check_combo_adjoint(case) > 32


def _check_combo_adjoint(case):
    P, cfg = case.P, case.cfg
    o = case.orc
    go = O.greedy(o["T"], cfg.tol, cfg.cap, keep_Z=False)
    n_r = go["n_r"]
    S_t = torch.from_numpy(go["S"]).to(case.dev)
    alpha_t = torch.from_numpy(go["alpha"]).to(case.dev)
    ops = P.principal_ops(case.ug, case.mu_t, case.lam_t, S_t, n_r, parts=True)
    X, Xp = case.rhs()
    Yb, Ybp = case.rhs(stream=1)
    ad = P.apply_combo_adjoint(ops["K"], n_r, alpha_t, Xp, Ybp, case.m, K_mu=ops["K_mu"], K_lam=ops["K_lam"], S=S_t)
    Kp = o["T"][go["S"][:n_r]]
    Xb = case.unpack(ad["Xbar"])
    assert rel(Xb, O.combo_apply(case.dim, case.nel, Kp, go["alpha"], case.l2g, Yb, transpose=True)) <= 1e-10
    Go = O.combo_forms(case.dim, case.nel, Kp, cfg.cap, case.l2g, X, Yb)
    assert rel(ad["alpha_bar"].cpu().numpy(), Go) <= 1e-10
    Ns = cfg.n_cells
    ev_m = O.cells_eval(case.dim, case.nel, case.keep, case.uloc, np.ones(Ns), np.zeros(Ns), want_f=False,
                        want_energy=False)["T"]
    Gm = O.combo_forms(case.dim, case.nel, ev_m[go["S"][:n_r]], cfg.cap, case.l2g, X, Yb)
    mub = np.zeros(Ns)
    for k, s in enumerate(go["S"][:n_r]):
        mub[s] = np.sum(go["alpha"][:, k] * Gm[:, k])
    assert rel(ad["mu_bar"].cpu().numpy(), mub) <= 1e-10
    return n_r


def test_residual_adjoint(case):
    P = case.P
    rng = np.random.default_rng(11)
    o = case.orc
    rbar = rng.standard_normal((P.nglobal, case.dim))
    w_cil = P.gather(torch.from_numpy(rbar).to(case.dev), case.dim)
    res = P.residual_adjoint(case.ug, case.mu_t, case.lam_t, w_cil)
    P.check_status()
    w = O.gather_local(rbar, case.l2g)
    ub_o = np.zeros_like(w)
    for c in range(case.cfg.n_cells):
        ub_o[c] = O.stencil_apply(case.dim, case.nel, o["T"][c], case.l2g[c], w[c][:, :, None], transpose=True)[:, :, 0]
    ub = case.canon_field(res["ubar_local"], case.dim)
    assert rel(ub, ub_o) <= 1e-10
    ug = res["ubar_global"][: P.nglobal * case.dim].cpu().numpy().reshape(-1, case.dim)
    assert rel(ug, O.assemble(ub_o, case.l2g, P.nglobal)) <= 1e-10
    Ns = case.cfg.n_cells
    fm = O.cells_eval(case.dim, case.nel, case.keep, case.uloc, np.ones(Ns), np.zeros(Ns), want_T=False)["f"]
    fl = O.cells_eval(case.dim, case.nel, case.keep, case.uloc, np.zeros(Ns), np.ones(Ns), want_T=False)["f"]
    np.testing.assert_allclose(res["mu_bar"].cpu().numpy(), np.sum((w * fm).reshape(Ns, -1), 1), rtol=1e-10,
                               atol=1e-12 * np.abs(w * fm).sum())
    np.testing.assert_allclose(res["lam_bar"].cpu().numpy(), np.sum((w * fl).reshape(Ns, -1), 1), rtol=1e-10,
                               atol=1e-12 * np.abs(w * fl).sum())


def test_reduced_rule_snapshot(case):
    # one-point snapshots: every cell on the small cases, 24 seeded cells (plus the first and last)
    # on the 1024-cell lattice, compared entry by entry with the oracle's one-point rule
    P = case.P
    r = P.residual_tangent(case.ug, case.mu_t, case.lam_t, snap_rule=1, f=False, energy=False, snap=True)
    T = case.canon_T(r["snap"])
    Ns = case.cfg.n_cells
    cells = np.arange(Ns)
    if Ns > 64:
        rng = np.random.default_rng(1)
        cells = np.unique(np.concatenate([[0, Ns - 1], rng.choice(Ns, 24, replace=False)]))
    To = O.cells_eval(case.dim, case.nel, case.keep[cells], case.uloc[cells], case.mu[cells], case.lam[cells],
                      rule=O.RULE_REDUCED, want_f=False, want_energy=False)["T"]
    assert np.abs(T[cells] - To).max() <= 1e-12 * np.abs(To).max()
    # and the rule is really in use: the full-rule snapshot of the same cells differs
    Tf = case.canon_T(P.residual_tangent(case.ug, case.mu_t, case.lam_t, f=False, energy=False, snap=True)["snap"])
    assert np.linalg.norm(Tf[cells] - T[cells]) > 1e-3 * np.linalg.norm(Tf[cells])
