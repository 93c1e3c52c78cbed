"""Degenerate and edge cases of the GPU path, checked against the FP64 oracle and against what
the method states exactly:

* identical cells (zero displacement, one hole radius): Algorithm 1 keeps one principal cell,
  the lowest index on ties, every coefficient is 1 and the ROM operator is the plain one;
* an empty cell (every element removed): no active DOF, zero snapshot norm, never principal,
  zero coefficients and zero outputs, while the other cells still match the oracle;
* an empty basis (tolerance above every snapshot's max-norm): n_r = 0 and every ROM apply, in
  every precision, returns zeros;
* an odd number of right-hand sides (the generic kernels) and a cell count that is not a
  multiple of the 64-lane group;
* rigid translations lie in the kernel of every cell tangent at zero load.
"""
import numpy as np
import pytest
import torch

import lattice as L
import oracle as O
from gpu_common import Case, rel

pytestmark = pytest.mark.gpu


def _sub3():
    return L.config(0).with_sub((3, 3))          # 9 cells: one partly filled lane group


def test_identical_cells_single_principal():
    cfg = _sub3()
    u0 = np.zeros_like(L.make_displacement(cfg))
    c = Case(cfg, u_bg=u0)
    P = c.P
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True, plain=True)
    g = P.select_principal(r["snap"], cfg.tol)
    n_r = int(g["n_r"].item())
    assert n_r == 1
    assert int(g["S"][0].item()) == 0                     # ties go to the lowest cell index
    alpha = g["alpha"].cpu().numpy()
    assert np.all(alpha[:, 0] == 1.0)
    assert g["achieved"].item() <= 1e-14
    ops = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r)
    X, Xp = c.rhs()
    Yr = c.unpack(P.apply_combo(ops["K"], n_r, g["alpha"], Xp, c.m))
    Yp = c.unpack(P.apply_plain(r["plain"], Xp, c.m))
    assert rel(Yr, Yp) <= 1e-14
    Yo = O.plain_apply(c.dim, c.nel, c.orc["T"], c.l2g, X)
    assert rel(Yp, Yo) <= 1e-12


def test_empty_cell():
    cfg = _sub3()
    keep = L.make_keep(cfg).copy()
    keep[4] = 0                                           # the middle cell loses every element
    c = Case(cfg, keep=keep)
    P = c.P
    assert np.array_equal(c.nact_gpu.cpu().numpy(), c.nact)
    assert c.nact[4] == 0
    assert np.all(c.l2g_gpu.cpu().numpy()[4] == -1)
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=True, energy=True, snap=True, plain=True)
    g = P.select_principal(r["snap"], cfg.tol, keep_Z=True)
    n_r = int(g["n_r"].item())
    S = g["S"].cpu().numpy()[:n_r]
    assert 4 not in S
    assert g["nu"][4].item() == 0.0
    assert np.all(g["alpha"][4].cpu().numpy() == 0.0)
    assert r["energy"][4].item() == 0.0
    ops = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r)
    X, Xp = c.rhs()
    Yr = c.unpack(P.apply_combo(ops["K"], n_r, g["alpha"], Xp, c.m))
    Yp = c.unpack(P.apply_plain(r["plain"], Xp, c.m))
    assert np.all(Yr[4] == 0.0) and np.all(Yp[4] == 0.0)
    Yo = O.combo_apply(c.dim, c.nel, c.orc["T"][S], g["alpha"].cpu().numpy(), c.l2g, X)
    Ypo = O.plain_apply(c.dim, c.nel, c.orc["T"], c.l2g, X)
    assert rel(Yr, Yo) <= 1e-10 and rel(Yp, Ypo) <= 1e-10
    bs = P.basis_stack(g["Z"], g["nu"], g["beta"], n_r)
    Yb = c.unpack(P.apply_combo(bs["stack"], n_r, bs["coef"], Xp, c.m, prec=c.B.BF16, refine_tol=2.0 ** -16))
    assert np.all(Yb[4] == 0.0) and rel(Yb, Yo) <= 1e-5


def test_empty_basis_gives_zero():
    cfg = _sub3()
    c = Case(cfg)
    P = c.P
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True)
    g = P.select_principal(r["snap"], 10.0, keep_Z=True)   # every max-norm of a unit vector is <= 1
    assert int(g["n_r"].item()) == 0
    ops = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], 0)
    bs = P.basis_stack(g["Z"], g["nu"], g["beta"], 0)
    X, Xp = c.rhs()
    B = c.B
    assert torch.count_nonzero(P.apply_combo(ops["K"], 0, g["alpha"], Xp, c.m)).item() == 0
    for prec in (B.F32, B.BF16):
        Y = P.apply_combo(bs["stack"], 0, bs["coef"], Xp, c.m, prec=prec, refine_tol=1e-6)
        assert torch.count_nonzero(Y).item() == 0


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_small_and_odd_rhs_counts(m):
    # m in {1, 2, 4}: the ROM applies run the 2D row walk with idle waves past m, the plain apply the
    # per-group kernel; 3 and 5 the per-group kernels throughout
    cfg = _sub3()
    c = Case(cfg, m=m)
    P = c.P
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True, plain=True)
    g = P.select_principal(r["snap"], cfg.tol)
    n_r = int(g["n_r"].item())
    ops = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r)
    X, Xp = c.rhs(m=m)
    S = g["S"].cpu().numpy()[:n_r]
    Yr = c.unpack(P.apply_combo(ops["K"], n_r, g["alpha"], Xp, m), m)
    Yt = c.unpack(P.apply_combo(ops["K"], n_r, g["alpha"], Xp, m, transpose=True), m)
    Yp = c.unpack(P.apply_plain(r["plain"], Xp, m), m)
    alpha = g["alpha"].cpu().numpy()
    assert rel(Yr, O.combo_apply(c.dim, c.nel, c.orc["T"][S], alpha, c.l2g, X)) <= 1e-10
    assert rel(Yt, O.combo_apply(c.dim, c.nel, c.orc["T"][S], alpha, c.l2g, X, transpose=True)) <= 1e-10
    assert rel(Yp, O.plain_apply(c.dim, c.nel, c.orc["T"], c.l2g, X)) <= 1e-10


@pytest.mark.parametrize("cfg_fn", [lambda: _sub3(), lambda: L.config(2).with_sub((2, 2, 2))], ids=["hole", "bcc"])
def test_rigid_translation_in_kernel(cfg_fn):
    cfg = cfg_fn()
    u0 = np.zeros_like(L.make_displacement(cfg))
    c = Case(cfg, u_bg=u0, m=cfg.dim)
    P = c.P
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True, plain=True)
    # right-hand side r = unit translation along axis r at every node of every cell
    X = np.zeros((cfg.n_cells, P.nloc, cfg.dim, cfg.dim))
    for ax in range(cfg.dim):
        X[:, :, ax, ax] = 1.0
    X *= (c.l2g >= 0)[:, :, None, None]
    Xp = P.pack(torch.from_numpy(X).to(c.dev), cfg.dim)
    Y = c.unpack(P.apply_plain(r["plain"], Xp, cfg.dim), cfg.dim)
    scale = np.abs(c.orc["T"]).max() * 27
    assert np.abs(Y).max() <= 1e-12 * scale
