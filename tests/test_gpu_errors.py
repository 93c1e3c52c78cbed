"""Failure handling and the C-ABI contract of the hot-path calls, through the C ABI:

* data-dependent failures reach the device status word with the first bad cell: a non-finite
  displacement (LAT_E_NONFINITE), an inverted element (LAT_E_INVERTED); a cap warning raised after
  them by the greedy never hides them, and the binding's status check raises;
* argument and shape errors of lat_residual_tangent, lat_select_principal, lat_apply_combo and
  lat_apply_combo_adjoint are returned synchronously (null pointers, n_r or cap beyond the plan's
  cap, a workspace below lat_plan_query's minimum or misaligned, bad precision or tolerance);
* a caller workspace (minimum or fast size) gives the same bits as the plan's own.
"""
import ctypes

import numpy as np
import pytest
import torch

import lattice as L
from gpu_common import Case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c():
    return Case(L.config(0))


def _lib():
    from paper_2603_10741_amd import binding as B
    return B._lib()


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_nonfinite_displacement_first_cell_and_cap_does_not_hide_it(c):
    from paper_2603_10741_amd import binding as B
    P = c.P
    ug = c.ug.clone().view(-1, c.dim)
    # a global node shared by several cells: the status names the lowest of them
    counts = np.bincount(c.l2g[c.l2g >= 0], minlength=P.nglobal)
    gnode = int(np.nonzero(counts >= 2)[0][len(np.nonzero(counts >= 2)[0]) // 2])
    owners = np.nonzero((c.l2g == gnode).any(axis=1))[0]
    ug[gnode, 0] = float("nan")
    P.reset_status()
    r = P.residual_tangent(ug.view(-1), c.mu_t, c.lam_t, f=True, energy=False, snap=True)
    torch.cuda.synchronize()
    code, cell = (int(x) for x in P.status_word.cpu())
    assert code == B.LAT_E_NONFINITE and cell == int(owners.min())
    # a greedy that stops at its cap raises LAT_W_CAP afterwards: the error stays
    P.select_principal(r["snap"], 1e-14, cap=1)
    torch.cuda.synchronize()
    code2, cell2 = (int(x) for x in P.status_word.cpu())
    assert (code2, cell2) == (code, cell)
    with pytest.raises(B.LatError) as ei:
        P.check_status()
    assert ei.value.code == B.LAT_E_NONFINITE


def test_inverted_element_first_cell(c):
    from paper_2603_10741_amd import binding as B
    P, cfg = c.P, c.cfg
    nel, nn = cfg.nel, cfg.nel + 1
    cell = 5
    a = 8 + nn * 2                                 # an interior node of cell 5 with kept elements around it
    gnode = int(c.l2g[cell, a])
    assert gnode >= 0 and np.count_nonzero((c.l2g == gnode).any(axis=1)) == 1
    ug = c.ug.clone().view(-1, c.dim)
    ug[gnode, 1] += 3.0 / nel                      # moves the node three elements up: elements above invert
    P.reset_status()
    r = P.residual_tangent(ug.view(-1), c.mu_t, c.lam_t, f=True, energy=False, snap=True)
    P.select_principal(r["snap"], 1e-14, cap=1)     # capped greedy after the error
    torch.cuda.synchronize()
    code, first = (int(x) for x in P.status_word.cpu())
    assert code == B.LAT_E_INVERTED and first == cell
    with pytest.raises(B.LatError):
        P.check_status(allow_cap=True)


def test_cap_warning_alone_is_a_warning(c):
    from paper_2603_10741_amd import binding as B
    P = c.P
    P.reset_status()
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True)
    P.select_principal(r["snap"], 1e-14, cap=2)
    code, cell = P.check_status(allow_cap=True)
    assert code == B.LAT_W_CAP and cell == 0x7fffffff
    with pytest.raises(B.LatError):
        P.check_status(allow_cap=False)


def test_argument_and_shape_errors(c):
    from paper_2603_10741_amd import binding as B
    L_ = _lib()
    P = c.P
    p = P._p
    dev = c.dev
    f64 = lambda n: torch.zeros(n, dtype=torch.float64, device=dev)
    st = P.status_word
    snap = f64(P.nsnap * P.ld)
    K = f64(P.nloc * P.E * P.cap)
    alpha = f64(P.ncells * P.cap)
    X = f64(P.packed_size(c.m))
    Y = f64(P.packed_size(c.m))
    S = torch.zeros(P.cap, dtype=torch.int32, device=dev)
    nr = torch.zeros(1, dtype=torch.int32, device=dev)
    R = f64(P.cap * P.cap)
    ach = f64(1)
    Z0 = ctypes.c_size_t(0)
    ok_w = P.workspace(B.CALL_APPLY_COMBO)
    # ---- lat_residual_tangent
    assert L_.lat_residual_tangent(None, _p(c.ug), _p(c.mu_t), _p(c.lam_t), 0, None, None, _p(snap), None, _p(st), None,
                                   Z0, _s()) == B.LAT_E_ARG
    assert L_.lat_residual_tangent(p, None, _p(c.mu_t), _p(c.lam_t), 0, None, None, _p(snap), None, _p(st), None, Z0,
                                   _s()) == B.LAT_E_ARG
    assert L_.lat_residual_tangent(p, _p(c.ug), _p(c.mu_t), _p(c.lam_t), 9, None, None, _p(snap), None, _p(st), None,
                                   Z0, _s()) == B.LAT_E_ARG
    small = torch.zeros(256, dtype=torch.uint8, device=dev)
    assert L_.lat_residual_tangent(p, _p(c.ug), _p(c.mu_t), _p(c.lam_t), 0, None, None, _p(snap), None, _p(st),
                                   _p(small), ctypes.c_size_t(256), _s()) == B.LAT_E_SHAPE
    # ---- lat_select_principal
    args = lambda cap: (p, _p(snap), ctypes.c_double(1e-8), cap, _p(S), _p(nr), _p(alpha), None, None, _p(R), None,
                        _p(ach), _p(st), None, Z0, _s())
    assert L_.lat_select_principal(*args(P.cap + 1)) == B.LAT_E_SHAPE
    assert L_.lat_select_principal(*args(0)) == B.LAT_E_ARG
    bad = list(args(P.cap)); bad[1] = None
    assert L_.lat_select_principal(*bad) == B.LAT_E_ARG
    bad = list(args(P.cap)); bad[2] = ctypes.c_double(-1.0)
    assert L_.lat_select_principal(*bad) == B.LAT_E_ARG
    assert L_.lat_select_principal_rows(p, _p(snap), P.nsnap + 1, ctypes.c_double(1e-8), P.cap, _p(S), _p(nr), _p(alpha),
                                        None, None, _p(R), None, _p(ach), _p(st), None, Z0, _s()) == B.LAT_E_SHAPE
    # ---- lat_apply_combo
    ac = lambda n_r, m, prec, tol, w, wb: L_.lat_apply_combo(p, _p(K), n_r, _p(alpha), _p(X), _p(Y), m, prec,
                                                              ctypes.c_double(tol), 0, None, w, wb, _s())
    assert ac(P.cap + 1, c.m, B.F64, 0.0, None, Z0) == B.LAT_E_SHAPE
    assert ac(-1, c.m, B.F64, 0.0, None, Z0) == B.LAT_E_SHAPE
    assert ac(4, 0, B.F64, 0.0, None, Z0) == B.LAT_E_ARG
    assert ac(4, c.m, 7, 0.0, None, Z0) == B.LAT_E_ARG
    assert ac(4, c.m, B.BF16, -1.0, None, Z0) == B.LAT_E_ARG
    assert ac(4, c.m, B.F64, 0.0, _p(small), ctypes.c_size_t(16)) == B.LAT_E_SHAPE
    wt, wb = ok_w
    mis = ctypes.c_void_p(wt.value + 8)
    assert ac(4, c.m, B.F64, 0.0, mis, ctypes.c_size_t(wb.value - 8)) == B.LAT_E_ARG
    assert L_.lat_apply_combo(p, None, 4, _p(alpha), _p(X), _p(Y), c.m, B.F64, ctypes.c_double(0.0), 0, None, None, Z0,
                              _s()) == B.LAT_E_ARG
    # ---- lat_apply_combo_adjoint
    ad = lambda n_r, mu_bar, S_, prec: L_.lat_apply_combo_adjoint(
        p, _p(K), _p(K), _p(K), S_, n_r, _p(alpha), _p(X), _p(Y), c.m, _p(f64(P.packed_size(c.m))), _p(alpha), mu_bar,
        None, prec, ctypes.c_double(1e-6), None, None, Z0, _s())
    assert ad(P.cap + 1, None, _p(S), B.F64) == B.LAT_E_SHAPE
    assert ad(4, _p(f64(P.ncells)), None, B.F64) == B.LAT_E_ARG            # mu_bar needs S
    assert ad(4, None, _p(S), 5) == B.LAT_E_ARG
    torch.cuda.synchronize()
    # ---- the binding refuses tensors smaller than the call touches
    with pytest.raises(ValueError):
        P.apply_combo(K[:10], 4, alpha, X, c.m)
    with pytest.raises(ValueError):
        P.select_principal(snap, 1e-8, out={"S": S[:2], "n_r": nr, "alpha": alpha, "beta": None, "nu": None, "R": R,
                                            "achieved": ach})


def test_query_sizes(c):
    from paper_2603_10741_amd import binding as B
    P = c.P
    for call in range(B.N_CALLS):
        assert 0 < P.work_min[call] <= P.work_fast[call]
    # the adjoint's fast size holds the cells' W (n_snap x ld doubles)
    assert P.work_fast[B.CALL_APPLY_COMBO_ADJOINT] - P.work_min[B.CALL_APPLY_COMBO_ADJOINT] >= P.nsnap * P.ld * 8


def test_caller_workspace_same_bits(c):
    from paper_2603_10741_amd import binding as B
    L_ = _lib()
    P = c.P
    dev, m = c.dev, c.m
    p = P._p
    Z0 = ctypes.c_size_t(0)
    # residual / snapshots with the plan's own scratch vs the caller's
    r1 = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=True, energy=True, snap=True)
    snap0 = torch.empty_like(r1["snap"]); f0 = torch.empty_like(r1["f"]); e0 = torch.empty_like(r1["energy"])
    assert L_.lat_residual_tangent(p, _p(c.ug), _p(c.mu_t), _p(c.lam_t), 0, _p(f0), _p(e0), _p(snap0), None,
                                   _p(P.status_word), None, Z0, _s()) == 0
    assert torch.equal(snap0, r1["snap"]) and torch.equal(f0, r1["f"]) and torch.equal(e0, r1["energy"])
    g = P.select_principal(r1["snap"].clone(), c.cfg.tol, keep_Z=True)
    g0 = P.select_principal(snap0.clone(), c.cfg.tol, keep_Z=True)
    for k in ("S", "n_r", "alpha", "R", "achieved"):
        assert torch.equal(g[k], g0[k])
    n_r = int(g["n_r"].item())
    parts = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r, parts=True)
    X, Xp = c.rhs()
    _, Ybp = c.rhs(stream=1)
    Y1 = P.apply_combo(parts["K"], n_r, g["alpha"], Xp, m)
    Y0 = torch.empty_like(Y1)
    assert L_.lat_apply_combo(p, _p(parts["K"]), n_r, _p(g["alpha"]), _p(Xp), _p(Y0), m, B.F64, ctypes.c_double(0.0),
                              0, None, None, Z0, _s()) == 0
    assert torch.equal(Y0, Y1)
    # adjoint: fast workspace (W pass), minimum workspace and the plan's own (fused kernel) agree
    kw = dict(K_mu=parts["K_mu"], K_lam=parts["K_lam"], S=g["S"])
    a_fast = P.apply_combo_adjoint(parts["K"], n_r, g["alpha"], Xp, Ybp, m, fast=True, **kw)
    a_min = P.apply_combo_adjoint(parts["K"], n_r, g["alpha"], Xp, Ybp, m, fast=False, **kw)
    assert torch.equal(a_fast["Xbar"], a_min["Xbar"])
    for k in ("alpha_bar", "mu_bar", "lam_bar"):
        ref = a_fast[k]
        assert torch.max(torch.abs(a_min[k] - ref)).item() <= 1e-12 * torch.max(torch.abs(ref)).item()


def test_adjoint_lane_batches_same_bits():
    # a workspace with room for one 64-lane group of W past its minimum: the W pass and the
    # contractions run in 16 batches on the 1024-cell lattice, with every lane's arithmetic unchanged
    from paper_2603_10741_amd import binding as B
    c = Case(L.config(1))
    P, m = c.P, c.m
    L_ = _lib()
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True)
    g = P.select_principal(r["snap"], c.cfg.tol)
    n_r = int(g["n_r"].item())
    parts = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r, parts=True)
    _, Xp = c.rhs()
    _, Ybp = c.rhs(stream=1)
    kw = dict(K_mu=parts["K_mu"], K_lam=parts["K_lam"], S=g["S"])
    mn, fs = P.work_min[B.CALL_APPLY_COMBO_ADJOINT], P.work_fast[B.CALL_APPLY_COMBO_ADJOINT]
    nbytes = mn + (fs - mn) * 64 // P.ld + 4096
    assert nbytes < mn + (fs - mn) * 128 // P.ld          # room for one group, not two
    work = torch.empty(nbytes, dtype=torch.uint8, device=c.dev)
    for prec in (B.F64, B.BF16):
        ref = P.apply_combo_adjoint(parts["K"], n_r, g["alpha"], Xp, Ybp, m, fast=True, prec=prec, **kw)
        out = {k: torch.empty_like(v) for k, v in ref.items()}
        st = L_.lat_apply_combo_adjoint(P._p, _p(parts["K"]), _p(parts["K_mu"]), _p(parts["K_lam"]), _p(g["S"]), n_r,
                                        _p(g["alpha"]), _p(Xp), _p(Ybp), m, _p(out["Xbar"]), _p(out["alpha_bar"]),
                                        _p(out["mu_bar"]), _p(out["lam_bar"]), prec, ctypes.c_double(1e-6), None,
                                        _p(work), ctypes.c_size_t(nbytes), _s())
        assert st == B.LAT_OK
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (prec, k)
