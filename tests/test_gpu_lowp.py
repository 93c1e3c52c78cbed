"""Reduced-precision ROM apply (FP32 / bf16 slices on the matrix cores, FP64 apply) against the
FP64 oracle, with the FP64-measured refinement:

* relative error <= 1e-5 at refine_tol 1e-6, and each added starting level reduces the error;
* err_est is at most refine_tol, and it is an estimate of the true error (within a factor 10);
* a tolerance that three bf16 levels cannot meet ends in the FP64 combination (same bits as
  prec = LAT_F64, err_est = 0);
* the principal tangents with their least-squares alpha (large, cancelling coefficients) still
  meet the tolerance, by the refinement;
* right-hand-side counts that are not a walk's width (chunks of 16, 8 and fewer);
* the adjoint's reduced precision: Xbar within 1e-5, the forms (W in FP32) within 1e-6.
"""
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
}


@pytest.fixture(scope="module", params=list(CASES))
def lp(request):
    c = Case(CASES[request.param]())
    P, cfg = c.P, c.cfg
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True)
    g = P.select_principal(r["snap"], cfg.tol, keep_Z=True)
    n_r = int(g["n_r"].item())
    ops = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r, parts=True)
    bs = P.basis_stack(g["Z"], g["nu"], g["beta"], n_r)
    X, Xp = c.rhs()
    # FP64 reference: the oracle's ROM apply with the GPU's principal cells and coefficients
    S = g["S"].cpu().numpy()[:n_r]
    Kp = c.orc["T"][S]
    alpha = g["alpha"].cpu().numpy()
    Yo = O.combo_apply(c.dim, c.nel, Kp, alpha, c.l2g, X)
    return dict(c=c, g=g, n_r=n_r, ops=ops, bs=bs, X=X, Xp=Xp, Yo=Yo, Kp=Kp, alpha=alpha)


def _err(c):
    return torch.zeros(1, dtype=torch.float64, device=c.dev)


def test_basis_form_equals_rom_fp64(lp):
    c = lp["c"]
    Yb = c.unpack(c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m))
    assert rel(Yb, lp["Yo"]) <= 1e-9


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_lowp_within_1e5(lp, prec):
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    pr = B.F32 if prec == "f32" else B.BF16
    e = _err(c)
    Y = c.unpack(c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m, prec=pr,
                                 refine_tol=1e-6, err_est=e))
    err, est = rel(Y, lp["Yo"]), e.item()
    print(f"[lowp] {c.cfg.name} {prec} rel err {err:.3e} estimate {est:.3e}")
    assert err <= 1e-5
    assert est <= 1e-6
    assert err <= 10 * est + 1e-12
    assert np.all(Y[c.l2g < 0] == 0)


def test_bf16_refinement_levels_and_estimates(lp):
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    errs, ests = [], []
    for tol in (1e-2, 1e-4, 1e-6):          # starts at 1, 2, 3 levels of slice products
        e = _err(c)
        Y = c.unpack(c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m, prec=B.BF16,
                                     refine_tol=tol, err_est=e))
        errs.append(rel(Y, lp["Yo"]))
        ests.append(e.item())
        assert ests[-1] <= tol
        # the estimate is of the right size: the true error is neither far above nor far below it
        assert errs[-1] <= 10 * ests[-1] + 1e-12
        assert ests[-1] <= 10 * errs[-1] + 1e-12
    print(f"[lowp] {c.cfg.name} bf16 tol 1e-2/1e-4/1e-6: err " + " ".join(f"{x:.2e}" for x in errs) +
          "  est " + " ".join(f"{x:.2e}" for x in ests))
    assert errs[0] <= 2e-2
    assert errs[1] < errs[0] and errs[2] <= errs[1]


def test_unreachable_tolerance_ends_in_fp64(lp):
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    for pr in (B.BF16, B.F32):
        e = _err(c)
        e.fill_(1.0)
        Y = c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m, prec=pr, refine_tol=1e-13,
                            err_est=e)
        Y64 = c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m)
        assert torch.equal(Y, Y64)
        assert e.item() == 0.0


def test_principal_tangents_with_alpha(lp):
    # the principal-stack form: alpha can be large and cancelling; the FP64-measured refinement
    # must still deliver the tolerance
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    amax = np.abs(lp["alpha"]).max()
    for pr in (B.BF16, B.F32):
        e = _err(c)
        Y = c.unpack(c.P.apply_combo(lp["ops"]["K"], lp["n_r"], lp["g"]["alpha"], lp["Xp"], c.m, prec=pr,
                                     refine_tol=1e-6, err_est=e))
        err = rel(Y, lp["Yo"])
        print(f"[lowp] {c.cfg.name} principal+alpha prec {pr}: |alpha|max {amax:.2e} err {err:.3e} est {e.item():.3e}")
        assert e.item() <= 1e-6
        assert err <= 1e-5


@pytest.mark.parametrize("m", [3, 5, 20, 24, 32])
def test_rhs_chunks(lp, m):
    # the walks take 16, 8 or fewer right-hand sides at a time: FP64 and bf16 with every count
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    P = c.P
    X, Xp = c.rhs(m=m, stream=3)
    Yo = O.combo_apply(c.dim, c.nel, lp["Kp"], lp["alpha"], c.l2g, X)
    Y = c.unpack(P.apply_combo(lp["ops"]["K"], lp["n_r"], lp["g"]["alpha"], Xp, m), m)
    assert rel(Y, Yo) <= 1e-10 and np.abs(Y - Yo).max() <= 1e-10 * np.abs(Yo).max()
    YT = c.unpack(P.apply_combo(lp["ops"]["K"], lp["n_r"], lp["g"]["alpha"], Xp, m, transpose=True), m)
    assert rel(YT, O.combo_apply(c.dim, c.nel, lp["Kp"], lp["alpha"], c.l2g, X, transpose=True)) <= 1e-10
    e = _err(c)
    Yb = c.unpack(P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], Xp, m, prec=B.BF16,
                                refine_tol=2.0 ** -16, err_est=e), m)
    assert rel(Yb, Yo) <= 1e-5 and e.item() <= 2.0 ** -16


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_adjoint_reduced_precision(lp, prec):
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    P = c.P
    pr = B.F32 if prec == "f32" else B.BF16
    X, Xp = lp["X"], lp["Xp"]
    Yb, Ybp = c.rhs(stream=1)
    ops, g, n_r = lp["ops"], lp["g"], lp["n_r"]
    kw = dict(K_mu=ops["K_mu"], K_lam=ops["K_lam"], S=g["S"])
    a64 = P.apply_combo_adjoint(ops["K"], n_r, g["alpha"], Xp, Ybp, c.m, **kw)
    e = _err(c)
    alo = P.apply_combo_adjoint(ops["K"], n_r, g["alpha"], Xp, Ybp, c.m, prec=pr, refine_tol=1e-6, err_est=e,
                                fast=True, **kw)
    Xbo = O.combo_apply(c.dim, c.nel, lp["Kp"], lp["alpha"], c.l2g, Yb, transpose=True)
    errx = rel(c.unpack(alo["Xbar"]), Xbo)
    print(f"[lowp] {c.cfg.name} adjoint {prec}: Xbar err {errx:.3e} est {e.item():.3e}")
    assert errx <= 1e-5 and e.item() <= 1e-6
    for k in ("alpha_bar", "mu_bar", "lam_bar"):
        assert rel(alo[k].cpu().numpy(), a64[k].cpu().numpy()) <= 1e-6, k
