"""Reduced-precision ROM apply (FP32 VALU, bf16 matrix cores with sliced operands) against the
FP64 oracle: relative error <= 1e-5 at the default refinement, and each added refinement level
reduces the error."""
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
    ops = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r)
    bs = P.basis_stack(g["Z"], g["nu"], g["beta"], n_r)
    X, Xp = c.rhs()
    # FP64 reference: the oracle's ROM apply with the GPU's principal cells and coefficients
    S = g["S"].cpu().numpy()[:n_r]
    Kp = c.orc["T"][S]
    Yo = O.combo_apply(c.dim, c.nel, Kp, g["alpha"].cpu().numpy(), c.l2g, X)
    return dict(c=c, g=g, n_r=n_r, ops=ops, bs=bs, X=X, Xp=Xp, Yo=Yo)


def test_basis_form_equals_rom_fp64(lp):
    c = lp["c"]
    Yb = c.unpack(c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m))
    assert rel(Yb, lp["Yo"]) <= 1e-9


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_lowp_within_1e5(lp, prec):
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    pr = B.F32 if prec == "f32" else B.BF16
    Y = c.unpack(c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m, prec=pr,
                                 refine_tol=1e-6))
    err = rel(Y, lp["Yo"])
    print(f"[lowp] {c.cfg.name} {prec} rel err {err:.3e}")
    assert err <= 1e-5
    assert np.all(Y[c.l2g < 0] == 0)


def test_bf16_refinement_levels(lp):
    from paper_2603_10741_amd import binding as B
    c = lp["c"]
    errs = []
    for tol in (1e-2, 1e-4, 1e-6):          # 1, 2, 3 levels of slice products
        Y = c.unpack(c.P.apply_combo(lp["bs"]["stack"], lp["n_r"], lp["bs"]["coef"], lp["Xp"], c.m, prec=B.BF16,
                                     refine_tol=tol))
        errs.append(rel(Y, lp["Yo"]))
    print(f"[lowp] {c.cfg.name} bf16 levels 1/2/3: " + " ".join(f"{e:.2e}" for e in errs))
    assert errs[0] <= 2e-2
    assert errs[1] < errs[0] and errs[2] <= errs[1]
