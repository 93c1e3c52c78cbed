"""lat_apply_combo_noalloc (the ROM apply whose scratch is a fixed device array) against
lat_apply_combo with a caller workspace, through the C ABI: two calls in a row on the same GPU, the
second on a smaller lattice with fewer right-hand sides, in FP64 (same bits) and bf16 (same bits and
the same error estimate; both take the same kernels)."""
import ctypes

import numpy as np
import pytest
import torch

import lattice as L
from gpu_common import Case

pytestmark = pytest.mark.gpu


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _setup(cfg, m):
    c = Case(cfg, m=m)
    P = c.P
    r = P.residual_tangent(c.ug, c.mu_t, c.lam_t, f=False, energy=False, snap=True)
    g = P.select_principal(r["snap"], cfg.tol, keep_Z=True)
    n_r = int(g["n_r"].item())
    ops = P.principal_ops(c.ug, c.mu_t, c.lam_t, g["S"], n_r)
    bs = P.basis_stack(g["Z"], g["nu"], g["beta"], n_r)
    _, Xp = c.rhs(m=m)
    return c, n_r, ops, g, bs, Xp


def _both(c, K, n_r, coef, Xp, m, prec, tol, transpose):
    from paper_2603_10741_amd import binding as B
    L_ = B._lib()
    P = c.P
    Y_ref = torch.full((P.packed_size(m),), float("nan"), dtype=torch.float64, device=c.dev)
    Y_na = torch.full_like(Y_ref, float("nan"))
    e_ref = torch.full((1,), -1.0, dtype=torch.float64, device=c.dev)
    e_na = torch.full_like(e_ref, -1.0)
    w, wb = P.workspace(B.CALL_APPLY_COMBO)
    st = L_.lat_apply_combo(P._p, _p(K), n_r, _p(coef), _p(Xp), _p(Y_ref), m, prec, ctypes.c_double(tol), transpose,
                            _p(e_ref), w, wb, _s())
    assert st == B.LAT_OK
    st = L_.lat_apply_combo_noalloc(P._p, _p(K), n_r, _p(coef), _p(Xp), _p(Y_na), m, prec, ctypes.c_double(tol),
                                    transpose, _p(e_na), _s())
    assert st == B.LAT_OK
    torch.cuda.synchronize()
    assert torch.equal(Y_na, Y_ref)
    assert torch.equal(e_na, e_ref)
    return Y_na


def test_noalloc_matches_workspace_entry_two_calls():
    from paper_2603_10741_amd import binding as B
    big = _setup(L.config(1), 16)              # 1024 cells, m = 16
    small = _setup(L.config(0), 8)             # 16 cells, m = 8: the second call is smaller
    for (c, n_r, ops, g, bs, Xp), m in ((big, 16), (small, 8)):
        print(f"[noalloc] {c.cfg.name} cells={c.cfg.n_cells} m={m} n_r={n_r}", flush=True)
        _both(c, ops["K"], n_r, g["alpha"], Xp, m, B.F64, 0.0, 0)
        _both(c, ops["K"], n_r, g["alpha"], Xp, m, B.F64, 0.0, 1)
        Y = _both(c, bs["stack"], n_r, bs["coef"], Xp, m, B.BF16, 2.0 ** -16, 0)
        assert torch.isfinite(Y).all()


def test_noalloc_rejects_oversized_scratch():
    # 192 x 192 cells of 2 x 2 elements with cap 64: 64 x 36864 x 8 bytes of coefficients alone exceed
    # the fixed array, so the call is refused on the host and nothing is launched
    from paper_2603_10741_amd import binding as B
    keep = np.ones((192 * 192, 4), np.uint8)
    P = B.Plan(2, (192, 192), 2, keep, cap=64)
    assert P.work_min[B.CALL_APPLY_COMBO] > (16 << 20)
    dev = torch.device("cuda:0")
    K = torch.zeros(P.nloc * P.E * P.cap, dtype=torch.float64, device=dev)
    a = torch.zeros(P.ncells * P.cap, dtype=torch.float64, device=dev)
    X = torch.zeros(P.packed_size(1), dtype=torch.float64, device=dev)
    Y = torch.zeros_like(X)
    st = B._lib().lat_apply_combo_noalloc(P._p, _p(K), 4, _p(a), _p(X), _p(Y), 1, B.F64, ctypes.c_double(0.0), 0, None,
                                          _s())
    assert st == B.LAT_E_SHAPE
