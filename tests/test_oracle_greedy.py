"""Pins of the oracle's greedy selection (Algorithm 1) and RB coefficients (least-squares
formula of Sec. 3.2.2).

Independent checks: a numpy re-statement of the loop with ordinary dot products, the
least-squares solution from numpy.linalg.lstsq, orthonormality of the basis, the certified
decomposition, the behaviour on identical cells, scaling and permutation invariance, and
the exactness of the fixed-order dot product against math.fsum.
"""
import math

import numpy as np
import pytest

import lattice as L


def _numpy_greedy(T, tol, cap):
    D = T / np.linalg.norm(T, axis=1, keepdims=True)
    S, B = [], []
    while True:
        m = np.abs(D).max(axis=1)
        if m.max() <= tol or len(S) == cap:
            break
        s = int(np.argmax(m))
        z = D[s] / np.linalg.norm(D[s])
        b = D @ z
        D = D - b[:, None] * z[None, :]
        S.append(s); B.append(b)
    return S, np.array(B).T, np.abs(D).max()


def _low_rank_T(rng, Ns, n, rank, noise):
    U = rng.standard_normal((Ns, rank)) * np.logspace(0, -3, rank)
    V = rng.standard_normal((rank, n))
    return U @ V + noise * rng.standard_normal((Ns, n))


@pytest.mark.parametrize("seed", range(5))
def test_greedy_matches_independent_mgs(orc, seed):
    rng = np.random.default_rng(seed)
    T = _low_rank_T(rng, 12, 700, 6, 1e-9)
    res = orc.greedy(T, 1e-6, 12)
    S, B, ach = _numpy_greedy(T, 1e-6, 12)
    assert res["n_r"] == len(S)
    assert list(res["S"][:res["n_r"]]) == S
    np.testing.assert_allclose(res["beta"][:, :res["n_r"]], B, atol=1e-11)
    np.testing.assert_allclose(res["nu"], np.linalg.norm(T, axis=1), rtol=1e-14)
    assert abs(res["achieved"] - ach) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_basis_orthonormal_and_certificate(orc, seed):
    rng = np.random.default_rng(10 + seed)
    T = _low_rank_T(rng, 20, 1000, 8, 1e-10)
    tol = 1e-7
    r = orc.greedy(T, tol, 20)
    nr = r["n_r"]
    Z = r["Z"][:nr]
    np.testing.assert_allclose(Z @ Z.T, np.eye(nr), atol=1e-12)
    # certified affine decomposition: || t^s - nu_s Z^T beta^s ||_inf <= eps nu_s
    rec = r["nu"][:, None] * (r["beta"][:, :nr] @ Z)
    err = np.abs(T - rec).max(axis=1)
    assert np.all(err <= tol * r["nu"] * (1 + 1e-6) + 1e-15)
    assert r["achieved"] <= tol
    assert nr <= np.linalg.matrix_rank(T)


def test_max_residual_non_increasing(orc):
    rng = np.random.default_rng(3)
    T = _low_rank_T(rng, 15, 500, 7, 1e-8)
    prev = np.inf
    for cap in range(1, 9):
        r = orc.greedy(T, 1e-12, cap)
        assert r["achieved"] <= prev + 1e-15
        prev = r["achieved"]


def test_identical_cells_one_principal(orc):
    # With zero perturbation every cell of the 4x4 hole lattice sees the same homogeneous
    # compression: one principal cell reproduces every tangent exactly (alpha = 1).
    cfg = L.config(0).with_(pert_amp=0.0)
    keep = L.make_keep(cfg)
    l2g, _, g2bg = orc.dofmap(2, cfg.ncell, cfg.nel, keep)
    uloc = orc.gather_local(L.make_displacement(cfg)[g2bg], l2g)
    # remove the rigid translation each cell sees (u differs by a constant between cells)
    for c in range(cfg.n_cells):
        m = l2g[c] >= 0
        uloc[c][m] -= uloc[c][m][0]
    mu, lam = L.make_material(cfg)
    T = orc.cells_eval(2, cfg.nel, keep, uloc, mu, lam)["T"]
    r = orc.greedy(T, 1e-8, 16)
    assert r["n_r"] == 1
    np.testing.assert_allclose(r["alpha"][:, 0], 1.0, rtol=1e-12)
    # bitwise-identical cells: every ||Delta||_inf ties and the lowest cell index is chosen
    uloc[:] = uloc[0]
    T = orc.cells_eval(2, cfg.nel, keep, uloc, mu, lam)["T"]
    r = orc.greedy(T, 1e-8, 16)
    assert r["n_r"] == 1 and r["S"][0] == 0
    np.testing.assert_array_equal(r["alpha"][:, 0], 1.0)


def test_scaling_invariance(orc):
    rng = np.random.default_rng(5)
    T = _low_rank_T(rng, 10, 400, 5, 1e-9)
    r1 = orc.greedy(T, 1e-6, 10)
    c = rng.uniform(0.1, 10.0, size=10)
    r2 = orc.greedy(T * c[:, None], 1e-6, 10)
    assert r1["n_r"] == r2["n_r"]
    assert list(r1["S"][:r1["n_r"]]) == list(r2["S"][:r2["n_r"]])
    np.testing.assert_allclose(r2["alpha"][:, :r2["n_r"]] * (1 / c[:, None]) * c[r2["S"][:r2["n_r"]]][None, :],
                               r1["alpha"][:, :r1["n_r"]], rtol=1e-8, atol=1e-10)


def test_permutation_equivariance(orc):
    rng = np.random.default_rng(6)
    T = _low_rank_T(rng, 10, 400, 5, 1e-9)
    perm = rng.permutation(10)
    r1 = orc.greedy(T, 1e-6, 10)
    r2 = orc.greedy(T[perm], 1e-6, 10)
    assert [int(perm[s]) for s in r2["S"][:r2["n_r"]]] == list(r1["S"][:r1["n_r"]])


def test_zero_snapshot_never_selected(orc):
    rng = np.random.default_rng(7)
    T = _low_rank_T(rng, 8, 300, 4, 1e-9)
    T[3] = 0.0
    r = orc.greedy(T, 1e-6, 8)
    assert 3 not in list(r["S"][:r["n_r"]])
    assert r["nu"][3] == 0.0
    assert np.all(r["alpha"][3] == 0.0)


def test_cap_warning(orc):
    rng = np.random.default_rng(8)
    T = rng.standard_normal((8, 200))
    r = orc.greedy(T, 1e-12, 3)
    assert r["n_r"] == 3 and r["status"] == orc.W_CAP
    r = orc.greedy(T, 1e-12, 8)
    assert r["n_r"] == 8 and r["status"] == orc.OK


@pytest.mark.parametrize("seed", range(4))
def test_alpha_is_least_squares(orc, seed):
    rng = np.random.default_rng(20 + seed)
    T = _low_rank_T(rng, 14, 600, 6, 1e-6)
    r = orc.greedy(T, 1e-4, 14)
    nr = r["n_r"]
    TS = T[r["S"][:nr]].T
    ls = np.linalg.lstsq(TS, T.T, rcond=None)[0].T
    np.testing.assert_allclose(r["alpha"][:, :nr], ls, rtol=1e-9, atol=1e-10)
    for k, s in enumerate(r["S"][:nr]):
        e = np.zeros(nr); e[k] = 1.0
        np.testing.assert_allclose(r["alpha"][s, :nr], e, atol=1e-12)


@pytest.mark.parametrize("n", [1, 255, 256, 257, 1000, 5000, 65536 * 2 + 17])
def test_fixed_order_dot(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n); y = rng.standard_normal(n)
    exact = math.fsum(x * y)   # products are not exact, but the error bound below covers it
    d = orc.dot(x, y)
    bound = (256 + math.ceil(math.log2(max(n / 256, 1))) + 2) * 2.0 ** -53 * float(np.abs(x * y).sum())
    assert abs(d - exact) <= bound
    # the same order reproduced by hand: chunk sums with an exactly rounded fused multiply-add
    # (Fraction arithmetic rounded once by float()), then the pairwise tree of chunk sums
    if n > 5000:
        return
    from fractions import Fraction
    parts = []
    for b in range(0, n, 256):
        s = 0.0
        for j in range(b, min(b + 256, n)):
            s = float(Fraction(float(x[j])) * Fraction(float(y[j])) + Fraction(s))
        parts.append(s)
    while len(parts) > 1:
        parts = [parts[2 * k] + parts[2 * k + 1] for k in range(len(parts) // 2)] + \
                ([parts[-1]] if len(parts) % 2 else [])
    assert d == parts[0]
