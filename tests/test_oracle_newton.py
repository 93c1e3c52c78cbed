"""Pins of the oracle's load-stepped Newton-Raphson (Sec. 2.2.5) against facts it does not compute.

* Armijo's rule (smallest m with the sufficient-decrease inequality) by brute force on scalar
  residuals, including an inadmissible trial.
* The assembled ROM matrix against the C oracle's per-cell combination apply (two independent
  codings of eq. romstiffnessmatrix + eq. residualvector), and its symmetry (the tangent of a
  hyperelastic potential).
* Uniaxial stretch of a solid block on symmetry rollers: an affine field solves the discrete problem
  exactly, with the lateral stretch the root of the neo-Hookean zero-lateral-stress condition
  (plane strain: mu (a - 1/a) + lam ln(a l) / a = 0; 3D with two equal lateral stretches:
  mu (a - 1/a) + lam ln(a^2 l) / a = 0).
* Equilibrium: at the converged state the total energy is stationary along free directions.
* With an exact tangent (tolerance below round-off, all cells principal) Newton converges
  quadratically; the converged state does not depend on the number of load increments.
* After the affine predictor of the first increment, the cells of one column of the graded
  lattice are identical, so the greedy needs exactly one principal cell per column.
* Reduced-quadrature snapshots change the principal set, not the equilibrium reached.
"""
import numpy as np
import pytest
import scipy.optimize as so

import lattice as L
import oracle as O
from oracle import newton as ON


def _graded_case(sub=(4, 4), strain=0.04, shear=0.01):
    cfg = L.config(0).with_(radius=(0.25, 0.35)).with_sub(sub)
    bvp = L.make_bvp(cfg, L.LoadCase("compress_shear", strain, shear, 4))
    mu, lam = L.make_material(cfg)
    P = ON.Problem(2, cfg.ncell_eff, cfg.nel, L.make_keep(cfg), mu, lam, bvp["fixed"], bvp["ubar"])
    return cfg, P


def test_armijo_brute_force():
    # Newton on g(x) = atan(x) from x = 3 overshoots: the full step must be cut.
    x0 = 3.0
    g = np.arctan
    dx = -g(x0) * (1 + x0 * x0)
    phi = lambda s: (abs(g(x0 + s * dx)), None)
    m, s, val, _ = ON.armijo(phi, abs(g(x0)))
    want = next(k for k in range(31) if abs(g(x0 + 0.5 ** k * dx)) <= (1 - 1e-4 * 0.5 ** k) * abs(g(x0)))
    assert m == want and m >= 1 and s == 0.5 ** m
    # an inadmissible first trial is skipped, a good second one is taken
    vals = {1.0: np.inf, 0.5: 0.1}
    m, s, val, _ = ON.armijo(lambda s: (vals.get(s, 5.0), None), 1.0)
    assert (m, s, val) == (1, 0.5, 0.1)
    # the sufficient-decrease factor is (1 - c s): 0.99995 passes at s = 0.5, 0.99996 does not
    assert ON.armijo(lambda s: (0.99995 if s == 0.5 else 2.0, None), 1.0)[0] == 1
    assert ON.armijo(lambda s: (0.99996 if s == 0.5 else 2.0, None), 1.0, max_bt=1) is None


def test_rom_matrix_matches_combination_apply():
    cfg = L.config(0).with_sub((3, 2))
    keep = L.make_keep(cfg)
    l2g, _, g2bg = O.dofmap(2, cfg.ncell_eff, cfg.nel, keep)
    ub = L.make_displacement(cfg)
    uglob = ub[g2bg]
    T = O.cells_eval(2, cfg.nel, keep, O.gather_local(uglob, l2g), 1.0, 10.0, want_f=False, want_energy=False)["T"]
    g = O.greedy(T, 1e-3, 6)
    S = g["S"][:g["n_r"]]
    K = ON.rom_matrix(2, cfg.nel, T[S], g["alpha"], l2g, g2bg.size)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((g2bg.size, 2))
    y1 = (K @ x.ravel()).reshape(-1, 2)
    Xl = O.gather_local(x, l2g)[..., None]
    y2 = O.assemble(O.combo_apply(2, cfg.nel, T[S], g["alpha"], l2g, Xl)[..., 0], l2g, g2bg.size)
    assert np.abs(y1 - y2).max() <= 1e-12 * np.abs(y2).max()
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_uniaxial_roller_closed_form(dim):
    if dim == 2:
        ncell, nel, cfg0, rad, lam = (2, 2), 4, 0, (0.0, 0.0), 10.0
    else:
        ncell, nel, cfg0, rad, lam = (2, 2, 2), 2, 2, (2.0, 2.0), 5.0
    cfg = L.config(cfg0).with_(ncell=ncell, nel=nel, radius=rad)
    keep = L.make_keep(cfg)
    assert keep.all()
    mu, l3 = 1.0, 0.9
    bvp = L.make_bvp(cfg, L.LoadCase("uniaxial_roller", 1.0 - l3))
    P = ON.Problem(dim, ncell, nel, keep, mu, lam, bvp["fixed"], bvp["ubar"])
    out = ON.newton_solve(P, n_inc=4, rb_tol=1e-8, cap=8, newton_tol=1e-12)
    assert out["status"] == O.OK
    assert all(r["n_r"] == 1 for r in out["records"])       # homogeneous state: every cell alike
    nlat = dim - 1
    a = so.brentq(lambda a: mu * (a - 1 / a) + lam * np.log(a ** nlat * l3) / a, 0.5, 2.0, xtol=1e-15)
    shp = [c * nel + 1 for c in ncell]
    X = np.zeros((P.ng, dim))
    r = P.g2bg.copy()
    for ax in range(dim):
        X[:, ax] = (r % shp[ax]) / nel
        r //= shp[ax]
    uex = X * (a - 1)
    uex[:, -1] = X[:, -1] * (l3 - 1)
    assert np.abs(out["u"] - uex).max() <= 1e-11


@pytest.fixture(scope="module")
def exact_graded():
    cfg, P = _graded_case()
    out = ON.newton_solve(P, n_inc=4, rb_tol=1e-13, cap=16, newton_tol=1e-10)
    return cfg, P, out


def test_equilibrium_is_energy_stationary(exact_graded):
    cfg, P, out = exact_graded
    assert out["status"] == O.OK
    u = out["u"]
    rng = np.random.default_rng(5)
    v = rng.standard_normal(u.shape)
    v[P.fixed] = 0.0
    h = 1e-6
    d_sol = (P.total_energy(u + h * v, 1.0) - P.total_energy(u - h * v, 1.0)) / (2 * h)
    # the same derivative at the predictor state of the last increment is far from zero
    u_pred = u - P.ubar / 4
    d_pred = (P.total_energy(u_pred + h * v, 1.0) - P.total_energy(u_pred - h * v, 1.0)) / (2 * h)
    assert abs(d_pred) > 1e-3
    assert abs(d_sol) <= 1e-6 * abs(d_pred)


def test_exact_tangent_converges_quadratically(exact_graded):
    cfg, P, out = exact_graded
    recs = out["records"]
    assert all(r["backtracks"] == 0 for r in recs)
    for t in range(1, 5):
        e = [r["res_after"] / r["res0"] for r in recs if r["increment"] == t]
        assert len(e) <= 4
        for k in range(len(e) - 1):
            if e[k] < 1e-2:
                assert e[k + 1] <= 10.0 * e[k] ** 2 + 1e-13


def test_load_path_independence(exact_graded):
    cfg, P, out4 = exact_graded
    out2 = ON.newton_solve(P, n_inc=2, rb_tol=1e-13, cap=16, newton_tol=1e-10)
    assert out2["status"] == O.OK
    assert np.abs(out2["u"] - out4["u"]).max() <= 1e-8 * np.abs(out4["u"]).max()


def test_first_iteration_one_principal_cell_per_column():
    cfg, P = _graded_case()
    out = ON.newton_solve(P, n_inc=4, rb_tol=1e-4, cap=16, max_newton=1)
    first = out["records"][0]
    assert first["increment"] == 1 and first["iteration"] == 0
    assert first["n_r"] == cfg.ncell_eff[0]
    assert first["achieved"] <= 1e-12


def test_reduced_snapshots_reach_the_same_equilibrium(exact_graded):
    # Reduced-quadrature snapshots (eq. snapshots) only change which cells are principal and
    # their coefficients; the residual stays exact, so the converged state is the same.
    cfg, P_full, out_full = exact_graded
    mu, lam = L.make_material(cfg)
    bvp = L.make_bvp(cfg, L.LoadCase("compress_shear", 0.04, 0.01, 4))
    P = ON.Problem(2, cfg.ncell_eff, cfg.nel, L.make_keep(cfg), mu, lam, bvp["fixed"], bvp["ubar"],
                   rule=O.RULE_REDUCED)
    out = ON.newton_solve(P, n_inc=4, rb_tol=1e-4, cap=16, newton_tol=1e-10)
    assert out["status"] == O.OK
    assert any(r["n_r"] < 16 for r in out["records"])
    assert np.abs(out["u"] - out_full["u"]).max() <= 1e-10 * np.abs(out_full["u"]).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_coarse_prolongation_is_q1_interpolation(dim):
    # Q1 interpolation on the cell-corner grid: a partition of unity, exact on affine fields,
    # and equal to the corner value at every corner node.
    cfg = L.config(0 if dim == 2 else 2).with_(ncell=(3, 2) if dim == 2 else (2, 2, 2), nel=4)
    keep = L.make_keep(cfg)
    l2g, _, g2bg = O.dofmap(dim, cfg.ncell, cfg.nel, keep)
    P = ON.coarse_prolongation(dim, cfg.ncell, cfg.nel, g2bg)
    nc = P.shape[1] // dim
    np.testing.assert_allclose(np.asarray(P.sum(axis=1)).ravel(), dim * 0 + 1.0, rtol=0, atol=1e-15)
    cs = [c + 1 for c in cfg.ncell]
    Xc = np.zeros((nc, dim))
    r = np.arange(nc)
    for ax in range(dim):
        Xc[:, ax] = r % cs[ax]
        r //= cs[ax]
    gs = [c * cfg.nel + 1 for c in cfg.ncell]
    Xf = np.zeros((g2bg.size, dim))
    r = g2bg.copy()
    for ax in range(dim):
        Xf[:, ax] = (r % gs[ax]) / cfg.nel
        r //= gs[ax]
    A = np.arange(1, dim * dim + 1).reshape(dim, dim) / 7.0
    b = np.arange(dim) - 0.5
    uc = Xc @ A.T + b
    uf = (P @ uc.ravel()).reshape(-1, dim)
    np.testing.assert_allclose(uf, Xf @ A.T + b, rtol=0, atol=1e-13)


def test_coarse_operator_kills_translations_and_is_galerkin():
    # No prescribed components: rigid translations lie in the kernel of every cell tangent at
    # u = 0, and P maps coarse translations to fine translations, so K_0 annihilates them.
    cfg = L.config(0).with_(ncell=(3, 2), nel=8, radius=(0.25, 0.35))
    keep = L.make_keep(cfg)
    l2g, _, g2bg = O.dofmap(2, cfg.ncell, cfg.nel, keep)
    ul = np.zeros((cfg.n_cells, (cfg.nel + 1) ** 2, 2))
    T = O.cells_eval(2, cfg.nel, keep, ul, 1.0, 10.0, want_f=False, want_energy=False)["T"]
    g = O.greedy(T, 1e-10, 6)
    K = ON.rom_matrix(2, cfg.nel, T[g["S"][:g["n_r"]]], g["alpha"], l2g, g2bg.size)
    P = ON.coarse_prolongation(2, cfg.ncell, cfg.nel, g2bg)
    K0 = ON.coarse_operator(K, P)
    assert np.abs(K0 - K0.T).max() <= 1e-12 * np.abs(K0).max()
    nc = K0.shape[0] // 2
    for i in range(2):
        t = np.zeros((nc, 2)); t[:, i] = 1.0
        assert np.abs(K0 @ t.ravel()).max() <= 1e-11 * np.abs(K0).max()
    rng = np.random.default_rng(3)
    a, c = rng.standard_normal(2 * nc), rng.standard_normal(2 * nc)
    assert abs(a @ K0 @ c - (P @ a) @ (K @ (P @ c))) <= 1e-11 * np.abs(K0).max() * 2 * nc


def test_sampled_snapshots_reach_the_same_equilibrium(exact_graded):
    # Snapshots of sampled tangent entries change the principal cells, never the residual.
    cfg, P_full, out_full = exact_graded
    mu, lam = L.make_material(cfg)
    bvp = L.make_bvp(cfg, L.LoadCase("compress_shear", 0.04, 0.01, 4))
    P = ON.Problem(2, cfg.ncell_eff, cfg.nel, L.make_keep(cfg), mu, lam, bvp["fixed"], bvp["ubar"],
                   rule=O.RULE_SAMPLED)
    out = ON.newton_solve(P, n_inc=4, rb_tol=1e-4, cap=16, newton_tol=1e-10)
    assert out["status"] == O.OK
    assert np.abs(out["u"] - out_full["u"]).max() <= 1e-10 * np.abs(out_full["u"]).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_material_snapshots_at_rest_are_the_elasticity_tensor(dim):
    # At u = 0 every kept element carries the isotropic tensor
    # C_iJkL = lam d_iJ d_kL + mu (d_ik d_JL + d_iL d_Jk); elements that are not kept carry zeros.
    cfg = L.config(0 if dim == 2 else 2).with_(ncell=(2, 1) if dim == 2 else (1, 1, 1), nel=4 if dim == 2 else 3)
    keep = L.make_keep(cfg)
    keep[0, 0] = 0
    Ns = keep.shape[0]
    mu, lam = 1.3, 7.0
    T, st = O.material_snapshots(dim, cfg.nel, keep, np.zeros((Ns, (cfg.nel + 1) ** dim, dim)), mu, lam)
    assert st == O.OK
    I = np.eye(dim)
    C = (lam * np.einsum("ij,kl->ijkl", I, I) + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))
    d4 = dim ** 4
    for s in range(Ns):
        for e in range(cfg.nel ** dim):
            blk = T[s, e * d4:(e + 1) * d4]
            np.testing.assert_allclose(blk, C.reshape(-1) if keep[s, e] else 0.0, rtol=0, atol=1e-13)
    assert not T[:, cfg.nel ** dim * d4:].any()


def test_material_snapshots_follow_a_homogeneous_stretch():
    # An affine displacement gives the same F in every element: the snapshot block is the oracle's
    # tangent at that F, and a cell with every element kept has N_s identical blocks.
    cfg = L.config(0).with_(ncell=(1, 1), nel=4, radius=(0.0, 0.0))
    keep = L.make_keep(cfg)
    F = np.array([[1.05, 0.02], [-0.01, 0.93]])
    nn = cfg.nel + 1
    a = np.arange(nn * nn)
    X = np.stack([a % nn, a // nn], 1) / cfg.nel
    u = (X @ (F - np.eye(2)).T)[None]
    T, st = O.material_snapshots(2, cfg.nel, keep, u, 1.0, 10.0)
    F3 = np.eye(3); F3[:2, :2] = F
    A = O.neo_hooke(F3, 1.0, 10.0)[2][:2, :2, :2, :2].reshape(-1)
    for e in range(cfg.nel ** 2):
        np.testing.assert_allclose(T[0, e * 16:(e + 1) * 16], A, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim,nel", [(2, 6), (3, 3)])
def test_sampled_snapshots_are_force_derivatives_at_sampled_nodes(dim, nel):
    # some_data(K): every stored entry (j, o, i, c) is d f_(a_j, i) / d u_(a_j + o, c) of the cell's
    # internal force at the j-th node of the stride-2 sub-grid, by central differences of the force
    # alone; neighbours outside the cell give zeros, and the rows past the sampled nodes are zero.
    rng = np.random.default_rng(4)
    nn = nel + 1
    nloc = nn ** dim
    if dim == 2:
        keep = np.ones(nel * nel, np.uint8); keep[[nel + 2, 2 * nel + 5]] = 0
    else:
        keep = (rng.random(nel ** 3) < 0.8).astype(np.uint8)
    u = 0.02 * rng.standard_normal((nloc, dim))
    mu, lam = 1.2, 6.0
    T_full = O.cells_eval(dim, nel, keep[None], u[None], mu, lam, want_f=False, want_energy=False)["T"]
    T = O.sampled_snapshots(dim, nel, T_full)[0]
    nodes = O.sampled_nodes(dim, nel)
    assert len(nodes) == (nel // 2 + 1) ** dim and nodes[1] == 2 and nodes == sorted(nodes)
    # every element has exactly one corner on the sub-grid, so every element enters the snapshot
    for e in range(nel ** dim):
        ce = [(e // nel ** ax) % nel for ax in range(dim)]
        on = [c for c in range(2 ** dim)
              if sum((ce[ax] + ((c >> ax) & 1)) * nn ** ax for ax in range(dim)) in set(nodes)]
        assert len(on) == 1
    E = 3 ** dim * dim * dim
    h = 1e-6
    fd = {}
    for j, a in enumerate(nodes):
        ca = [(a // nn ** ax) % nn for ax in range(dim)]
        for o in range(3 ** dim):
            off = [(o // 3 ** ax) % 3 - 1 for ax in range(dim)]
            cb = [ca[ax] + off[ax] for ax in range(dim)]
            inside = all(0 <= cb[ax] < nn for ax in range(dim))
            for c in range(dim):
                blk = np.array([T[j * E + (o * dim + i) * dim + c] for i in range(dim)])
                if not inside:
                    assert not blk.any()
                    continue
                b = sum(cb[ax] * nn ** ax for ax in range(dim))
                if (b, c) not in fd:
                    up = u.copy(); up[b, c] += h
                    um = u.copy(); um[b, c] -= h
                    fd[(b, c)] = (O.cell_eval(dim, nel, keep, up, mu, lam)["f"]
                                  - O.cell_eval(dim, nel, keep, um, mu, lam)["f"]) / (2 * h)
                np.testing.assert_allclose(blk, fd[(b, c)][a], rtol=0, atol=1e-7 * np.abs(T).max())
    assert not T[len(nodes) * E:].any()


def test_sampled_snapshots_at_stride_one_are_the_full_snapshots():
    cfg = L.config(0).with_(ncell=(2, 2), nel=4)
    keep = L.make_keep(cfg)
    u = 0.01 * np.random.default_rng(2).standard_normal((4, 25, 2))
    T_full = O.cells_eval(2, 4, keep, u, 1.0, 10.0, want_f=False, want_energy=False)["T"]
    np.testing.assert_array_equal(O.sampled_snapshots(2, 4, T_full, stride=1), T_full)
    assert O.sampled_nodes(2, 4, stride=4) == [0, 4, 20, 24]
