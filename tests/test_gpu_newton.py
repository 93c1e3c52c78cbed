"""GPU parity of the nonlinear solve (Sec. 2.2.5): the ROM tangent solve and the load-stepped
Newton-Raphson with Armijo backtracking, through the C ABI, against the FP64 oracle.

Tolerances.  The tangent solve (preconditioned MINRES, D = |diag K~|) stops at
||r||_{D^-1} <= 1e-12 ||b||_{D^-1}; in the 2-norm that is 1e-12 times sqrt(max D / min D) (< 10
here), hence the 1e-10 bound on the oracle's residual of the GPU solution, and its error
against the oracle's exact sparse solve is at most cond(K~) times that.  On the 4x4 graded hole
lattice (n = 16) at 1% compression cond(K~) is 5.6e4, hence the 1e-6 bound on the solution; at
3% uniform compression the tangent of this lattice is indefinite (one eigenvalue -7.8e-4 of a
spectrum reaching 51), which MINRES solves as well.  In the Newton comparison both sides take
the same iterations; the per-step solve errors (<= 1e-7 relative) change each accepted residual
by at most that fraction of the residual before the step.
"""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse.linalg as spla
import torch

import lattice as L
import oracle as O
from oracle import newton as ON
from gpu_common import rel

pytestmark = pytest.mark.gpu


class NCase:
    """A lattice with Dirichlet data on both sides."""

    def __init__(self, cfg, case, keep=None, mu=None, lam=None, cap=16):
        from paper_2603_10741_amd import binding as B
        self.B = B
        self.cfg = cfg
        self.dev = torch.device("cuda:0")
        self.keep = L.make_keep(cfg) if keep is None else keep
        mu0, lam0 = L.make_material(cfg)
        self.mu = mu0 if mu is None else np.broadcast_to(mu, mu0.shape).copy()
        self.lam = lam0 if lam is None else np.broadcast_to(lam, lam0.shape).copy()
        self.bvp = L.make_bvp(cfg, case)
        self.case = case
        print(f"[newton case] {cfg.name} ncell={cfg.ncell_eff} nel={cfg.nel} {case}", flush=True)
        self.P = B.Plan(cfg.dim, cfg.ncell_eff, cfg.nel, self.keep, cap=cap)
        _, _, g2bg, _ = self.P.dofmap()
        g2bg = g2bg.cpu().numpy()
        self.fixed_t = torch.from_numpy(np.ascontiguousarray(self.bvp["fixed"][g2bg])).to(self.dev)
        self.ubar_t = torch.from_numpy(np.ascontiguousarray(self.bvp["ubar"][g2bg])).to(self.dev)
        self.mu_t = torch.from_numpy(np.ascontiguousarray(self.mu)).to(self.dev)
        self.lam_t = torch.from_numpy(np.ascontiguousarray(self.lam)).to(self.dev)
        self.orc = ON.Problem(cfg.dim, cfg.ncell_eff, cfg.nel, self.keep, self.mu, self.lam, self.bvp["fixed"],
                              self.bvp["ubar"])
        assert np.array_equal(self.orc.g2bg, g2bg)

    def zeros_u(self):
        return torch.zeros(self.P.nglobal, self.cfg.dim, dtype=torch.float64, device=self.dev)


def graded_cfg():
    return L.config(0).with_(radius=(0.25, 0.35))


@pytest.fixture(scope="module")
def graded():
    return NCase(graded_cfg(), L.LoadCase("compress_shear", 0.04, 0.01, 4))


def _rom_at(nc, u_glob, tol, cap):
    """GPU: snapshots at u, greedy, principal tangents.  Oracle: the same from its own pieces."""
    P = nc.P
    u_t = torch.from_numpy(np.ascontiguousarray(u_glob)).to(nc.dev)
    out = P.residual_tangent(u_t, nc.mu_t, nc.lam_t, f=False, energy=False, snap=True)
    sel = P.select_principal(out["snap"], tol, cap=cap)
    n_r = int(sel["n_r"].item())
    K = P.principal_ops(u_t, nc.mu_t, nc.lam_t, sel["S"], n_r)["K"]
    _, T, st, _ = nc.orc.evaluate(u_glob, 1.0)
    g = O.greedy(T, tol, cap, keep_Z=False)
    assert g["n_r"] == n_r
    Ko = ON.rom_matrix(nc.cfg.dim, nc.cfg.nel, T[g["S"][:n_r]], g["alpha"], nc.orc.l2g, nc.orc.ng)
    return K, n_r, sel["alpha"], Ko


def test_rom_solve_matches_direct_solve(graded):
    nc = graded
    cfg = nc.cfg
    u = L.make_displacement(cfg.with_(strain=0.01, pert_amp=1e-3))[nc.orc.g2bg]
    K, n_r, alpha, Ko = _rom_at(nc, u, 1e-4, 16)
    rng = np.random.default_rng(21)
    b = rng.standard_normal((nc.P.nglobal, cfg.dim))
    b_t = torch.from_numpy(b).to(nc.dev)
    x, st, its, rr = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, b_t, tol=1e-12, maxit=50000, check=64)
    assert st == nc.B.LAT_OK and rr <= 1e-12 and its > 0
    x = x.reshape(-1, cfg.dim).cpu().numpy()
    f = nc.orc.free
    bf = b.ravel()[f]
    xo = np.zeros(b.size)
    xo[f] = spla.spsolve(Ko[f][:, f].tocsc(), bf)
    assert np.all(x.ravel()[~f] == 0.0)
    assert np.linalg.norm(Ko[f][:, f] @ x.ravel()[f] - bf) <= 1e-10 * np.linalg.norm(bf)
    assert rel(x.ravel(), xo) <= 1e-6
    # the same solve again is bit-identical (fixed-order reductions)
    x2, _, its2, _ = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, b_t, tol=1e-12, maxit=50000, check=64)
    assert its2 == its and np.array_equal(x2.reshape(-1, cfg.dim).cpu().numpy(), x)
    # products formed on the fly by the ROM apply instead of from the combined stencils
    x3, st3, _, rr3 = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, b_t, tol=1e-12, maxit=50000, check=64,
                                     materialize=False)
    assert st3 == nc.B.LAT_OK and rr3 <= 1e-12
    assert rel(x3.reshape(-1, cfg.dim).cpu().numpy().ravel(), xo) <= 1e-6


def test_rom_solve_edge_cases(graded):
    nc = graded
    cfg = nc.cfg
    u = L.make_displacement(cfg.with_(strain=0.005, pert_amp=1e-3))[nc.orc.g2bg]
    K, n_r, alpha, _ = _rom_at(nc, u, 1e-3, 16)
    B = nc.B
    zero = torch.zeros(nc.P.nglobal, cfg.dim, dtype=torch.float64, device=nc.dev)
    x, st, its, rr = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, zero)
    assert st == B.LAT_OK and its == 0 and rr == 0.0 and torch.count_nonzero(x).item() == 0
    # b supported on prescribed components only is the zero right-hand side
    b = nc.fixed_t.to(torch.float64) * 3.0
    x, st, its, _ = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, b)
    assert st == B.LAT_OK and its == 0 and torch.count_nonzero(x).item() == 0
    rng = np.random.default_rng(22)
    bt = torch.from_numpy(rng.standard_normal((nc.P.nglobal, cfg.dim))).to(nc.dev)
    # iteration limit
    x, st, its, rr = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, bt, tol=1e-14, maxit=5, check=2)
    assert st == B.LAT_E_NOCONV and its == 5 and rr > 1e-14
    # a negative definite operator (coefficients negated): the solution changes sign
    xp, st, _, _ = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, bt, tol=1e-12, maxit=50000)
    assert st == B.LAT_OK
    xn, st, _, _ = nc.P.rom_solve(K, n_r, (-alpha).contiguous(), nc.fixed_t, bt, tol=1e-12, maxit=50000)
    assert st == B.LAT_OK
    assert rel(xn.cpu().numpy(), -xp.cpu().numpy()) <= 1e-8
    # the zero operator is singular on the first Krylov vector
    x, st, its, _ = nc.P.rom_solve(K, n_r, torch.zeros_like(alpha), nc.fixed_t, bt)
    assert st == B.LAT_E_SINGULAR and its == 0 and torch.count_nonzero(x).item() == 0


def test_rom_solve_indefinite_matches_direct_solve(graded):
    nc = graded
    cfg = nc.cfg
    u = L.make_displacement(cfg.with_(strain=0.03, pert_amp=2e-3))[nc.orc.g2bg]
    K, n_r, alpha, Ko = _rom_at(nc, u, 1e-4, 16)
    f = nc.orc.free
    Kf = Ko[f][:, f]
    lo = spla.eigsh(Kf, k=1, sigma=-1e-3, which="LM", return_eigenvectors=False)[0]
    assert lo < 0.0                                      # the case is indefinite indeed
    rng = np.random.default_rng(23)
    b = rng.standard_normal((nc.P.nglobal, cfg.dim))
    x, st, its, rr = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, torch.from_numpy(b).to(nc.dev), tol=1e-12,
                                    maxit=100000, check=128)
    assert st == nc.B.LAT_OK and rr <= 1e-12
    x = x.reshape(-1, cfg.dim).cpu().numpy().ravel()
    bf = b.ravel()[f]
    xo = np.zeros(b.size)
    xo[f] = spla.spsolve(Kf.tocsc(), bf)
    assert np.linalg.norm(Kf @ x[f] - bf) <= 1e-10 * np.linalg.norm(bf)
    assert rel(x, xo) <= 1e-5


@pytest.mark.parametrize("rule", [O.RULE_FULL, O.RULE_REDUCED, O.RULE_MATERIAL, O.RULE_SAMPLED])
def test_newton_matches_oracle(graded, rule):
    nc = graded
    u = nc.zeros_u()
    st, recs = nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, nc.ubar_t, u, n_inc=4, rb_tol=1e-4, cap=16,
                                 cg_tol=1e-12, cg_maxit=50000, snap_rule=rule)
    assert st == nc.B.LAT_OK
    orc = nc.orc if rule == O.RULE_FULL else ON.Problem(
        nc.cfg.dim, nc.cfg.ncell_eff, nc.cfg.nel, nc.keep, nc.mu, nc.lam, nc.bvp["fixed"], nc.bvp["ubar"], rule=rule)
    out = ON.newton_solve(orc, n_inc=4, rb_tol=1e-4, cap=16)
    assert out["status"] == O.OK
    ro = out["records"]
    assert len(recs) == len(ro)
    for g, o in zip(recs, ro):
        assert (g["increment"], g["iteration"], g["n_r"], g["backtracks"]) == \
               (o["increment"], o["iteration"], o["n_r"], o["backtracks"])
        assert g["cg_status"] == nc.B.LAT_OK and g["cg_relres"] <= 1e-12
        assert abs(g["res0"] - o["res0"]) <= 1e-9 * o["res0"]
        assert abs(g["res_before"] - o["res_before"]) <= 1e-6 * o["res0"]
        assert abs(g["res_after"] - o["res_after"]) <= 1e-6 * o["res_before"]
        assert g["res_after"] <= (1 - 1e-4 * g["step"]) * g["res_before"]
    uo = out["u"]
    ug = u.cpu().numpy()
    assert np.abs(ug - uo).max() <= 1e-7 * np.abs(uo).max()
    # the prescribed components take the same four predictor additions on both sides (the
    # Newton corrections vanish there), so they agree bit for bit and carry the full load
    fx = nc.orc.fixed
    np.testing.assert_array_equal(ug[fx], uo[fx])
    assert np.abs(ug[fx] - nc.orc.ubar[fx]).max() <= 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_newton_uniaxial_closed_form(dim):
    # 2D: products from the combined stencils; 3D: ROM applies forming them on the fly
    if dim == 2:
        cfg = L.config(0).with_(ncell=(3, 2), nel=8, radius=(0.0, 0.0))
        lam = 10.0
    else:
        cfg = L.config(2).with_(ncell=(2, 2, 2), nel=4, radius=(2.0, 2.0))
        lam = 5.0
    mu, l3 = 1.0, 0.88
    nc = NCase(cfg, L.LoadCase("uniaxial_roller", 1.0 - l3, 0.0, 4), mu=mu, lam=lam, cap=8)
    assert nc.keep.all()
    u = nc.zeros_u()
    st, recs = nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, nc.ubar_t, u, n_inc=4, rb_tol=1e-8, cap=8,
                                 newton_tol=1e-11, cg_tol=1e-13, cg_maxit=50000, matvec=dim - 2)
    summary = [(r["increment"], r["iteration"], r["n_r"], r["rb_achieved"], r["backtracks"], r["cg_iters"],
                r["cg_status"], r["res_after"] / r["res0"]) for r in recs]
    assert st == nc.B.LAT_OK, summary
    assert all(r["n_r"] == 1 and r["backtracks"] == 0 for r in recs), summary
    a = so.brentq(lambda a: mu * (a - 1 / a) + lam * np.log(a ** (dim - 1) * l3) / a, 0.5, 2.0, xtol=1e-15)
    shp = [c * cfg.nel + 1 for c in cfg.ncell_eff]
    X = np.zeros((nc.P.nglobal, dim))
    r = nc.orc.g2bg.copy()
    for ax in range(dim):
        X[:, ax] = (r % shp[ax]) / cfg.nel
        r //= shp[ax]
    uex = X * (a - 1)
    uex[:, -1] = X[:, -1] * (l3 - 1)
    assert np.abs(u.cpu().numpy() - uex).max() <= 1e-9


def test_newton_degenerate_loads(graded):
    nc = graded
    B = nc.B
    # no load: nothing to do, the state is unchanged
    u = nc.zeros_u()
    st, recs = nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, torch.zeros_like(nc.ubar_t), u)
    assert st == B.LAT_OK and recs == [] and torch.count_nonzero(u).item() == 0
    # a predictor that inverts elements is refused with the device status
    u = nc.zeros_u()
    st, recs = nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, (nc.ubar_t * 60.0).contiguous(), u, n_inc=1)
    assert st == B.LAT_E_INVERTED and recs == []
    # iteration limit: one Newton iteration per increment is not enough
    u = nc.zeros_u()
    st, recs = nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, nc.ubar_t, u, max_newton=1, rb_tol=1e-4, cap=16,
                                 cg_tol=1e-12, cg_maxit=50000)
    assert st == B.LAT_E_NOCONV and len(recs) == 1 and recs[0]["increment"] == 1
    # invalid options are rejected on the host
    with pytest.raises(B.LatError):
        nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, nc.ubar_t, u, armijo_beta=1.0)
    with pytest.raises(B.LatError):
        nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, nc.ubar_t, u, cap=nc.P.cap + 1)


@pytest.fixture(scope="module")
def two_groups():
    # 12 x 8 = 96 cells: two 64-lane groups, so the packed layout spans group offsets
    cfg = L.config(0).with_(ncell=(12, 8), radius=(0.25, 0.35))
    return NCase(cfg, L.LoadCase("compress_shear", 0.02, 0.005, 2), cap=64)


def test_rom_solve_two_groups(two_groups):
    nc = two_groups
    cfg = nc.cfg
    assert nc.P.ngroups == 2
    u = L.make_displacement(cfg.with_(strain=0.005, pert_amp=1e-3))[nc.orc.g2bg]
    K, n_r, alpha, Ko = _rom_at(nc, u, 1e-4, 64)
    rng = np.random.default_rng(24)
    xs = rng.standard_normal((nc.P.nglobal, cfg.dim))
    xs[nc.orc.fixed] = 0.0
    b = (Ko @ xs.ravel()).reshape(-1, cfg.dim)
    b[nc.orc.fixed] = 0.0
    for mat in (True, False):
        x, st, its, rr = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, torch.from_numpy(b).to(nc.dev), tol=1e-12,
                                        maxit=100000, check=128, materialize=mat)
        assert st == nc.B.LAT_OK and rr <= 1e-12
        f = nc.orc.free
        xg = x.reshape(-1, cfg.dim).cpu().numpy().ravel()
        assert np.linalg.norm(Ko[f][:, f] @ xg[f] - b.ravel()[f]) <= 1e-10 * np.linalg.norm(b)
        assert rel(xg, xs.ravel()) <= 1e-5


def test_newton_two_groups_matches_oracle(two_groups):
    nc = two_groups
    # ROM at a tolerance where it keeps the exact Newton's iteration count on this lattice (N_r 47-58
    # of 96), then the standard method (every cell's own tangent: the ROM with all cells principal)
    for tangent, tol in ((0, 3e-5), (1, None)):
        u = nc.zeros_u()
        st, recs = nc.P.newton_solve(nc.mu_t, nc.lam_t, nc.fixed_t, nc.ubar_t, u, n_inc=2, rb_tol=tol or 1e-4, cap=64,
                                     cg_tol=1e-12, cg_maxit=100000, tangent=tangent)
        assert st == nc.B.LAT_OK
        out = ON.newton_solve(nc.orc, n_inc=2, rb_tol=tol if tol else 1e-14, cap=64 if tol else 96)
        assert out["status"] == O.OK
        ro = out["records"]
        assert len(recs) == len(ro)
        for g, o in zip(recs, ro):
            assert (g["increment"], g["iteration"], g["backtracks"]) == (o["increment"], o["iteration"], o["backtracks"])
            assert g["n_r"] == (o["n_r"] if tangent == 0 else 0)
            assert abs(g["res_after"] - o["res_after"]) <= 1e-6 * o["res_before"]
        assert np.abs(u.cpu().numpy() - out["u"]).max() <= 1e-7 * np.abs(out["u"]).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_coarse_operator_matches_oracle(dim):
    # K0 = P^T K~ P over the cell-corner nodes, against the oracle's sparse ROM matrix and Q1
    # prolongation (prescribed rows removed)
    if dim == 2:
        cfg = L.config(0).with_(radius=(0.25, 0.35))
        case = L.LoadCase("compress_shear", 0.04, 0.01, 4)
    else:
        cfg = L.config(2).with_(ncell=(2, 2, 2), nel=6)
        case = L.LoadCase("compress_shear", 0.02, 0.005, 4)
    nc = NCase(cfg, case, cap=16)
    u = L.make_displacement(cfg.with_(strain=0.01, pert_amp=1e-3))[nc.orc.g2bg]
    K, n_r, alpha, Ko = _rom_at(nc, u, 1e-4, 16)
    Pc = ON.coarse_prolongation(dim, cfg.ncell_eff, cfg.nel, nc.orc.g2bg, nc.orc.fixed)
    K0o = ON.coarse_operator(Ko, Pc)
    for mat in (True, False):
        K0 = nc.P.coarse_operator(K, n_r, alpha, nc.fixed_t, materialize=mat).cpu().numpy()
        assert np.abs(K0 - K0o).max() <= 1e-11 * np.abs(K0o).max()


def test_rom_solve_two_level(graded):
    nc = graded
    cfg = nc.cfg
    u = L.make_displacement(cfg.with_(strain=0.01, pert_amp=1e-3))[nc.orc.g2bg]
    K, n_r, alpha, Ko = _rom_at(nc, u, 1e-4, 16)
    rng = np.random.default_rng(25)
    b = rng.standard_normal((nc.P.nglobal, cfg.dim))
    b_t = torch.from_numpy(b).to(nc.dev)
    f = nc.orc.free
    xo = np.zeros(b.size)
    xo[f] = spla.spsolve(Ko[f][:, f].tocsc(), b.ravel()[f])
    its = {}
    for pc in (0, 1):
        info = {}
        x, st, it, rr = nc.P.rom_solve(K, n_r, alpha, nc.fixed_t, b_t, tol=1e-12, maxit=50000, check=64, precond=pc,
                                       info=info)
        assert st == nc.B.LAT_OK and rr <= 1e-12
        assert info["coarse_used"] == (pc == 1)
        assert rel(x.reshape(-1, cfg.dim).cpu().numpy().ravel(), xo) <= 1e-6
        its[pc] = it
    assert its[1] < its[0]


@pytest.mark.parametrize("which", ["hole", "bcc"])
def test_material_snapshots_match_oracle(which):
    # the material-tangent snapshots (snap_rule MATERIAL) and the greedy on them
    from gpu_common import Case
    cfg = L.config(0).with_(radius=(0.25, 0.35)) if which == "hole" else L.config(2).with_sub((2, 2, 2))
    c = Case(cfg, m=1)
    P = c.P
    out = P.residual_tangent(c.ug, c.mu_t, c.lam_t, snap_rule=c.B.RULE_MATERIAL, f=False, energy=False, snap=True)
    T = c.canon_T(out["snap"])
    To, st = O.material_snapshots(cfg.dim, cfg.nel, c.keep, c.uloc, c.mu, c.lam)
    assert st == O.OK
    assert rel(T, To) <= 1e-13
    code, _ = P.check_status(allow_cap=True)
    assert code == c.B.LAT_OK
    for tol in (1e-2, 1e-3):
        g = P.select_principal(out["snap"] if tol == 1e-2 else c.to_cil_T(To), tol, keep_Z=False)
        go = O.greedy(To, tol, cfg.cap, keep_Z=False)
        assert int(g["n_r"].item()) == go["n_r"]


@pytest.mark.parametrize("which", ["hole", "bcc"])
def test_sampled_snapshots_are_the_full_rows_of_the_subgrid_nodes(which):
    # snap_rule SAMPLED: the full-rule snapshot's rows of the stride-2 sub-grid nodes, bit for bit,
    # zeros past them; against the oracle's selection of its own full-rule snapshots
    from gpu_common import Case
    cfg = L.config(0).with_(radius=(0.25, 0.35)) if which == "hole" else L.config(2).with_sub((2, 2, 2))
    c = Case(cfg, m=1)
    P = c.P
    full = P.residual_tangent(c.ug, c.mu_t, c.lam_t, snap_rule=c.B.RULE_FULL, f=False, energy=False,
                              snap=True)["snap"].view(P.nsnap, P.ld)
    samp = P.residual_tangent(c.ug, c.mu_t, c.lam_t, snap_rule=c.B.RULE_SAMPLED, f=False, energy=False,
                              snap=True)["snap"].view(P.nsnap, P.ld)
    nodes = O.sampled_nodes(cfg.dim, cfg.nel)
    E = P.E
    rows = P.snapshot_rows(c.B.RULE_SAMPLED)
    assert rows == len(nodes) * E
    for j, a in enumerate(nodes):
        assert torch.equal(samp[j * E:(j + 1) * E], full[a * E:(a + 1) * E]), (j, a)
    assert not samp[rows:].any()
    To = O.sampled_snapshots(cfg.dim, cfg.nel, c.orc["T"])
    assert np.abs(c.canon_T(samp) - To).max() <= 1e-12 * np.abs(To).max()
    code, _ = P.check_status(allow_cap=True)
    assert code == c.B.LAT_OK
    g = P.select_principal(c.to_cil_T(To), 1e-3, keep_Z=False, rows=rows)
    go = O.greedy(To, 1e-3, cfg.cap, keep_Z=False)
    assert int(g["n_r"].item()) == go["n_r"]
    np.testing.assert_array_equal(g["S"].cpu().numpy()[:go["n_r"]], go["S"][:go["n_r"]])


@pytest.mark.parametrize("rule", ["material", "sampled"])
def test_greedy_on_the_data_rows_is_bit_identical(rule):
    # material and sampled snapshots fill only their leading rows; the greedy restricted to them
    # returns the full sweep's outputs bit for bit
    from gpu_common import Case
    cfg = L.config(0).with_(radius=(0.25, 0.35))
    c = Case(cfg, m=1)
    P = c.P
    code = c.B.RULE_MATERIAL if rule == "material" else c.B.RULE_SAMPLED
    rows = P.snapshot_rows(code)
    assert rows == (cfg.n_elems * cfg.dim ** 4 if rule == "material" else (cfg.nel // 2 + 1) ** 2 * P.E)
    outs = []
    for r in (None, rows):
        snap = P.residual_tangent(c.ug, c.mu_t, c.lam_t, snap_rule=code, f=False, energy=False,
                                  snap=True)["snap"]
        g = P.select_principal(snap, 1e-3, keep_Z=True, rows=r)
        outs.append({k: v.cpu().numpy() for k, v in g.items()} | {"delta": snap.cpu().numpy()})
    assert outs[0]["n_r"][0] > 1
    for k in ("S", "n_r", "alpha", "beta", "nu", "R", "Z", "achieved", "delta"):
        assert np.array_equal(outs[0][k], outs[1][k]), k
