"""Load-stepped Newton-Raphson on the ROM tangent: FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by `tests/` and the benchmark's CPU-baseline leg, never by the
product library.  It shares no code with the GPU path.

What it computes (Sec. 2.2.5, Newton-Raphson method; Sec. 3.2, fast assembly):
  * residual r(u) = sum_s A^s f^{int,s}(A^{sT} u) - lf f_ext (eq. residualvector), zero on the
    prescribed components;
  * at every Newton iteration the reduced basis is rebuilt from the snapshots at the current
    state (Algorithm 1, Sec. 3.2.3; full or reduced quadrature, eq. snapshots) and the tangent of
    eq. linsys is replaced by the ROM operator K~ = sum_s A^s M_s (sum_k alpha_sk K_k) M_s A^{sT}
    (eq. romstiffnessmatrix), K_k the full-rule tangents of the principal cells;
  * the tangent system K~ du = -r is solved exactly on the free components (sparse LU);
  * Armijo's rule: the smallest m >= 0 with ||r(u + beta^m du)|| <= (1 - c beta^m) ||r(u)||,
    beta = 1/2, c = 1e-4; an inverted element (J <= 0) at a trial counts as a failed trial;
  * stop when ||r(u_{k+1})|| / ||r(u_0)|| <= 1e-6, u_0 the first iterate of the increment;
  * load increments: increment t adds ubar / n_inc to every node (which carries the
    prescribed components to t/n_inc of their final value) and scales f_ext by t / n_inc.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import (OK, RULE_FULL, RULE_MATERIAL, RULE_SAMPLED, assemble, cells_eval, dofmap, gather_local, greedy,
               material_snapshots, sampled_snapshots)

NOCONV = 8


def neighbour_pairs(dim: int, nel: int):
    """All (a, o, b = a + o) with local nodes a, b inside the cell and offset index
    o = (ox+1) + 3(oy+1) + 9(oz+1)."""
    nn = nel + 1
    nloc = nn ** dim
    a = np.arange(nloc)
    coords = [(a // nn ** ax) % nn for ax in range(dim)]
    A, O, B = [], [], []
    for o in range(3 ** dim):
        off = [(o // 3 ** ax) % 3 - 1 for ax in range(dim)]
        ok = np.ones(nloc, bool)
        b = np.zeros(nloc, np.int64)
        for ax in range(dim):
            c = coords[ax] + off[ax]
            ok &= (c >= 0) & (c <= nel)
            b += c * nn ** ax
        A.append(a[ok]); O.append(np.full(int(ok.sum()), o)); B.append(b[ok])
    return np.concatenate(A), np.concatenate(O), np.concatenate(B)


def rom_matrix(dim, nel, Kp, alpha, l2g, n_global):
    """Global sparse K~ (eq. romstiffnessmatrix assembled by eq. residualvector's A^s).

    Kp [n_r][n_snap] principal stencils, alpha [N_s][>= n_r]; rows/cols (node, component)."""
    n_r = Kp.shape[0]
    Ns, nloc = l2g.shape
    d, no = dim, 3 ** dim
    Kc = (alpha[:, :n_r] @ Kp).reshape(Ns, nloc, no, d, d)      # combined stencil of every cell
    A, O, B = neighbour_pairs(dim, nel)
    ci = np.arange(d)
    rows, cols, vals = [], [], []
    for s in range(Ns):
        ga = l2g[s][A].astype(np.int64)
        gb = l2g[s][B].astype(np.int64)
        ok = (ga >= 0) & (gb >= 0)                               # M_s on both sides
        blk = Kc[s][A[ok], O[ok]]                                # [npair][d][d]
        r = ga[ok][:, None, None] * d + ci[None, :, None]
        c = gb[ok][:, None, None] * d + ci[None, None, :]
        rows.append(np.broadcast_to(r, blk.shape).ravel())
        cols.append(np.broadcast_to(c, blk.shape).ravel())
        vals.append(blk.ravel())
    N = n_global * d
    if not rows:
        return sp.csr_matrix((N, N))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def armijo(phi, phi0, beta=0.5, c=1e-4, max_bt=30):
    """Backtracking (Armijo's rule): the smallest m in [0, max_bt] with phi(beta^m) <= (1 - c beta^m) phi0.

    phi(s) returns (value, payload); value = inf marks an inadmissible trial.
    Returns (m, s, value, payload) or None when no m qualifies."""
    for m in range(max_bt + 1):
        s = beta ** m
        val, payload = phi(s)
        if np.isfinite(val) and val <= (1.0 - c * s) * phi0:
            return m, s, val, payload
    return None


class Problem:
    """A lattice, its material and its Dirichlet data, in global numbering."""

    def __init__(self, dim, ncell, nel, keep, mu, lam, fixed_bg, ubar_bg, fext_bg=None, rule=RULE_FULL):
        self.dim, self.nel, self.keep, self.rule = dim, nel, np.ascontiguousarray(keep, np.uint8), rule
        self.ncell = tuple(ncell)
        self.l2g, self.nact, self.g2bg = dofmap(dim, ncell, nel, self.keep)
        self.ng = self.g2bg.size
        Ns = self.keep.shape[0]
        self.mu = np.broadcast_to(np.asarray(mu, np.float64), (Ns,)).copy()
        self.lam = np.broadcast_to(np.asarray(lam, np.float64), (Ns,)).copy()
        self.fixed = np.asarray(fixed_bg)[self.g2bg].astype(bool)          # [n_global][d]
        self.ubar = np.asarray(ubar_bg, np.float64)[self.g2bg]
        self.fext = (np.zeros_like(self.ubar) if fext_bg is None
                     else np.asarray(fext_bg, np.float64)[self.g2bg])
        self.free = ~self.fixed.ravel()

    def evaluate(self, u, lf, want_T=True, want_energy=False):
        """(r masked [n_global][d], T [N_s][n_snap] or None, status, energy per cell or None).

        The residual and energy always use the full rule (the residual is not reduced, Sec. 4);
        the snapshots T use the problem's snapshot rule (full, one-point, the material tangent
        at the kept elements' centres, or the full tangent's entries at sampled nodes)."""
        ul = gather_local(u, self.l2g)
        full = self.rule in (RULE_FULL, RULE_SAMPLED)
        ev = cells_eval(self.dim, self.nel, self.keep, ul, self.mu, self.lam, rule=RULE_FULL, want_f=True,
                        want_energy=want_energy, want_T=want_T and full)
        T = ev["T"]
        if want_T and self.rule == RULE_SAMPLED:
            T = sampled_snapshots(self.dim, self.nel, T)
        elif want_T and self.rule == RULE_MATERIAL:
            T, _ = material_snapshots(self.dim, self.nel, self.keep, ul, self.mu, self.lam)
        elif want_T and not full:
            T = cells_eval(self.dim, self.nel, self.keep, ul, self.mu, self.lam, rule=self.rule, want_f=False,
                           want_energy=False, want_T=True)["T"]
        r = assemble(ev["f"], self.l2g, self.ng) - lf * self.fext
        r[self.fixed] = 0.0
        return r, T, ev["status"], ev["energy"]

    def principal_tangents(self, u, S, T):
        """Full-rule tangents K_k of the principal cells S (eq. reducedbasis); these are the
        snapshots themselves when the snapshots use the full rule."""
        if self.rule == RULE_FULL:
            return T[S]
        ul = gather_local(u, self.l2g)[S]
        return cells_eval(self.dim, self.nel, self.keep[S], ul, self.mu[S], self.lam[S], rule=RULE_FULL,
                          want_f=False, want_energy=False, want_T=True)["T"]

    def total_energy(self, u, lf):
        """Pi(u) = sum_s W_s(u^s) - lf f_ext . u (the potential whose gradient is r)."""
        _, _, st, en = self.evaluate(u, lf, want_T=False, want_energy=True)
        if st != OK:
            return np.inf
        return float(np.sum(en) - lf * np.sum(self.fext * u))

    def tangent_solve(self, u, T, rhs, rb_tol, cap):
        """Greedy on the snapshots T at u, then K~ du = rhs on the free components.
        Returns (du, greedy dict)."""
        g = greedy(T, rb_tol, cap, keep_Z=False)
        S = g["S"][:g["n_r"]]
        K = rom_matrix(self.dim, self.nel, self.principal_tangents(u, S, T), g["alpha"], self.l2g, self.ng)
        f = self.free
        du = np.zeros(self.ng * self.dim)
        if f.any():
            du[f] = spla.spsolve(K[f][:, f].tocsc(), rhs.ravel()[f])
        return du.reshape(self.ng, self.dim), g


def newton_solve(prob: Problem, n_inc=4, rb_tol=3e-4, cap=64, newton_tol=1e-6, max_newton=30, beta=0.5, c=1e-4,
                 max_bt=30, u0=None):
    """Load-stepped Newton-Raphson with Armijo backtracking (Sec. 2.2.5) on the ROM tangent.

    Returns dict(u, records, status); one record per Newton iteration with the increment, the
    iteration, n_r, the greedy's achieved tolerance, the Armijo exponent m and step beta^m, and
    the residual norms before/after and at the increment's start."""
    u = np.zeros((prob.ng, prob.dim)) if u0 is None else np.array(u0, np.float64, copy=True)
    recs = []
    status = OK
    for t in range(1, n_inc + 1):
        lf = t / n_inc
        u = u + prob.ubar / n_inc
        r, T, st, _ = prob.evaluate(u, lf)
        if st != OK:
            return {"u": u, "records": recs, "status": st}
        rn = float(np.linalg.norm(r))
        r0 = rn
        if r0 == 0.0:
            continue
        done = False
        for it in range(max_newton):
            du, g = prob.tangent_solve(u, T, -r, rb_tol, cap)

            def phi(s, u=u, du=du):
                rt, Tt, stt, _ = prob.evaluate(u + s * du, lf)
                if stt != OK:
                    return np.inf, None
                return float(np.linalg.norm(rt)), (rt, Tt)

            res = armijo(phi, rn, beta, c, max_bt)
            if res is None:
                return {"u": u, "records": recs, "status": NOCONV}
            m, s, val, (r, T) = res
            u = u + s * du
            recs.append({"increment": t, "iteration": it, "n_r": g["n_r"], "achieved": g["achieved"],
                         "greedy_status": g["status"], "backtracks": m, "step": s, "res_before": rn,
                         "res_after": val, "res0": r0})
            rn = val
            if rn <= newton_tol * r0:
                done = True
                break
        if not done:
            return {"u": u, "records": recs, "status": NOCONV}
    return {"u": u, "records": recs, "status": status}


# ----------------------------------------------------------------------------- coarse space (cell corners)
def coarse_prolongation(dim, ncell, nel, g2bg, fixed=None):
    """Prolongation P [n_global d][n_coarse d] from the cell-corner nodes: the Q1 (bi/trilinear)
    interpolation on the grid of cell corners, evaluated at every global fine node; rows of
    prescribed components are zero.  Coarse node C = cx + (C_x+1)(cy + (C_y+1) cz)."""
    ncell = list(ncell)
    gs = [c * nel + 1 for c in ncell]
    cs = [c + 1 for c in ncell]
    ng = g2bg.size
    gc = np.zeros((ng, dim), np.int64)
    r = g2bg.astype(np.int64).copy()
    for ax in range(dim):
        gc[:, ax] = r % gs[ax]
        r //= gs[ax]
    base = np.minimum(gc // nel, np.array(ncell[:dim]) - 1)          # enclosing coarse cell
    t = (gc - base * nel) / nel                                       # local coordinate in [0, 1]
    rows, cols, vals = [], [], []
    for corner in range(2 ** dim):
        bits = [(corner >> ax) & 1 for ax in range(dim)]
        w = np.ones(ng)
        C = np.zeros(ng, np.int64)
        stride = 1
        for ax in range(dim):
            w *= t[:, ax] if bits[ax] else 1.0 - t[:, ax]
            C += (base[:, ax] + bits[ax]) * stride
            stride *= cs[ax]
        for i in range(dim):
            rows.append(np.arange(ng) * dim + i)
            cols.append(C * dim + i)
            vals.append(w)
    nc = int(np.prod(cs[:dim]))
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ng * dim, nc * dim)).tocsr()
    P.eliminate_zeros()
    if fixed is not None:
        keep = sp.diags((~np.asarray(fixed, bool).ravel()).astype(np.float64))
        P = (keep @ P).tocsr()
    return P


def coarse_operator(K, P):
    """Galerkin coarse operator K_0 = P^T K P (dense); rows and columns of coarse components with
    no free fine support get a unit diagonal."""
    K0 = np.asarray((P.T @ (K @ P)).todense())
    empty = np.asarray(abs(P).sum(axis=0)).ravel() == 0.0
    K0[empty, empty] = 1.0
    return K0
