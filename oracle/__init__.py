"""FP64 CPU oracle for the principal-cell lattice operators.

TEST INFRASTRUCTURE ONLY: imported by `tests/`, by the smoke check and by the CPU-baseline
leg of the benchmark, never by the product library.  It shares no code with the GPU path.

The heavy loops live in `lat_oracle.c` (plain C, FP64, explicit fma only); this module
builds and loads it with gcc/ctypes and adds the few steps that are most plainly written
with numpy linear algebra (the adjoint of the least-squares coefficients).

Layouts are cell-major ("canonical"):
  local fields  [N_s][(n+1)^d][d]        right-hand sides [N_s][(n+1)^d][d][m]
  stencil / snapshot of a cell  [(n+1)^d][3^d][d][d], entry (a,o,i,j) = K[(a,i),(a+o,j)]
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lat_oracle.c")
_LIB = os.path.join(_HERE, "liblat_oracle.so")
_lib = None

OK, E_INVERTED, E_NONFINITE, W_CAP = 0, 5, 6, 7
RULE_FULL, RULE_REDUCED, RULE_MATERIAL, RULE_SAMPLED = 0, 1, 2, 3
SAMPLE_STRIDE = 2          # node stride of the sampled-entry snapshots (every element has one corner there)


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, FP64, no implicit contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.orc_dofmap.restype = i64
        L.orc_dofmap.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P, P]
        L.orc_neo_hooke.restype = ctypes.c_int
        L.orc_neo_hooke.argtypes = [P, f64, f64, P, P, P]
        L.orc_cell_eval.restype = ctypes.c_int
        L.orc_cell_eval.argtypes = [ctypes.c_int, ctypes.c_int, P, P, f64, f64, ctypes.c_int, P, P, P, P]
        L.orc_cells_eval.restype = ctypes.c_int
        L.orc_cells_eval.argtypes = [ctypes.c_int, ctypes.c_int, i64, P, P, P, P, ctypes.c_int, P, P, P, P]
        L.orc_dot.restype = f64
        L.orc_dot.argtypes = [P, P, i64]
        L.orc_greedy.restype = ctypes.c_int
        L.orc_greedy.argtypes = [i64, i64, P, f64, ctypes.c_int, P, P, P, P, P, P, P]
        L.orc_alpha.restype = None
        L.orc_alpha.argtypes = [i64, ctypes.c_int, ctypes.c_int, P, P, P, P]
        L.orc_stencil_apply.restype = None
        L.orc_stencil_apply.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int, P]
        L.orc_plain_apply.restype = None
        L.orc_plain_apply.argtypes = [ctypes.c_int, ctypes.c_int, i64, P, P, P, ctypes.c_int, ctypes.c_int, P]
        L.orc_combo_apply.restype = None
        L.orc_combo_apply.argtypes = [ctypes.c_int, ctypes.c_int, i64, ctypes.c_int, P, P, ctypes.c_int, P, P,
                                      ctypes.c_int, ctypes.c_int, P]
        L.orc_combo_forms.restype = None
        L.orc_combo_forms.argtypes = [ctypes.c_int, ctypes.c_int, i64, ctypes.c_int, P, ctypes.c_int, P, P, P,
                                      ctypes.c_int, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def n_snap(dim: int, nel: int) -> int:
    return (nel + 1) ** dim * 3 ** dim * dim * dim


# ----------------------------------------------------------------------------- a1: DOF maps
def dofmap(dim, ncell, nel, keep):
    """Local-to-global map (eq. residualvector's Boolean A^s as an index map).

    Returns l2g int32 [N_s][(n+1)^d] (-1 = node not active in the cell), n_active int32 [N_s],
    g2bg int64 [n_global] (background-grid id of each global active node)."""
    keep = _c(keep, np.uint8)
    ncell = _c(list(ncell) + [1] * (3 - len(ncell)), np.int32)
    Ns = int(np.prod(ncell[:dim]))
    nloc = (nel + 1) ** dim
    l2g = np.empty((Ns, nloc), np.int32)
    nact = np.empty(Ns, np.int32)
    G = int(np.prod([c * nel + 1 for c in ncell[:dim]]))
    g2bg = np.empty(G, np.int64)
    ng = lib().orc_dofmap(dim, _p(ncell), nel, _p(keep), _p(l2g), _p(nact), _p(g2bg))
    return l2g, nact, g2bg[:ng].copy()


def gather_local(u_global, l2g):
    """u^s = A^{sT} u: per-cell local displacements, zero at nodes the cell does not own."""
    u_global = np.asarray(u_global)
    out = np.zeros(l2g.shape + (u_global.shape[1],))
    m = l2g >= 0
    out[m] = u_global[l2g[m]]
    return out


def assemble(local, l2g, n_global):
    """r = sum_s A^s f^s (eq. residualvector): scatter-add cell-local vectors to global nodes."""
    d = local.shape[-1]
    out = np.zeros((n_global, d))
    m = l2g >= 0
    np.add.at(out, l2g[m], local[m])
    return out


# ----------------------------------------------------------------------------- a2/a3: cell operators
def neo_hooke(F, mu, lam):
    """(W, P, A) at one 3x3 deformation gradient (material form)."""
    F = _c(F, np.float64).reshape(9)
    W = np.zeros(1); P = np.zeros(9); A = np.zeros(81)
    ok = lib().orc_neo_hooke(_p(F), float(mu), float(lam), _p(W), _p(P), _p(A))
    if not ok:
        raise ValueError("J <= 0")
    return W[0], P.reshape(3, 3), A.reshape(3, 3, 3, 3)


def cell_eval(dim, nel, keep_c, u_c, mu, lam, rule=RULE_FULL, dense=False):
    """One cell: dict(f, energy, stencil, [K dense], status)."""
    nloc = (nel + 1) ** dim
    keep_c = _c(keep_c, np.uint8); u_c = _c(u_c, np.float64).reshape(nloc, dim)
    f = np.zeros((nloc, dim)); en = np.zeros(1)
    st = np.zeros(n_snap(dim, nel))
    Kd = np.zeros((nloc * dim, nloc * dim)) if dense else None
    s = lib().orc_cell_eval(dim, nel, _p(keep_c), _p(u_c), float(mu), float(lam), int(rule), _p(f), _p(en),
                            _p(st), _p(Kd))
    out = {"f": f, "energy": en[0], "stencil": st, "status": s}
    if dense:
        out["K"] = Kd
    return out


def cells_eval(dim, nel, keep, u_loc, mu, lam, rule=RULE_FULL, want_f=True, want_energy=True, want_T=True):
    """All cells: f [N_s][(n+1)^d][d], energy [N_s], T [N_s][n_snap] (stencil snapshots)."""
    keep = _c(keep, np.uint8)
    Ns = keep.shape[0]
    nloc = (nel + 1) ** dim
    u_loc = _c(u_loc, np.float64)
    mu = _c(np.broadcast_to(mu, (Ns,)), np.float64)
    lam = _c(np.broadcast_to(lam, (Ns,)), np.float64)
    f = np.zeros((Ns, nloc, dim)) if want_f else None
    en = np.zeros(Ns) if want_energy else None
    T = np.zeros((Ns, n_snap(dim, nel))) if want_T else None
    st = np.zeros(Ns, np.int32)
    worst = lib().orc_cells_eval(dim, nel, Ns, _p(keep), _p(u_loc), _p(mu), _p(lam), int(rule), _p(f), _p(en),
                                 _p(T), _p(st))
    return {"f": f, "energy": en, "T": T, "status": worst, "status_cell": st}


# ----------------------------------------------------------------------------- a5/a6: greedy and alpha
def dot(x, y):
    x = _c(x, np.float64); y = _c(y, np.float64)
    return lib().orc_dot(_p(x), _p(y), x.size)


def greedy(T, tol, cap, keep_Z=True):
    """Algorithm 1 on snapshots T [N_s][n_snap] (copied). Returns a dict with S, n_r, beta, nu, R,
    Z, Delta, achieved, status, alpha."""
    D = np.array(T, dtype=np.float64, order="C", copy=True)
    Ns, ns = D.shape
    S = np.empty(cap, np.int32); nr = np.zeros(1, np.int32)
    beta = np.zeros((Ns, cap)); nu = np.zeros(Ns); R = np.zeros((cap, cap)); ach = np.zeros(1)
    Z = np.zeros((cap, ns)) if keep_Z else None
    st = lib().orc_greedy(ns, Ns, _p(D), float(tol), int(cap), _p(S), _p(nr), _p(beta), _p(nu), _p(R), _p(Z),
                          _p(ach))
    n_r = int(nr[0])
    alpha = np.zeros((Ns, cap))
    lib().orc_alpha(Ns, cap, n_r, _p(R), _p(nu), _p(beta), _p(alpha))
    return {"S": S, "n_r": n_r, "beta": beta, "nu": nu, "R": R, "Z": Z, "Delta": D, "achieved": ach[0],
            "status": st, "alpha": alpha}


# ----------------------------------------------------------------------------- a7/a8: applies
def stencil_apply(dim, nel, st, l2g_c, x, transpose=False):
    st = _c(st, np.float64); l2g_c = _c(l2g_c, np.int32); x = _c(x, np.float64)
    m = x.shape[-1]
    y = np.zeros_like(x)
    lib().orc_stencil_apply(dim, nel, _p(st), _p(l2g_c), _p(x), m, int(bool(transpose)), _p(y))
    return y


def plain_apply(dim, nel, Kst, l2g, X, transpose=False):
    Kst = _c(Kst, np.float64); l2g = _c(l2g, np.int32); X = _c(X, np.float64)
    Y = np.zeros_like(X)
    lib().orc_plain_apply(dim, nel, X.shape[0], _p(Kst), _p(l2g), _p(X), X.shape[-1], int(bool(transpose)), _p(Y))
    return Y


def combo_apply(dim, nel, Kp, alpha, l2g, X, transpose=False):
    """Y_i = M_i (sum_k alpha_ik K_k) M_i X_i; Kp [n_r][n_snap], alpha [N_s][cap]."""
    Kp = _c(Kp, np.float64); alpha = _c(alpha, np.float64); l2g = _c(l2g, np.int32); X = _c(X, np.float64)
    Y = np.zeros_like(X)
    lib().orc_combo_apply(dim, nel, X.shape[0], Kp.shape[0], _p(Kp), _p(alpha), alpha.shape[1], _p(l2g), _p(X),
                          X.shape[-1], int(bool(transpose)), _p(Y))
    return Y


def combo_forms(dim, nel, Kp, cap, l2g, X, Ybar):
    """G[i,k] = <M Ybar_i, K_k M X_i> for every cell i and principal operator k; G [N_s][cap]."""
    Kp = _c(Kp, np.float64); l2g = _c(l2g, np.int32); X = _c(X, np.float64); Ybar = _c(Ybar, np.float64)
    G = np.zeros((X.shape[0], cap))
    lib().orc_combo_forms(dim, nel, X.shape[0], Kp.shape[0], _p(Kp), cap, _p(l2g), _p(X), _p(Ybar), X.shape[-1],
                          _p(G))
    return G


# ----------------------------------------------------------------------------- a9: adjoints
def alpha_ls_adjoint(T_S, T_all, alpha, alpha_bar):
    """Reverse mode of alpha_i = (T_S^T T_S)^{-1} T_S^T t_i with the principal set frozen.

    T_S [n_snap][n_r] principal snapshots, T_all [N_s][n_snap], alpha / alpha_bar [N_s][n_r].
    Returns (tbar_all [N_s][n_snap], TbarS [n_snap][n_r]): the cotangents of every snapshot
    through its own coefficients, and of the principal snapshots as basis columns.
      v_i = G^{-1} abar_i, tbar_i = T_S v_i, TbarS = sum_i (rho_i v_i^T - T_S v_i alpha_i^T),
      rho_i = t_i - T_S alpha_i."""
    G = T_S.T @ T_S
    V = np.linalg.solve(G, alpha_bar.T).T               # [N_s][n_r]
    tbar = V @ T_S.T                                     # [N_s][n_snap]
    rho = T_all - alpha @ T_S.T                          # [N_s][n_snap]
    TbarS = rho.T @ V - (T_S @ V.T) @ alpha              # [n_snap][n_r]
    return tbar, TbarS


# ----------------------------------------------------------------------------- f3: material snapshots
def material_snapshots(dim, nel, keep, u_loc, mu, lam):
    """Snapshots made of the material tangent A = dP/dF (the pulled-back fourth-order tensor of the
    Remark on snapshots in Sec. 3.2.2) at the centre of every kept element, [N_s][n_snap]:
    row (e d^2 + i d + J) d^2 + k d + L holds A_iJkL of element e; rows of elements that are not
    kept, and rows past n^d d^4, are zero.  2D is plane strain (F_33 = 1).
    Returns (T, status) with status E_INVERTED when J <= 0 at some kept centre."""
    keep = np.asarray(keep, np.uint8)
    Ns = keep.shape[0]
    nn = nel + 1
    h = 1.0 / nel
    d4 = dim ** 4
    T = np.zeros((Ns, n_snap(dim, nel)))
    status = OK
    corners = [[(c >> ax) & 1 for ax in range(dim)] for c in range(2 ** dim)]
    for s in range(Ns):
        mu_s = float(np.broadcast_to(mu, (Ns,))[s]); lam_s = float(np.broadcast_to(lam, (Ns,))[s])
        for e in range(nel ** dim):
            if not keep[s, e]:
                continue
            ec = [(e // nel ** ax) % nel for ax in range(dim)]
            F = np.eye(3)
            for cb in corners:
                a = sum((ec[ax] + cb[ax]) * nn ** ax for ax in range(dim))
                # gradient of the Q1 shape function of corner cb at the element centre
                g = np.array([(1.0 if cb[ax] else -1.0) / h * 0.5 ** (dim - 1) for ax in range(dim)])
                F[:dim, :dim] += np.outer(u_loc[s, a, :dim], g)
            try:
                _, _, A = neo_hooke(F, mu_s, lam_s)
            except ValueError:
                status = E_INVERTED
                continue
            T[s, e * d4:(e + 1) * d4] = A[:dim, :dim, :dim, :dim].reshape(-1)
    return T, status


# ----------------------------------------------------------------------------- f3: sampled entries
def sampled_nodes(dim, nel, stride=SAMPLE_STRIDE):
    """Local nodes whose every coordinate is a multiple of `stride`, lexicographic (x fastest)."""
    nn = nel + 1
    axis = list(range(0, nn, stride))
    return [sum(c[ax] * nn ** ax for ax in range(dim)) for c in _lex(axis, dim)]


def _lex(axis, dim):
    if dim == 0:
        yield []
        return
    for hi in axis:                                   # slowest axis outermost
        for lo in _lex(axis, dim - 1):
            yield lo + [hi]


def sampled_snapshots(dim, nel, T_full, stride=SAMPLE_STRIDE):
    """Snapshots made of a limited number of entries of the true tangent (the some_data(K) choice of
    the Remark on snapshots in Sec. 3.2.2): the full-rule stencil rows (every 3^d d^2 entry) of the
    local nodes on the sub-grid of node stride `stride`, node j of `sampled_nodes` in rows
    j 3^d d^2 ... (j+1) 3^d d^2 - 1; rows past them are zero.  T_full [N_s][n_snap] is the cells'
    full-rule snapshot matrix."""
    E = 3 ** dim * dim * dim
    T_full = np.asarray(T_full, np.float64)
    T = np.zeros_like(T_full)
    for j, a in enumerate(sampled_nodes(dim, nel, stride)):
        T[:, j * E:(j + 1) * E] = T_full[:, a * E:(a + 1) * E]
    return T
