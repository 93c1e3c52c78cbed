"""ctypes binding of liblat.so (the C ABI declared in include/lat.h).

Argument marshalling only: torch supplies device memory and the current HIP stream, every
step of the computation runs in the library's kernels.  There is no fallback: if the
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LAT_LIBRARY may name another build of the same ABI (e.g. a tuning variant)
LIB_PATH = os.environ.get("LAT_LIBRARY") or os.path.join(_HERE, "liblat.so")

(LAT_OK, LAT_E_ARG, LAT_E_SHAPE, LAT_E_DEVICE, LAT_E_NOMEM, LAT_E_INVERTED, LAT_E_NONFINITE, LAT_W_CAP, LAT_E_NOCONV,
 LAT_E_SINGULAR) = range(10)
RULE_FULL, RULE_REDUCED, RULE_MATERIAL, RULE_SAMPLED = 0, 1, 2, 3
(CALL_RESIDUAL_TANGENT, CALL_PRINCIPAL_OPS, CALL_SELECT_PRINCIPAL, CALL_APPLY_COMBO, CALL_APPLY_COMBO_ADJOINT,
 CALL_ALPHA_ADJOINT, CALL_RESIDUAL_ADJOINT) = range(7)
N_CALLS = 7
# the binding gives a call its fast workspace when that stays within this many bytes, else the minimum
WORK_FAST_LIMIT = int(os.environ.get("LAT_WORK_FAST_LIMIT", str(24 << 30)))
SAMPLE_STRIDE = 2
F64, F32, BF16 = 0, 1, 2
INFO_KEYS = ["dim", "nel", "ncells", "nloc", "nelem", "E", "nsnap", "ld", "ngroups", "npacked", "nglobal", "cap"]


class NewtonOpts(ctypes.Structure):
    """lat_newton_opts"""
    _fields_ = [("n_inc", ctypes.c_int32), ("max_newton", ctypes.c_int32), ("max_backtrack", ctypes.c_int32),
                ("cap", ctypes.c_int32), ("cg_maxit", ctypes.c_int32), ("cg_check", ctypes.c_int32),
                ("snap_rule", ctypes.c_int32), ("verbose", ctypes.c_int32), ("matvec", ctypes.c_int32),
                ("tangent", ctypes.c_int32), ("precond", ctypes.c_int32), ("feti_n_delta", ctypes.c_int32),
                ("rb_tol", ctypes.c_double),
                ("newton_tol", ctypes.c_double), ("armijo_beta", ctypes.c_double), ("armijo_c", ctypes.c_double),
                ("cg_tol", ctypes.c_double)]


class NewtonRecord(ctypes.Structure):
    """lat_newton_record"""
    _fields_ = [("increment", ctypes.c_int32), ("iteration", ctypes.c_int32), ("n_r", ctypes.c_int32),
                ("backtracks", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("greedy_status", ctypes.c_int32),
                ("cg_status", ctypes.c_int32), ("coarse", ctypes.c_int32), ("step", ctypes.c_double),
                ("res_before", ctypes.c_double), ("res_after", ctypes.c_double), ("res0", ctypes.c_double),
                ("rb_achieved", ctypes.c_double), ("cg_relres", ctypes.c_double), ("t_init_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_eval_ms", ctypes.c_double), ("t_product_us", ctypes.c_double),
                ("solver", ctypes.c_int32), ("feti_iters", ctypes.c_int32), ("feti_enrich", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("feti_relres", ctypes.c_double), ("t_feti_setup_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FetiOpts(ctypes.Structure):
    """lat_feti_opts"""
    _fields_ = [("n_delta", ctypes.c_int32), ("enrich", ctypes.c_int32), ("max_enrich", ctypes.c_int32),
                ("inner_it", ctypes.c_int32), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("materialize", ctypes.c_int32), ("indefinite", ctypes.c_int32), ("coords", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("tol", ctypes.c_double), ("inner_tol", ctypes.c_double)]


class FetiInfo(ctypes.Structure):
    """lat_feti_info"""
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("enrich", ctypes.c_int32),
                ("n_delta", ctypes.c_int32), ("n_shift", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_primal", ctypes.c_int64), ("n_mult", ctypes.c_int64),
                ("n_rdofs", ctypes.c_int64), ("n_ddofs", ctypes.c_int64), ("relres", ctypes.c_double),
                ("max_shift", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LatError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = int(code)
        super().__init__(f"liblat {where}: {_lib().lat_status_string(int(code)).decode()} (status {int(code)})")


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              f"python -m paper_2603_10741_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        Z = ctypes.c_size_t
        sig = {
            "lat_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "lat_plan_create": (ctypes.c_int, [I32, P, I32, P, I32, P, P]),
            "lat_plan_destroy": (ctypes.c_int, [P]),
            "lat_plan_info": (ctypes.c_int, [P, P]),
            "lat_plan_query": (ctypes.c_int, [P, P, P]),
            "lat_status_reset": (ctypes.c_int, [P, P]),
            "lat_dofmap": (ctypes.c_int, [P, P, P, P, P, P]),
            "lat_residual_tangent": (ctypes.c_int, [P, P, P, P, ctypes.c_int, P, P, P, P, P, P, Z, P]),
            "lat_snapshot_rows": (I64, [P, ctypes.c_int]),
            "lat_principal_ops": (ctypes.c_int, [P, P, P, P, P, I32, P, P, P, P, P, Z, P]),
            "lat_select_principal": (ctypes.c_int, [P, P, F, I32, P, P, P, P, P, P, P, P, P, P, Z, P]),
            "lat_select_principal_rows": (ctypes.c_int, [P, P, I64, F, I32, P, P, P, P, P, P, P, P, P, P, Z, P]),
            "lat_apply_combo": (ctypes.c_int, [P, P, I32, P, P, P, I32, ctypes.c_int, F, I32, P, P, Z, P]),
            "lat_apply_combo_noalloc": (ctypes.c_int, [P, P, I32, P, P, P, I32, ctypes.c_int, F, I32, P, P]),
            "lat_basis_stack": (ctypes.c_int, [P, P, P, P, I32, P, P, P]),
            "lat_apply_plain": (ctypes.c_int, [P, P, P, P, I32, P]),
            "lat_apply_combo_adjoint": (ctypes.c_int, [P, P, P, P, P, I32, P, P, P, I32, P, P, P, P, ctypes.c_int, F, P,
                                                       P, Z, P]),
            "lat_alpha_adjoint": (ctypes.c_int, [P, P, P, P, P, P, I32, P, P, P, P, P, P, P, Z, P]),
            "lat_residual_adjoint": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, P, P, Z, P]),
            "lat_assemble": (ctypes.c_int, [P, P, I32, P, P]),
            "lat_gather": (ctypes.c_int, [P, P, I32, P, P]),
            "lat_pack": (ctypes.c_int, [P, P, P, I32, P]),
            "lat_unpack": (ctypes.c_int, [P, P, P, I32, P]),
            "lat_cil_to_canon": (ctypes.c_int, [P, P, I64, P, P]),
            "lat_canon_to_cil": (ctypes.c_int, [P, P, I64, P, P]),
            "lat_plain_ops_to_canon": (ctypes.c_int, [P, P, P, P]),
            "lat_rom_solve": (ctypes.c_int, [P, P, I32, P, P, P, P, F, I32, I32, I32, I32, P, P, P, P]),
            "lat_coarse_operator": (ctypes.c_int, [P, P, I32, P, P, I32, P, P]),
            "lat_newton_solve": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, I32, P, P]),
            "lat_feti_partition": (ctypes.c_int, [P, I32, P, P, P, P, P]),
            "lat_feti_solve": (ctypes.c_int, [P, P, I32, P, P, P, P, P, P, P, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def exported_symbols():
    """Names of the C entry points this binding uses (all declared in include/lat.h)."""
    return ["lat_status_string", "lat_plan_create", "lat_plan_destroy", "lat_plan_info", "lat_plan_query",
            "lat_status_reset",
            "lat_dofmap", "lat_residual_tangent", "lat_snapshot_rows", "lat_principal_ops", "lat_select_principal", "lat_select_principal_rows",
            "lat_apply_combo", "lat_apply_combo_noalloc", "lat_basis_stack",
            "lat_apply_plain", "lat_apply_combo_adjoint", "lat_alpha_adjoint", "lat_residual_adjoint",
            "lat_assemble", "lat_gather", "lat_pack", "lat_unpack", "lat_cil_to_canon", "lat_canon_to_cil",
            "lat_plain_ops_to_canon", "lat_rom_solve", "lat_coarse_operator", "lat_newton_solve",
            "lat_feti_partition", "lat_feti_solve"]


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return ctypes.c_void_p(t.data_ptr())


def _need(t, n, dtype, name):
    """Host-side check of a tensor handed to the library: the C ABI takes bare pointers, so a
    tensor smaller than the size the call will touch must be refused here."""
    if t is None:
        return
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.numel() < n:
        raise ValueError(f"{name}: {t.numel()} elements, the call needs {n}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ok(st, where):
    if st != LAT_OK:
        raise LatError(st, where)


class Plan:
    """A lattice plan: DOF maps, lane grouping, packed layouts and workspace on one GPU."""

    def __init__(self, dim, ncell, nel, keep, cap=64, device="cuda"):
        self.device = torch.device(device)
        self.ncell = tuple(int(c) for c in ncell)
        keep = np.ascontiguousarray(keep, dtype=np.uint8)
        nc = (ctypes.c_int32 * 3)(*(list(ncell) + [1] * (3 - len(ncell))))
        out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _ok(_lib().lat_plan_create(dim, nc, nel, keep.ctypes.data_as(ctypes.c_void_p), cap, _stream(),
                                       ctypes.byref(out)), "plan_create")
        self._p = out
        info = (ctypes.c_int64 * len(INFO_KEYS))()
        _ok(_lib().lat_plan_info(self._p, info), "plan_info")
        self.info = {k: int(info[i]) for i, k in enumerate(INFO_KEYS)}
        for k, v in self.info.items():
            setattr(self, k, v)
        mn = (ctypes.c_size_t * N_CALLS)()
        fs = (ctypes.c_size_t * N_CALLS)()
        _ok(_lib().lat_plan_query(self._p, mn, fs), "plan_query")
        self.work_min = [int(x) for x in mn]
        self.work_fast = [int(x) for x in fs]
        self._work = {}
        self.status_word = torch.zeros(2, dtype=torch.int32, device=self.device)
        self.reset_status()

    def __del__(self):
        try:
            if getattr(self, "_p", None):
                _lib().lat_plan_destroy(self._p)
                self._p = None
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def _f64(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def workspace(self, call, fast=None):
        """The cached device workspace of a call, a uint8 tensor: (pointer, bytes).  Default: the
        call's fast size when that is at most WORK_FAST_LIMIT bytes, else that limit (the ROM
        adjoint then takes its W in lane batches); fast=True the fast size, fast=False the minimum."""
        key = (call, fast)
        if key not in self._work:
            mn, fs = self.work_min[call], self.work_fast[call]
            if fast is None:
                n = fs if fs <= WORK_FAST_LIMIT else max(mn, WORK_FAST_LIMIT)
            else:
                n = fs if fast else mn
            self._work[key] = torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
        t = self._work[key]
        return _ptr(t), ctypes.c_size_t(t.numel())

    def _stack_elems(self):
        return self.nloc * self.E * self.cap

    def reset_status(self):
        _ok(_lib().lat_status_reset(_ptr(self.status_word), _stream()), "status_reset")

    def check_status(self, allow_cap=True):
        torch.cuda.current_stream().synchronize()
        code, cell = (int(x) for x in self.status_word.cpu())
        if code != LAT_OK and not (allow_cap and code == LAT_W_CAP):
            raise LatError(code, f"device status (first cell {cell})")
        return code, cell

    # ------------------------------------------------------------------ a1
    def dofmap(self):
        l2g = torch.empty(self.ncells, self.nloc, dtype=torch.int32, device=self.device)
        nact = torch.empty(self.ncells, dtype=torch.int32, device=self.device)
        g2bg = torch.empty(max(self.nglobal, 1), dtype=torch.int64, device=self.device)
        perm = torch.empty(self.ld, dtype=torch.int32, device=self.device)
        _ok(_lib().lat_dofmap(self._p, _ptr(l2g), _ptr(nact), _ptr(g2bg), _ptr(perm), _stream()), "dofmap")
        return l2g, nact, g2bg[:self.nglobal], perm

    # ------------------------------------------------------------------ a2-a4
    def residual_tangent(self, u_global, mu, lam, snap_rule=RULE_FULL, f=True, energy=True, snap=True,
                         plain=False, out=None):
        out = dict(out or {})
        if f and "f" not in out:
            out["f"] = self._f64(self.nloc * self.dim * self.ld)
        if energy and "energy" not in out:
            out["energy"] = self._f64(self.ncells)
        if snap and "snap" not in out:
            out["snap"] = self._f64(self.nsnap * self.ld)
        if plain and "plain" not in out:
            out["plain"] = self._f64(self.npacked * self.E * 64)
        f64 = torch.float64
        _need(u_global, self.nglobal * self.dim, f64, "u_global")
        _need(mu, self.ncells, f64, "mu")
        _need(lam, self.ncells, f64, "lam")
        _need(out.get("f"), self.nloc * self.dim * self.ld, f64, "f")
        _need(out.get("energy"), self.ncells, f64, "energy")
        _need(out.get("snap"), self.nsnap * self.ld, f64, "snap")
        _need(out.get("plain"), self.npacked * self.E * 64, f64, "plain")
        w, wb = self.workspace(CALL_RESIDUAL_TANGENT)
        _ok(_lib().lat_residual_tangent(self._p, _ptr(u_global), _ptr(mu), _ptr(lam), snap_rule, _ptr(out.get("f")),
                                        _ptr(out.get("energy")), _ptr(out.get("snap")), _ptr(out.get("plain")),
                                        _ptr(self.status_word), w, wb, _stream()), "residual_tangent")
        return out

    def snapshot_rows(self, rule):
        """Leading snapshot rows the rule can make nonzero (the rest are zero)."""
        n = int(_lib().lat_snapshot_rows(self._p, int(rule)))
        if n < 0:
            raise ValueError(f"unknown snapshot rule {rule}")
        return n

    def principal_ops(self, u_global, mu, lam, S, n_r, parts=False, out=None):
        out = dict(out or {})
        for key in (["K", "K_mu", "K_lam"] if parts else ["K"]):
            if key not in out:
                out[key] = self._f64(self.nloc * self.E * self.cap)
        for key in ("K", "K_mu", "K_lam"):
            _need(out.get(key), self._stack_elems(), torch.float64, key)
        _need(S, min(int(n_r), self.cap), torch.int32, "S")
        w, wb = self.workspace(CALL_PRINCIPAL_OPS)
        _ok(_lib().lat_principal_ops(self._p, _ptr(u_global), _ptr(mu), _ptr(lam), _ptr(S), int(n_r), _ptr(out["K"]),
                                     _ptr(out.get("K_mu")), _ptr(out.get("K_lam")), _ptr(self.status_word),
                                     w, wb, _stream()), "principal_ops")
        return out

    # ------------------------------------------------------------------ a5-a6
    def select_principal(self, snap, tol, cap=None, keep_Z=True, out=None, rows=None):
        cap = self.cap if cap is None else cap
        out = dict(out or {})
        dev = self.device
        if "S" not in out:
            out.update(S=torch.empty(self.cap, dtype=torch.int32, device=dev),
                       n_r=torch.empty(1, dtype=torch.int32, device=dev),
                       alpha=self._f64(self.ncells, self.cap), beta=self._f64(self.ncells, self.cap),
                       nu=self._f64(self.ncells), R=self._f64(self.cap, self.cap), achieved=self._f64(1))
            if keep_Z:
                out["Z"] = self._f64(self.cap, self.nsnap)
        f64, c = torch.float64, self.cap
        _need(snap, self.nsnap * self.ld, f64, "snap")
        _need(out["S"], c, torch.int32, "S")
        _need(out["alpha"], self.ncells * c, f64, "alpha")
        _need(out.get("beta"), self.ncells * c, f64, "beta")
        _need(out.get("nu"), self.ncells, f64, "nu")
        _need(out["R"], c * c, f64, "R")
        _need(out.get("Z"), c * self.nsnap, f64, "Z")
        w, wb = self.workspace(CALL_SELECT_PRINCIPAL)
        args = (_ptr(out["S"]), _ptr(out["n_r"]), _ptr(out["alpha"]), _ptr(out.get("beta")), _ptr(out.get("nu")),
                _ptr(out["R"]), _ptr(out.get("Z")), _ptr(out["achieved"]), _ptr(self.status_word), w, wb, _stream())
        if rows is None:
            _ok(_lib().lat_select_principal(self._p, _ptr(snap), float(tol), int(cap), *args), "select_principal")
        else:
            _ok(_lib().lat_select_principal_rows(self._p, _ptr(snap), int(rows), float(tol), int(cap), *args),
                "select_principal_rows")
        return out

    # ------------------------------------------------------------------ a7-a8
    def packed_size(self, m):
        return self.npacked * self.dim * m * 64

    def apply_combo(self, K, n_r, alpha, X, m, transpose=False, prec=F64, refine_tol=1e-6, out=None, err_est=None):
        """ROM apply (lat_apply_combo).  err_est: optional device float64 tensor of one element that
        receives the FP64-measured error estimate of a reduced-precision combination."""
        Y = self._f64(self.packed_size(m)) if out is None else out
        f64 = torch.float64
        _need(K, self._stack_elems(), f64, "K")
        _need(alpha, self.ncells * self.cap, f64, "alpha")
        _need(X, self.packed_size(m), f64, "X")
        _need(Y, self.packed_size(m), f64, "Y")
        _need(err_est, 1, f64, "err_est")
        w, wb = self.workspace(CALL_APPLY_COMBO)
        _ok(_lib().lat_apply_combo(self._p, _ptr(K), int(n_r), _ptr(alpha), _ptr(X), _ptr(Y), int(m), prec,
                                   float(refine_tol), int(bool(transpose)), _ptr(err_est), w, wb, _stream()),
            "apply_combo")
        return Y

    def basis_stack(self, Z, nu, beta, n_r, out=None):
        out = dict(out or {})
        if "stack" not in out:
            out["stack"] = self._f64(self.nloc * self.E * self.cap)
            out["coef"] = self._f64(self.ncells, self.cap)
        _ok(_lib().lat_basis_stack(self._p, _ptr(Z), _ptr(nu), _ptr(beta), int(n_r), _ptr(out["stack"]),
                                   _ptr(out["coef"]), _stream()), "basis_stack")
        return out

    def apply_plain(self, ops, X, m, out=None):
        Y = self._f64(self.packed_size(m)) if out is None else out
        _need(ops, self.npacked * self.E * 64, torch.float64, "ops")
        _need(X, self.packed_size(m), torch.float64, "X")
        _need(Y, self.packed_size(m), torch.float64, "Y")
        _ok(_lib().lat_apply_plain(self._p, _ptr(ops), _ptr(X), _ptr(Y), int(m), _stream()), "apply_plain")
        return Y

    # ------------------------------------------------------------------ a9
    def apply_combo_adjoint(self, K, n_r, alpha, X, Ybar, m, K_mu=None, K_lam=None, S=None, want_xbar=True,
                            want_alpha_bar=True, prec=F64, refine_tol=1e-6, err_est=None, fast=None):
        """Adjoint of the ROM apply (lat_apply_combo_adjoint).  fast: force (True) or refuse (False)
        the workspace of the fast size (default: as workspace() decides)."""
        Xbar = self._f64(self.packed_size(m)) if want_xbar else None
        abar = self._f64(self.ncells, self.cap) if want_alpha_bar else None
        mub = self._f64(self.ncells) if K_mu is not None else None
        lamb = self._f64(self.ncells) if K_lam is not None else None
        f64 = torch.float64
        for key, t in (("K", K), ("K_mu", K_mu), ("K_lam", K_lam)):
            _need(t, self._stack_elems(), f64, key)
        _need(alpha, self.ncells * self.cap, f64, "alpha")
        _need(X, self.packed_size(m), f64, "X")
        _need(Ybar, self.packed_size(m), f64, "Ybar")
        _need(S, min(int(n_r), self.cap), torch.int32, "S")
        _need(err_est, 1, f64, "err_est")
        w, wb = self.workspace(CALL_APPLY_COMBO_ADJOINT, fast=fast)
        _ok(_lib().lat_apply_combo_adjoint(self._p, _ptr(K), _ptr(K_mu), _ptr(K_lam), _ptr(S), int(n_r), _ptr(alpha),
                                           _ptr(X), _ptr(Ybar), int(m), _ptr(Xbar), _ptr(abar), _ptr(mub), _ptr(lamb),
                                           int(prec), float(refine_tol), _ptr(err_est), w, wb, _stream()),
            "apply_combo_adjoint")
        return {"Xbar": Xbar, "alpha_bar": abar, "mu_bar": mub, "lam_bar": lamb}

    def alpha_adjoint(self, delta, Z, R, nu, S, n_r, alpha, alpha_bar, snap_mu, snap_lam, mu_bar, lam_bar):
        f64, c = torch.float64, self.cap
        for key, t in (("delta", delta), ("snap_mu", snap_mu), ("snap_lam", snap_lam)):
            _need(t, self.nsnap * self.ld, f64, key)
        _need(Z, c * self.nsnap, f64, "Z")
        _need(R, c * c, f64, "R")
        _need(alpha, self.ncells * c, f64, "alpha")
        _need(alpha_bar, self.ncells * c, f64, "alpha_bar")
        w, wb = self.workspace(CALL_ALPHA_ADJOINT)
        _ok(_lib().lat_alpha_adjoint(self._p, _ptr(delta), _ptr(Z), _ptr(R), _ptr(nu), _ptr(S), int(n_r), _ptr(alpha),
                                     _ptr(alpha_bar), _ptr(snap_mu), _ptr(snap_lam), _ptr(mu_bar), _ptr(lam_bar),
                                     w, wb, _stream()), "alpha_adjoint")

    def residual_adjoint(self, u_global, mu, lam, w_cil, local=True, glob=True, lame=True):
        ub = self._f64(self.nloc * self.dim * self.ld) if (local or glob) else None
        ug = self._f64(max(self.nglobal, 1) * self.dim) if glob else None
        mub = self._f64(self.ncells) if lame else None
        lamb = self._f64(self.ncells) if lame else None
        _need(w_cil, self.nloc * self.dim * self.ld, torch.float64, "w")
        w, wb = self.workspace(CALL_RESIDUAL_ADJOINT)
        _ok(_lib().lat_residual_adjoint(self._p, _ptr(u_global), _ptr(mu), _ptr(lam), _ptr(w_cil), _ptr(ub), _ptr(ug),
                                        _ptr(mub), _ptr(lamb), _ptr(self.status_word), w, wb, _stream()),
            "residual_adjoint")
        return {"ubar_local": ub, "ubar_global": ug, "mu_bar": mub, "lam_bar": lamb}

    # ------------------------------------------------------------------ layouts
    def assemble(self, local_cil, k):
        out = self._f64(max(self.nglobal, 1) * k)
        _ok(_lib().lat_assemble(self._p, _ptr(local_cil), int(k), _ptr(out), _stream()), "assemble")
        return out

    def gather(self, glob, k):
        out = self._f64(self.nloc * k * self.ld)
        _ok(_lib().lat_gather(self._p, _ptr(glob), int(k), _ptr(out), _stream()), "gather")
        return out

    def pack(self, canon, m):
        out = self._f64(self.packed_size(m))
        _ok(_lib().lat_pack(self._p, _ptr(canon), _ptr(out), int(m), _stream()), "pack")
        return out

    def unpack(self, packed, m):
        out = self._f64(self.ncells, self.nloc, self.dim, m)
        _ok(_lib().lat_unpack(self._p, _ptr(packed), _ptr(out), int(m), _stream()), "unpack")
        return out

    def cil_to_canon(self, cil, k):
        out = torch.zeros(self.ncells, self.nloc, k, dtype=torch.float64, device=self.device)
        _ok(_lib().lat_cil_to_canon(self._p, _ptr(cil), int(k), _ptr(out), _stream()), "cil_to_canon")
        return out

    def canon_to_cil(self, canon, k):
        out = self._f64(self.nloc * k * self.ld)
        _ok(_lib().lat_canon_to_cil(self._p, _ptr(canon), int(k), _ptr(out), _stream()), "canon_to_cil")
        return out

    def plain_ops_to_canon(self, ops):
        out = self._f64(self.ncells, self.nsnap)
        _ok(_lib().lat_plain_ops_to_canon(self._p, _ptr(ops), _ptr(out), _stream()), "plain_ops_to_canon")
        return out

    # ------------------------------------------------------------------ nonlinear solve
    def rom_solve(self, K, n_r, alpha, fixed, b, tol=1e-10, maxit=20000, check=32, materialize=True, precond=1,
                  x=None, info=None):
        """K~ x = b on the free components (lat_rom_solve).  Returns (x, status, iters, relres);
        status is LAT_OK, LAT_E_NOCONV or LAT_E_SINGULAR, other codes raise.  `info` (a dict)
        receives whether the coarse correction ran."""
        x = self._f64(max(self.nglobal, 1) * self.dim) if x is None else x
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        cu = ctypes.c_int32(0)
        st = _lib().lat_rom_solve(self._p, _ptr(K), int(n_r), _ptr(alpha), _ptr(fixed), _ptr(b), _ptr(x), float(tol),
                                  int(maxit), int(check), int(bool(materialize)), int(precond), ctypes.byref(it),
                                  ctypes.byref(rel), ctypes.byref(cu), _stream())
        if st not in (LAT_OK, LAT_E_NOCONV, LAT_E_SINGULAR):
            raise LatError(st, "rom_solve")
        if info is not None:
            info["coarse_used"] = bool(cu.value)
        return x, st, it.value, rel.value

    def feti_partition(self, level=0):
        """FETI-DP partition tables at an enrichment level (lat_feti_partition): dict(cls [nloc],
        primal [n_p] global node ids, mult [n_mult][4] (cell_1, node_1, cell_2, node_2))."""
        import numpy as np
        counts = (ctypes.c_int64 * 4)()
        _ok(_lib().lat_feti_partition(self._p, int(level), None, counts, None, None, _stream()), "feti_partition")
        cls = np.zeros(self.nloc, np.int32)
        prim = np.zeros(max(counts[0], 1), np.int64)
        mult = np.zeros((max(counts[1], 1), 4), np.int32)
        _ok(_lib().lat_feti_partition(self._p, int(level), cls.ctypes.data_as(ctypes.c_void_p), counts,
                                      prim.ctypes.data_as(ctypes.c_void_p), mult.ctypes.data_as(ctypes.c_void_p),
                                      _stream()), "feti_partition")
        return {"cls": cls, "primal": prim[:counts[0]], "mult": mult[:counts[1]], "n_remaining": int(counts[2]),
                "n_dual": int(counts[3])}

    def feti_solve(self, K, n_r, alpha, S, fixed, b, R=None, nu=None, beta=None, n_delta=0, enrich=0, max_enrich=3,
                   inner_it=8, restart=60, maxit=600, tol=1e-8, materialize=True, indefinite=0, coords=None,
                   prec=F64, x=None, inner_tol=0.0):
        """K~ x = b on the free components by the inexact FETI-DP iteration (lat_feti_solve).
        coords: 1 = nearest principal cell (the default when R, nu, beta are given), 0 = least squares.
        Returns (x, status, info dict); status is LAT_OK, LAT_E_NOCONV or LAT_E_SINGULAR, other
        codes raise."""
        if coords is None:
            coords = 1 if R is not None else 0
        n = max(self.nglobal, 1) * self.dim
        _need(b, n, torch.float64, "b")
        _need(fixed, n, torch.uint8, "fixed")
        _need(alpha, self.ncells * self.cap, torch.float64, "alpha")
        _need(S, self.cap, torch.int32, "S")
        _need(K, self.nloc * self.E * self.cap, torch.float64, "K")
        for t, sz, nm in ((R, self.cap * self.cap, "R"), (nu, self.ncells, "nu"), (beta, self.ncells * self.cap, "beta")):
            _need(t, sz, torch.float64, nm)
        x = self._f64(n) if x is None else x
        o = FetiOpts(int(n_delta), int(enrich), int(max_enrich), int(inner_it), int(restart), int(maxit),
                     int(bool(materialize)), int(indefinite), int(coords), int(prec), float(tol), float(inner_tol))
        inf = FetiInfo()
        st = _lib().lat_feti_solve(self._p, _ptr(K), int(n_r), _ptr(alpha), _ptr(S), _ptr(R), _ptr(nu), _ptr(beta),
                                   _ptr(fixed), _ptr(b), _ptr(x), ctypes.byref(o), ctypes.byref(inf), _stream())
        if st not in (LAT_OK, LAT_E_NOCONV, LAT_E_SINGULAR):
            raise LatError(st, "feti_solve")
        return x, st, inf.as_dict()

    def coarse_operator(self, K, n_r, alpha, fixed, materialize=True):
        """Dense K0 = P^T K~ P over the cell-corner nodes (lat_coarse_operator)."""
        nc = 1
        for c in self.ncell[:self.dim]:
            nc *= c + 1
        K0 = self._f64(nc * self.dim, nc * self.dim)
        _ok(_lib().lat_coarse_operator(self._p, _ptr(K), int(n_r), _ptr(alpha), _ptr(fixed), int(bool(materialize)),
                                       _ptr(K0), _stream()), "coarse_operator")
        return K0

    def newton_solve(self, mu, lam, fixed, ubar, u, f_ext=None, n_inc=4, max_newton=30, max_backtrack=30, cap=None,
                     rb_tol=3e-4, newton_tol=1e-6, armijo_beta=0.5, armijo_c=1e-4, cg_tol=1e-10, cg_maxit=20000,
                     cg_check=32, snap_rule=RULE_FULL, max_records=1024, verbose=False, matvec=0,
                     tangent=0, precond=1, feti_n_delta=0):
        """Load-stepped Newton-Raphson with Armijo backtracking (lat_newton_solve); u is updated in
        place.  Returns (status, records); status is LAT_OK, LAT_E_NOCONV, LAT_E_INVERTED or
        LAT_E_NONFINITE, other codes raise."""
        o = NewtonOpts(int(n_inc), int(max_newton), int(max_backtrack), int(cap if cap is not None else self.cap),
                       int(cg_maxit), int(cg_check), int(snap_rule), int(bool(verbose)), int(matvec), int(tangent),
                       int(precond), int(feti_n_delta), float(rb_tol), float(newton_tol), float(armijo_beta),
                       float(armijo_c),
                       float(cg_tol))
        recs = (NewtonRecord * max(int(max_records), 1))()
        nrec = ctypes.c_int32(0)
        st = _lib().lat_newton_solve(self._p, _ptr(mu), _ptr(lam), _ptr(fixed), _ptr(ubar), _ptr(f_ext), ctypes.byref(o),
                                     _ptr(u), recs, int(max_records), ctypes.byref(nrec), _stream())
        if st not in (LAT_OK, LAT_E_NOCONV, LAT_E_INVERTED, LAT_E_NONFINITE):
            raise LatError(st, "newton_solve")
        return st, [recs[i].as_dict() for i in range(min(nrec.value, int(max_records)))]
