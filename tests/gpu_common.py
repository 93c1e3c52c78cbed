"""Shared helpers of the GPU parity tests: run the HIP path and the FP64 oracle on the same
seeded inputs and bring both to canonical (cell-major) layouts."""
from __future__ import annotations

import numpy as np
import torch

import lattice as L
import oracle as O


def rel(a, b):
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


class Case:
    """One workload on both sides."""

    def __init__(self, cfg, m=None, keep=None, mu=None, lam=None, u_bg=None):
        from paper_2603_10741_amd import binding as B
        self.B = B
        self.cfg = cfg
        self.dim, self.nel = cfg.dim, cfg.nel
        self.m = cfg.m if m is None else m
        self.keep = L.make_keep(cfg) if keep is None else keep
        mu0, lam0 = L.make_material(cfg)
        self.mu = mu0 if mu is None else mu
        self.lam = lam0 if lam is None else lam
        self.u_bg = L.make_displacement(cfg) if u_bg is None else u_bg
        self.dev = torch.device("cuda:0")
        print(f"[case] {cfg.name} sub={cfg.sub} cells={cfg.n_cells} m={self.m}", flush=True)
        self.P = B.Plan(self.dim, cfg.ncell_eff, self.nel, self.keep, cap=cfg.cap)
        l2g, nact, g2bg, perm = self.P.dofmap()
        self.l2g_gpu, self.nact_gpu, self.g2bg_gpu, self.perm = l2g, nact, g2bg, perm
        self.l2g, self.nact, self.g2bg = O.dofmap(self.dim, cfg.ncell_eff, self.nel, self.keep)
        self.ug = torch.from_numpy(self.u_bg).to(self.dev)[g2bg].contiguous()
        self.mu_t = torch.from_numpy(np.ascontiguousarray(self.mu)).to(self.dev)
        self.lam_t = torch.from_numpy(np.ascontiguousarray(self.lam)).to(self.dev)
        self.uloc = O.gather_local(self.u_bg[self.g2bg], self.l2g)
        self._oracle = None

    # ---------------------------------------------------------------- oracle side
    @property
    def orc(self):
        if self._oracle is None:
            self._oracle = O.cells_eval(self.dim, self.nel, self.keep, self.uloc, self.mu, self.lam)
        return self._oracle

    # ---------------------------------------------------------------- conversions
    def canon_T(self, snap_cil):
        P = self.P
        return P.cil_to_canon(snap_cil, P.E).reshape(P.ncells, -1).cpu().numpy()

    def to_cil_T(self, T):
        P = self.P
        return P.canon_to_cil(torch.from_numpy(np.ascontiguousarray(T)).to(self.dev).reshape(P.ncells, P.nloc, P.E)
                              .contiguous(), P.E)

    def canon_field(self, cil, k):
        return self.P.cil_to_canon(cil, k).cpu().numpy()

    def rhs(self, stream=0, m=None):
        m = self.m if m is None else m
        X = L.make_rhs(self.cfg, m=m, stream=stream)
        return X, self.P.pack(torch.from_numpy(X).to(self.dev), m)

    def unpack(self, packed, m=None):
        return self.P.unpack(packed, self.m if m is None else m).cpu().numpy()

    def masked(self, X):
        return X * (self.l2g >= 0)[:, :, None, None]
