"""Seeded synthetic lattice inputs shared by the oracle and the HIP path.

This module draws the inputs of the workloads only: element keep-masks of
voxelised unit cells, per-cell Lame parameters, a displacement field sampled
on the background node grid of the whole lattice, and random right-hand sides
for operator applies.  It contains none of the method's arithmetic (no DOF
numbering, no kinematics, no quadrature, no greedy).

Geometry and numbering conventions (the same on both sides of every test):

* a unit cell is the square/cube [0,1]^d (cell edge 1), meshed by n^d Q1
  elements of size h = 1/n; cells are congruent translates of each other;
* element e = ex + n*(ey + n*ez), node a = ix + (n+1)*(iy + (n+1)*iz);
* cells are numbered lexicographically over the lattice, x fastest;
* the background node grid of the lattice has (C_x n + 1) x (C_y n + 1)
  [x (C_z n + 1)] nodes numbered x fastest; global coordinates are in cell
  edges.

The workloads stand in for the paper's spline lattices (hole cells under
compression, body-centred-cubic strut cells under compression; the unit-cell
library of the numerical-results section), which are not available.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

BASE_SEED = 260310741


@dataclasses.dataclass(frozen=True)
class LatticeConfig:
    """One synthetic workload."""
    index: int
    name: str
    dim: int
    ncell: tuple            # cells per axis (length dim)
    nel: int                # Q1 elements per cell axis
    topology: str           # "hole", "bcc", "bcc_octet"
    radius: tuple           # hole: (r_left, r_right) graded along x; struts: (r_lo, r_hi) uniform
    mu_law: str             # "const" or "logu"
    mu: tuple               # const: (mu,); logu: (lo, hi)
    lam_over_mu: Optional[float]   # lam = lam_over_mu * mu when set
    lam: float              # used when lam_over_mu is None
    strain: float           # uniaxial compressive strain along the last axis
    pert_amp: float         # amplitude of the smooth perturbation (cell edges)
    m: int                  # right-hand sides per cell for operator applies
    tol: float              # greedy tolerance
    cap: int                # cap on the number of principal cells
    sub: Optional[tuple] = None    # optional sub-lattice (cells per axis) cut from the low corner

    @property
    def ncell_eff(self) -> tuple:
        return tuple(self.sub) if self.sub is not None else tuple(self.ncell)

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.ncell_eff))

    @property
    def n_local_nodes(self) -> int:
        return (self.nel + 1) ** self.dim

    @property
    def n_elems(self) -> int:
        return self.nel ** self.dim

    def with_sub(self, sub: Sequence[int]) -> "LatticeConfig":
        sub = tuple(int(s) for s in sub)
        assert len(sub) == self.dim and all(1 <= s <= c for s, c in zip(sub, self.ncell))
        return dataclasses.replace(self, sub=sub)

    def with_(self, **kw) -> "LatticeConfig":
        return dataclasses.replace(self, **kw)


CONFIGS = [
    LatticeConfig(0, "hole2d_4x4_n16", 2, (4, 4), 16, "hole", (0.30, 0.30), "const", (1.0,), None, 10.0,
                  0.05, 1e-3, 8, 1e-8, 16),
    LatticeConfig(1, "hole2d_32x32_n32_graded", 2, (32, 32), 32, "hole", (0.20, 0.35), "const", (1.0,), None, 10.0,
                  0.10, 1e-3, 16, 1e-8, 32),
    LatticeConfig(2, "bcc3d_10x10x10_n12", 3, (10, 10, 10), 12, "bcc", (0.10, 0.15), "const", (1.0,), None, 5.0,
                  0.08, 1e-3, 16, 1e-8, 64),
    LatticeConfig(3, "bcc3d_8x8x8_n12_logmu", 3, (8, 8, 8), 12, "bcc", (0.10, 0.15), "logu", (0.5, 2.0), 5.0, 5.0,
                  0.08, 1e-3, 1, 1e-8, 64),
    LatticeConfig(4, "bcc_octet3d_20x20x20_n16", 3, (20, 20, 20), 16, "bcc_octet", (0.08, 0.14), "const", (1.0,),
                  None, 5.0, 0.12, 1e-3, 16, 1e-8, 64),
]


def config(i: int) -> LatticeConfig:
    return CONFIGS[i]


def _streams(cfg: LatticeConfig):
    ss = np.random.SeedSequence(BASE_SEED + cfg.index)
    kids = ss.spawn(5)
    return {k: kids[i] for i, k in enumerate(["radius", "topology", "mu", "pert", "rhs"])}


def _sub_cell_ids(cfg: LatticeConfig) -> np.ndarray:
    """Full-lattice ids of the cells of the (sub-)lattice, in sub-lattice order."""
    full = cfg.ncell
    sub = cfg.ncell_eff
    axes = [np.arange(s) for s in sub]
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]   # x fastest
    ids = np.zeros(grids[0].shape, dtype=np.int64)
    stride = 1
    for ax in range(cfg.dim):
        ids += grids[ax] * stride
        stride *= full[ax]
    return ids.reshape(-1)


def _cell_coords_full(cfg: LatticeConfig) -> np.ndarray:
    full = cfg.ncell
    n = int(np.prod(full))
    c = np.arange(n)
    out = np.zeros((n, cfg.dim), dtype=np.int64)
    for ax in range(cfg.dim):
        out[:, ax] = c % full[ax]
        c = c // full[ax]
    return out


# ----------------------------------------------------------------------------- geometry
def _element_centroids(dim: int, nel: int) -> np.ndarray:
    h = 1.0 / nel
    idx = np.arange(nel ** dim)
    cen = np.zeros((nel ** dim, dim))
    r = idx.copy()
    for ax in range(dim):
        cen[:, ax] = (r % nel + 0.5) * h
        r //= nel
    return cen


def _segments(topology: str) -> np.ndarray:
    """Strut axes of a unit cube as (k, 2, 3) endpoint pairs."""
    if topology == "bcc":
        # the four body diagonals (centre-to-corner struts, paired through the centre)
        corners = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0)]
        return np.array([[c, tuple(1 - v for v in c)] for c in corners], dtype=float)
    if topology == "octet":
        segs = []
        for ax in range(3):                      # faces normal to ax at 0 and 1
            o1, o2 = [a for a in range(3) if a != ax]
            for f in (0.0, 1.0):
                for diag in ((0, 0, 1, 1), (1, 0, 0, 1)):
                    p = np.zeros(3); q = np.zeros(3)
                    p[ax] = q[ax] = f
                    p[o1], p[o2], q[o1], q[o2] = diag
                    segs.append((p.copy(), q.copy()))
        centres = []
        for ax in range(3):
            for f in (0.0, 1.0):
                c = np.full(3, 0.5); c[ax] = f
                centres.append((ax, c))
        for i in range(len(centres)):
            for j in range(i + 1, len(centres)):
                if centres[i][0] != centres[j][0]:   # adjacent faces: different normal axes
                    segs.append((centres[i][1], centres[j][1]))
        arr = np.array([[p, q] for p, q in segs], dtype=float)
        assert arr.shape == (24, 2, 3)
        return arr
    raise ValueError(topology)


def _dist_to_segments(pts: np.ndarray, segs: np.ndarray) -> np.ndarray:
    d = np.full(pts.shape[0], np.inf)
    for p, q in segs:
        v = q - p
        t = np.clip(((pts - p) @ v) / (v @ v), 0.0, 1.0)
        proj = p[None, :] + t[:, None] * v[None, :]
        d = np.minimum(d, np.linalg.norm(pts - proj, axis=1))
    return d


def cell_parameters(cfg: LatticeConfig) -> dict:
    """Per-cell radius and topology id (0 = hole/bcc, 1 = octet) for the (sub-)lattice."""
    st = _streams(cfg)
    nfull = int(np.prod(cfg.ncell))
    coords = _cell_coords_full(cfg)
    if cfg.topology == "hole":
        r0, r1 = cfg.radius
        cx = coords[:, 0]
        denom = max(cfg.ncell[0] - 1, 1)
        radius = r0 + (r1 - r0) * cx / denom
        topo = np.zeros(nfull, dtype=np.int32)
    else:
        rng = np.random.default_rng(st["radius"])
        radius = rng.uniform(cfg.radius[0], cfg.radius[1], size=nfull)
        if cfg.topology == "bcc":
            topo = np.zeros(nfull, dtype=np.int32)
        else:
            trng = np.random.default_rng(st["topology"])
            topo = (trng.random(nfull) < 0.5).astype(np.int32)
    ids = _sub_cell_ids(cfg)
    return {"radius": radius[ids], "topology": topo[ids]}


def make_keep(cfg: LatticeConfig) -> np.ndarray:
    """Element keep-mask, uint8 [N_s][n^d].

    hole: an element is removed when its centroid lies within the radius of
    the cell centre; struts: an element is kept when its centroid lies within
    the radius of a strut axis (finite segments).
    """
    par = cell_parameters(cfg)
    cen = _element_centroids(cfg.dim, cfg.nel)
    if cfg.topology == "hole":
        dist = np.linalg.norm(cen - 0.5, axis=1)
        keep = dist[None, :] > par["radius"][:, None]
    else:
        dists = [_dist_to_segments(cen, _segments("bcc"))]
        if cfg.topology == "bcc_octet":
            dists.append(_dist_to_segments(cen, _segments("octet")))
        dist_by_cell = np.stack(dists)[par["topology"]]          # [N_s][n^d]
        keep = dist_by_cell <= par["radius"][:, None]
    return np.ascontiguousarray(keep.astype(np.uint8))


# ----------------------------------------------------------------------------- material
def make_material(cfg: LatticeConfig):
    """Per-cell Lame parameters (mu, lam) as float64 [N_s]."""
    nfull = int(np.prod(cfg.ncell))
    if cfg.mu_law == "const":
        mu = np.full(nfull, cfg.mu[0])
    else:
        rng = np.random.default_rng(_streams(cfg)["mu"])
        lo, hi = cfg.mu
        mu = np.exp(rng.uniform(math.log(lo), math.log(hi), size=nfull))
    lam = cfg.lam_over_mu * mu if cfg.lam_over_mu is not None else np.full(nfull, cfg.lam)
    ids = _sub_cell_ids(cfg)
    return np.ascontiguousarray(mu[ids]), np.ascontiguousarray(lam[ids])


# ----------------------------------------------------------------------------- displacement
def background_shape(cfg: LatticeConfig) -> tuple:
    return tuple(c * cfg.nel + 1 for c in cfg.ncell_eff)


def perturbation_params(cfg: LatticeConfig) -> dict:
    """Three sinusoids per displacement component: wave vectors, phases, weights."""
    rng = np.random.default_rng(_streams(cfg)["pert"])
    d = cfg.dim
    k = rng.uniform(0.1, 0.5, size=(d, 3, d))       # [component][term][axis], cycles per cell edge
    phi = rng.uniform(0.0, 2 * math.pi, size=(d, 3))
    a = rng.uniform(0.5, 1.0, size=(d, 3))
    a = a / a.sum(axis=1, keepdims=True)              # |perturbation| <= amplitude
    return {"k": k, "phi": phi, "a": a}


def make_displacement(cfg: LatticeConfig, dtype=np.float64) -> np.ndarray:
    """Displacement on the background node grid, [G][d] with G = prod(background_shape).

    u(X) = -strain * X_d e_d + A sum_j a_j sin(2 pi k_j . X + phi_j) per component, X in cell
    edges (uniaxial strain along the last axis plus a smooth seeded perturbation).
    """
    d = cfg.dim
    shp = background_shape(cfg)
    h = 1.0 / cfg.nel
    axes = [np.arange(s) * h for s in shp]
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]     # x fastest in the flattened order
    Xs = [g.reshape(-1) for g in grids]
    par = perturbation_params(cfg)
    G = Xs[0].size
    u = np.zeros((G, d), dtype=dtype)
    for i in range(d):
        acc = np.zeros(G)
        for j in range(3):
            ph = par["phi"][i, j] + sum(2 * math.pi * par["k"][i, j, ax] * Xs[ax] for ax in range(d))
            acc += par["a"][i, j] * np.sin(ph)
        u[:, i] = cfg.pert_amp * acc
    u[:, d - 1] += -cfg.strain * Xs[d - 1]
    return u


def cell_background_nodes(cfg: LatticeConfig, cell: int) -> np.ndarray:
    """Background-grid ids of the (n+1)^d local nodes of one cell (x fastest)."""
    sub = cfg.ncell_eff
    shp = background_shape(cfg)
    n = cfg.nel
    cc = []
    r = cell
    for ax in range(cfg.dim):
        cc.append(r % sub[ax]); r //= sub[ax]
    loc = np.arange((n + 1) ** cfg.dim)
    gid = np.zeros_like(loc)
    stride = 1
    r = loc.copy()
    for ax in range(cfg.dim):
        gid += (cc[ax] * n + r % (n + 1)) * stride
        r //= (n + 1)
        stride *= shp[ax]
    return gid


def local_displacements(cfg: LatticeConfig, u_bg: np.ndarray) -> np.ndarray:
    """Displacement restricted to each cell's local nodes, [N_s][(n+1)^d][d] (no masking)."""
    out = np.empty((cfg.n_cells, cfg.n_local_nodes, cfg.dim))
    for c in range(cfg.n_cells):
        out[c] = u_bg[cell_background_nodes(cfg, c)]
    return out


# ----------------------------------------------------------------------------- right-hand sides
def make_rhs(cfg: LatticeConfig, cells: Optional[Sequence[int]] = None, m: Optional[int] = None,
             stream: int = 0) -> np.ndarray:
    """Right-hand sides X, float64 [len(cells)][(n+1)^d][d][m], i.i.d. N(0,1).

    Each cell's block comes from its own counter-keyed stream, so any subset of cells can be
    regenerated independently.  Entries at DOFs a cell does not own are ignored by the applies.
    `stream` selects an independent family (e.g. 1 for adjoint cotangents).
    """
    m = cfg.m if m is None else m
    cells = range(cfg.n_cells) if cells is None else cells
    seed = int(_streams(cfg)["rhs"].generate_state(1)[0])
    ids = _sub_cell_ids(cfg)
    out = np.empty((len(cells), cfg.n_local_nodes, cfg.dim, m))
    for t, c in enumerate(cells):
        rng = np.random.default_rng([seed, stream, int(ids[c]), m])
        out[t] = rng.standard_normal((cfg.n_local_nodes, cfg.dim, m))
    return out


# ----------------------------------------------------------------------------- boundary-value problems
@dataclasses.dataclass(frozen=True)
class LoadCase:
    """Loading of a lattice for the load-stepped Newton solve.

    kind "compress_shear": the bottom face (last coordinate 0) is clamped, the top face
      (last coordinate = lattice height H) is moved by (shear H, -strain H) [2D] or
      (shear H, 0, -strain H) [3D]; every component of both faces is prescribed.
    kind "uniaxial_roller": symmetry rollers: the last component is prescribed on the bottom (0)
      and top (-strain H) faces, the first component on the face x = 0 and, in 3D, the second
      component on the face y = 0 (all 0), so that no rigid motion remains.
    """
    kind: str
    strain: float
    shear: float = 0.0
    n_inc: int = 4


def make_bvp(cfg: LatticeConfig, case: LoadCase) -> dict:
    """Dirichlet data on the background node grid for a load case.

    Returns fixed uint8 [G][d] (1 = prescribed component) and ubar float64 [G][d]: the affine
    displacement field of the whole load at every background node, which equals the prescribed
    value on the constrained components (the solver adds ubar / n_inc to every node at the start
    of each increment).  f_ext float64 [G][d] is zero (displacement-driven cases).
    """
    d = cfg.dim
    shp = background_shape(cfg)
    h = 1.0 / cfg.nel
    axes = [np.arange(s) for s in shp]
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    I = [g.reshape(-1) for g in grids]                  # integer grid coordinates, x fastest
    G = I[0].size
    top = shp[d - 1] - 1
    H = top * h
    z = I[d - 1] * h
    fixed = np.zeros((G, d), np.uint8)
    ubar = np.zeros((G, d))
    bot_m = I[d - 1] == 0
    top_m = I[d - 1] == top
    if case.kind == "compress_shear":
        fixed[bot_m | top_m, :] = 1
        ubar[:, 0] = case.shear * z
        ubar[:, d - 1] = -case.strain * z
    elif case.kind == "uniaxial_roller":
        fixed[bot_m | top_m, d - 1] = 1
        for ax in range(d - 1):
            fixed[I[ax] == 0, ax] = 1
        ubar[:, d - 1] = -case.strain * z
    else:
        raise ValueError(case.kind)
    return {"fixed": fixed, "ubar": ubar, "f_ext": np.zeros((G, d)), "height": H}
