"""FETI-DP partition of the cells' local degrees of freedom: FP64/integer CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by `tests/`, never by the product library.  It shares no code
with the GPU path.

Sec. 3.3 treats every unit cell as a subdomain.  Its local nodes fall into
  * primal nodes: the cell corners, kept continuous by a global (coarse) numbering; when a local
    remaining matrix is not definite, one more primal node is added on every cell edge, and again
    (Sec. 3.3.2, "Enhanced coarse problem");
  * dual nodes: the other nodes on the cell boundary, whose continuity across the interface is
    imposed weakly by Lagrange multipliers (the rows of B);
  * interior nodes: the rest.  Remaining = dual + interior.
Readings fixed here (the paper leaves them to its reference solver):
  * edge primal nodes at enrichment level e sit at the edge coordinates round(k n / (e + 1)),
    k = 1..e (halves rounded up), so every cell sharing an edge selects the same nodes;
  * a dual node shared by k >= 2 cells (where it is active) carries k - 1 multipliers chaining
    the cells in ascending id, so B has full row rank;
  * multipliers are numbered by global node, then chain position; the node classes are those of
    the union of the cells' active nodes (a node active in no cell has no class, -1).
"""
from __future__ import annotations

import numpy as np

INTERIOR, DUAL, PRIMAL = 0, 1, 2


def edge_positions(nel: int, level: int):
    """Edge coordinates of the primal nodes added at enrichment `level` (sorted, within 1..nel-1)."""
    pos = set()
    for k in range(1, level + 1):
        t = (2 * k * nel + level + 1) // (2 * (level + 1))     # round(k nel / (level + 1)), halves up
        pos.add(min(max(t, 1), nel - 1))
    return sorted(pos)


def local_coords(dim: int, nel: int):
    nn = nel + 1
    a = np.arange(nn ** dim)
    return np.stack([(a // nn ** ax) % nn for ax in range(dim)], axis=1)


def node_classes(dim: int, nel: int, level: int, l2g: np.ndarray):
    """Class of every local node (identical in every cell): -1 never active, 0 interior, 1 dual,
    2 primal."""
    xy = local_coords(dim, nel)
    onb = (xy == 0) | (xy == nel)
    nb = onb.sum(axis=1)
    tpos = set(edge_positions(nel, level))
    cls = np.full(len(xy), INTERIOR, np.int32)
    for a in range(len(xy)):
        if nb[a] == dim:
            cls[a] = PRIMAL                                      # a cell corner
        elif nb[a] == dim - 1:                                   # on a cell edge: one free coordinate
            free = int(xy[a][~onb[a]][0])
            cls[a] = PRIMAL if free in tpos else DUAL
        elif nb[a] >= 1:
            cls[a] = DUAL                                        # on a face (3D)
    active = (l2g >= 0).any(axis=0)
    cls[~active] = -1
    return cls


def partition(dim: int, nel: int, l2g: np.ndarray, level: int):
    """Primal global nodes and multipliers of the lattice with local-to-global map l2g [N_s][nloc].

    Returns dict(cls [nloc], primal [n_p] sorted global node ids, mult [n_mult][4] rows
    (cell_1, a_1, cell_2, a_2) with cell_1 < cell_2 consecutive owners of one dual node)."""
    cls = node_classes(dim, nel, level, l2g)
    Ns, nloc = l2g.shape
    owners = {}
    for c in range(Ns):
        for a in range(nloc):
            g = int(l2g[c, a])
            if g >= 0:
                owners.setdefault(g, []).append((c, a))
    primal = sorted(g for g, ow in owners.items() if cls[ow[0][1]] == PRIMAL)
    mult = []
    for g in sorted(owners):
        ow = owners[g]
        if cls[ow[0][1]] != DUAL or len(ow) < 2:
            continue
        for t in range(len(ow) - 1):
            mult.append((ow[t][0], ow[t][1], ow[t + 1][0], ow[t + 1][1]))
    return {"cls": cls, "primal": np.asarray(primal, np.int64),
            "mult": np.asarray(mult, np.int32).reshape(-1, 4)}
