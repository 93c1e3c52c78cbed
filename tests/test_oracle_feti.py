"""Pins of the oracle's FETI-DP partition (Sec. 3.3: primal corner nodes, edge enrichment, dual
nodes with Lagrange multipliers) by closed-form counts on fully solid lattices, by structural
invariants on the masked lattices, and by the rank of the jump operator B."""
import itertools

import numpy as np
import pytest

import lattice as L
from oracle import feti as F


def _full(orc, dim, ncell, nel):
    keep = np.ones((int(np.prod(ncell)), nel ** dim), np.uint8)
    l2g, _, g2bg = orc.dofmap(dim, ncell, nel, keep)
    return l2g, g2bg


def test_edge_positions():
    assert F.edge_positions(32, 0) == []
    assert F.edge_positions(32, 1) == [16]
    assert F.edge_positions(32, 3) == [8, 16, 24]
    assert F.edge_positions(12, 2) == [4, 8]
    assert F.edge_positions(5, 1) == [3]                  # 2.5 rounds up
    assert F.edge_positions(2, 4) == [1]                  # clipped to the edge interior
    for n, e in itertools.product([6, 12, 16, 32], range(1, 5)):
        p = F.edge_positions(n, e)
        if n >= 2 * (e + 1):
            assert len(p) == e                    # distinct when the spacing is at least 2
        assert all(1 <= t <= n - 1 for t in p)


@pytest.mark.parametrize("cx,cy,n,e", [(3, 2, 4, 0), (4, 3, 6, 0), (4, 3, 6, 1), (2, 5, 8, 2), (1, 1, 4, 0)])
def test_counts_2d_full_lattice(orc, cx, cy, n, e):
    l2g, _ = _full(orc, 2, (cx, cy), n)
    p = F.partition(2, n, l2g, e)
    horiz = cx * (cy + 1)                         # cell edges parallel to x
    vert = (cx + 1) * cy
    assert len(p["primal"]) == (cx + 1) * (cy + 1) + e * (horiz + vert)
    # an interface edge between two cells: its n - 1 inner nodes minus the e edge primal nodes,
    # one multiplier each; outer edges carry none
    interfaces = (cx - 1) * cy + cx * (cy - 1)
    assert len(p["mult"]) == (n - 1 - e) * interfaces
    cls = p["cls"]
    assert (cls == F.PRIMAL).sum() == 4 + 4 * e
    assert (cls == F.DUAL).sum() == 4 * (n - 1 - e)
    assert (cls == F.INTERIOR).sum() == (n - 1) ** 2


@pytest.mark.parametrize("c,n,e", [((2, 2, 2), 3, 0), ((3, 2, 2), 4, 0), ((2, 3, 2), 4, 1)])
def test_counts_3d_full_lattice(orc, c, n, e):
    l2g, _ = _full(orc, 3, c, n)
    p = F.partition(3, n, l2g, e)
    nprim_edges = 0
    mult = 0
    for ax in range(3):                           # cell edges parallel to axis ax
        o1, o2 = [b for b in range(3) if b != ax]
        for j, k in itertools.product(range(c[o1] + 1), range(c[o2] + 1)):
            share = (1 if j in (0, c[o1]) else 2) * (1 if k in (0, c[o2]) else 2)
            nprim_edges += c[ax]
            mult += c[ax] * (n - 1 - e) * (share - 1)
    for ax in range(3):                           # interior faces normal to ax: (n - 1)^2 inner nodes
        o1, o2 = [b for b in range(3) if b != ax]
        mult += (c[ax] - 1) * c[o1] * c[o2] * (n - 1) ** 2
    assert len(p["primal"]) == np.prod([x + 1 for x in c]) + e * nprim_edges
    assert len(p["mult"]) == mult
    cls = p["cls"]
    assert (cls == F.PRIMAL).sum() == 8 + 12 * e
    assert (cls == F.DUAL).sum() == 12 * (n - 1 - e) + 6 * (n - 1) ** 2
    assert (cls == F.INTERIOR).sum() == (n - 1) ** 3


@pytest.mark.parametrize("idx,sub,e", [(0, (3, 3), 0), (1, (4, 3), 1), (2, (2, 2, 2), 0), (4, (2, 2, 2), 1)])
def test_invariants_masked_lattices(orc, idx, sub, e):
    cfg = L.config(idx).with_sub(sub)
    keep = L.make_keep(cfg)
    l2g, _, _ = orc.dofmap(cfg.dim, cfg.ncell_eff, cfg.nel, keep)
    p = F.partition(cfg.dim, cfg.nel, l2g, e)
    cls, mult, prim = p["cls"], p["mult"], p["primal"]
    owners = {}
    for cc in range(l2g.shape[0]):
        for a in np.nonzero(l2g[cc] >= 0)[0]:
            owners.setdefault(int(l2g[cc, a]), []).append((cc, int(a)))
    # every owner of a node gives it the same class (the classes are geometric)
    for g, ow in owners.items():
        assert len({int(cls[a]) for _, a in ow}) == 1
    # multipliers: same global node on both sides, ascending consecutive owners, k - 1 per dual
    # node of k owners, none on primal or interior nodes
    per = {}
    for c1, a1, c2, a2 in mult:
        g = int(l2g[c1, a1])
        assert g == int(l2g[c2, a2]) and c1 < c2 and cls[a1] == F.DUAL
        per.setdefault(g, []).append((int(c1), int(c2)))
    for g, ow in owners.items():
        k = len(ow)
        if cls[ow[0][1]] == F.DUAL and k >= 2:
            chain = per[g]
            assert chain == [(ow[t][0], ow[t + 1][0]) for t in range(k - 1)]
        else:
            assert g not in per
    assert sorted(prim.tolist()) == sorted(g for g, ow in owners.items() if cls[ow[0][1]] == F.PRIMAL)
    # the jump operator on the dual DOFs has full row rank
    if len(mult):
        col = {}
        for c1, a1, c2, a2 in mult:
            col.setdefault((int(c1), int(a1)), len(col))
            col.setdefault((int(c2), int(a2)), len(col))
        B = np.zeros((len(mult), len(col)))
        for r, (c1, a1, c2, a2) in enumerate(mult):
            B[r, col[(int(c1), int(a1))]] = 1.0
            B[r, col[(int(c2), int(a2))]] = -1.0
        assert np.linalg.matrix_rank(B) == len(mult)


def test_enrichment_only_adds_primal_nodes(orc):
    cfg = L.config(1).with_sub((3, 3))
    keep = L.make_keep(cfg)
    l2g, _, _ = orc.dofmap(cfg.dim, cfg.ncell_eff, cfg.nel, keep)
    p0 = F.partition(2, cfg.nel, l2g, 0)
    p1 = F.partition(2, cfg.nel, l2g, 1)
    assert set(p0["primal"].tolist()) < set(p1["primal"].tolist())
    assert np.all((p1["cls"] == F.PRIMAL) >= (p0["cls"] == F.PRIMAL))
    assert len(p1["mult"]) < len(p0["mult"])
