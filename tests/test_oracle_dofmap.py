"""Pins of the oracle's DOF maps (the Boolean assembly operators A^s of eq. residualvector)
against an independent set-based enumeration, plus interface consistency."""
import numpy as np
import pytest

import lattice as L


def _enumerate(cfg, keep):
    """Independent brute force: sets of background ids of kept elements' corners."""
    dim, n = cfg.dim, cfg.nel
    sub = cfg.ncell_eff
    shp = L.background_shape(cfg)
    per_cell = []
    allg = set()
    for c in range(cfg.n_cells):
        cc = []
        r = c
        for ax in range(dim):
            cc.append(r % sub[ax]); r //= sub[ax]
        nodes = {}
        for e in np.nonzero(keep[c])[0]:
            ie = [(int(e) // n ** ax) % n for ax in range(dim)]
            for k in range(2 ** dim):
                loc = [ie[ax] + ((k >> ax) & 1) for ax in range(dim)]
                a = sum(loc[ax] * (n + 1) ** ax for ax in range(dim))
                g = 0
                st = 1
                for ax in range(dim):
                    g += (cc[ax] * n + loc[ax]) * st
                    st *= shp[ax]
                nodes[a] = g
        per_cell.append(nodes)
        allg.update(nodes.values())
    order = {g: i for i, g in enumerate(sorted(allg))}
    return per_cell, order


@pytest.mark.parametrize("idx,sub", [(0, None), (1, (5, 4)), (2, (2, 3, 2)), (4, (2, 2, 2))])
def test_dofmap_matches_enumeration(orc, idx, sub):
    cfg = L.config(idx)
    if sub is not None:
        cfg = cfg.with_sub(sub)
    keep = L.make_keep(cfg)
    l2g, nact, g2bg = orc.dofmap(cfg.dim, cfg.ncell_eff, cfg.nel, keep)
    per_cell, order = _enumerate(cfg, keep)
    assert len(g2bg) == len(order)
    assert np.all(np.diff(g2bg) > 0)
    for c, nodes in enumerate(per_cell):
        assert nact[c] == len(nodes)
        exp = np.full(cfg.n_local_nodes, -1, np.int32)
        for a, g in nodes.items():
            exp[a] = order[g]
        np.testing.assert_array_equal(l2g[c], exp)


def test_hole_lattice_counts(orc):
    # 4x4 cells of 16^2 quads with a hole of radius 0.30: 180 kept elements, 232 active nodes
    # per cell; the interface nodes are shared, giving 3313 distinct active nodes.
    cfg = L.config(0)
    keep = L.make_keep(cfg)
    l2g, nact, g2bg = orc.dofmap(2, cfg.ncell, cfg.nel, keep)
    assert np.all(keep.sum(1) == 180)
    assert np.all(nact == 232)
    # independent count: distinct background ids over the cells' owned nodes
    ids = np.concatenate([L.cell_background_nodes(cfg, c)[l2g[c] >= 0] for c in range(cfg.n_cells)])
    assert len(g2bg) == len(np.unique(ids)) == 3313


def test_interface_consistency(orc):
    # a global id shared by two cells maps to the same background node from both sides
    cfg = L.config(2).with_sub((3, 2, 2))
    keep = L.make_keep(cfg)
    l2g, _, g2bg = orc.dofmap(3, cfg.ncell_eff, cfg.nel, keep)
    for c in range(cfg.n_cells):
        bg = L.cell_background_nodes(cfg, c)
        m = l2g[c] >= 0
        np.testing.assert_array_equal(g2bg[l2g[c][m]], bg[m])
