"""Comparison helpers shared by the GPU parity tests."""
import numpy as np


def canon_by_cells(tris, cells, dual_ids=None):
    """Canonical triangle order by topology.  Each vertex is keyed by its
    (A, B) cell pair; every triangle is rotated (winding kept) so that its
    smallest key comes first, then triangles are sorted by their six ints.
    Returns (tris [T,9], cells [T,6], dual keys or None)."""
    t = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    c = np.asarray(cells, np.int64).reshape(-1, 3, 2)
    n = len(t)
    if n == 0:
        return t.reshape(0, 9), c.reshape(0, 6), None
    key = c[:, :, 0] * (1 << 32) + c[:, :, 1]
    first = np.argmin(key, axis=1)
    idx = (first[:, None] + np.arange(3)[None]) % 3
    t = np.take_along_axis(t, idx[:, :, None], 1).reshape(n, 9)
    c = np.take_along_axis(c, idx[:, :, None], 1).reshape(n, 6)
    order = np.lexsort(tuple(c[:, i] for i in range(5, -1, -1)))
    d = None if dual_ids is None else np.asarray(dual_ids)[order]
    return t[order], c[order], d


def same_positions(a, b):
    """True when two float32 position arrays are equal bit for bit.  Both
    sides place a vertex with the same IEEE float32 operations (cell centres
    exact in float32, a correctly rounded division, one fused multiply-add),
    so the gate is equality of the bits, tighter than 1e-5 of the finest cell
    width and than one unit in the last place."""
    a = np.ascontiguousarray(np.asarray(a, np.float32))
    b = np.ascontiguousarray(np.asarray(b, np.float32))
    return a.shape == b.shape and np.array_equal(a.view(np.uint32), b.view(np.uint32))


def directed_edges(cells):
    from collections import Counter

    cnt = Counter()
    for tri in np.asarray(cells).reshape(-1, 3, 2):
        ks = [tuple(sorted(map(int, v))) for v in tri]
        for i in range(3):
            cnt[(ks[i], ks[(i + 1) % 3])] += 1
    return cnt


def owner_of_duals(pl, ids, level):
    """Generating cell of each dual under rule 3: the cell in the lowest slot
    whose level equals the dual's level."""
    lv = np.asarray(level)[ids]
    same = lv == pl[:, 3:4]
    first = np.argmax(same, axis=1)
    return ids[np.arange(len(ids)), first]


def window_matches_oracle(o, iso, pl, ids, tris, cells, dual, c0, c1):
    """The GPU's triangles whose generating dual is owned by a cell in
    [c0, c1) against the oracle's triangles for that range of cells: count,
    cell-pair topology after canonical order, positions bit for bit.
    `pl`, `ids` are the GPU's dual cells (numpy); `tris`, `cells`, `dual` its
    triangles with their cell pairs and dual indices.  Returns the number of
    triangles compared."""
    owner = owner_of_duals(pl, ids, o.level)
    sel = (owner >= c0) & (owner < c1)
    tsel = sel[np.asarray(dual)]
    ro = o.isosurface(float(iso), c0, c1)
    A, AC, _ = canon_by_cells(np.asarray(tris)[tsel], np.asarray(cells)[tsel])
    B, BC, _ = canon_by_cells(ro["tris"], ro["cells"])
    assert len(A) == len(B)
    assert np.array_equal(AC, BC)
    assert same_positions(A, B)
    return len(A)
