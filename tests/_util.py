"""Comparison helpers shared by the GPU parity tests (no method arithmetic)."""
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


def position_tolerance(ref, w0=1.0):
    """|delta| <= max(1e-5 * finest width, 2 ulp_f32(|x|))."""
    return np.maximum(1e-5 * w0, 2.0 * np.spacing(np.abs(np.asarray(ref, np.float32))).astype(np.float64))


def directed_edges(cells):
    from collections import Counter

    cnt = Counter()
    for tri in np.asarray(cells).reshape(-1, 3, 2):
        ks = [tuple(sorted(map(int, v))) for v in tri]
        for i in range(3):
            cnt[(ks[i], ks[(i + 1) % 3])] += 1
    return cnt
