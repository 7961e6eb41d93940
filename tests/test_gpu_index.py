"""Point location on the GPU through both indexes: the hash of sibling
groups (amr_build_index, what the extraction uses) and the paper's sorted
cells with a binary search per level (amr_build_sorted_index, sec. 3.2).

Bar: for every query point, both return the cell the oracle's locator
returns (the unique cell containing the point, -1 where none does), bit for
bit; the snap queries of every cell (27 points per cell) give the same
count and checksum through both, and through the oracle on small sets.
"""
import numpy as np
import pytest

import amrgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amr():
    import paper_2004_08475_amd as amr

    amr.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return amr


def _say(msg):
    print(msg, flush=True)


def _points(cs, k, seed, pad=3):
    w = (1 << cs.level.astype(np.int64))[:, None]
    lo = cs.xyz.min(0) - pad
    hi = (cs.xyz + w).max(0) + pad
    return np.random.default_rng(seed).integers(lo, hi, (k, 3)).astype(np.int32)


def _snap_oracle(o, cs):
    found, total = 0, 0
    offs = [(ox, oy, oz) for oz in (-1, 0, 1) for oy in (-1, 0, 1) for ox in (-1, 0, 1)]
    for (x, y, z), l in zip(cs.xyz.tolist(), cs.level.tolist()):
        w = 1 << l
        for ox, oy, oz in offs:
            c = o.locate((x + ox * w, y + oy * w, z + oz * w))
            if c >= 0:
                found += 1
                total += c + 1
    return found, total


CASES = {
    "two-level-sphere-16": lambda: amrgen.two_level_sphere(),
    "random-octree-holes": lambda: amrgen.random_octree(7, roots=3, root_level=4, p_split=0.45, p_hole=0.15,
                                                        values="smooth", origin=(-64, 32, -16)),
    "random-octree-deep": lambda: amrgen.random_octree(104, roots=2, root_level=5, p_split=0.4, p_hole=0.0),
    "grid-9-level1": lambda: amrgen.uniform_grid(9, level=1, origin=(-6, 10, 2)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_locate_and_snaps_match_oracle(amr, name):
    cs = CASES[name]()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    s.build_sorted_index()
    pts = _points(cs, 4000, 5)
    tp = torch.from_numpy(pts)
    h = s.locate(tp, amr.INDEX_HASH).cpu().numpy()
    q = s.locate(tp, amr.INDEX_SORTED).cpu().numpy()
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    want = np.array([o.locate(p) for p in pts.tolist()], np.int32)
    assert np.array_equal(h, want)
    assert np.array_equal(q, want)
    _say("%s: %d of %d points inside a cell" % (name, int((want >= 0).sum()), len(want)))
    out = torch.zeros(2, dtype=torch.int64, device=s.device)
    res = []
    for kind in (amr.INDEX_HASH, amr.INDEX_SORTED):
        s.snap_count_into(out, kind)
        res.append(tuple(out.cpu().tolist()))
    assert res[0] == res[1] == _snap_oracle(o, cs)


def test_index_edge_cases(amr):
    cs = amrgen.two_level_sphere()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    with pytest.raises(amr.AmrError):
        s.locate(torch.zeros((1, 3), dtype=torch.int32), amr.INDEX_SORTED)  # not built yet
    s.build_sorted_index()
    far = torch.tensor([[1 << 22, 0, 0], [-(1 << 22), 5, 5], [-1, -1, -1], [16, 16, 16]], dtype=torch.int32)
    for kind in (amr.INDEX_HASH, amr.INDEX_SORTED):
        assert (s.locate(far, kind) == -1).all()
        assert s.locate(torch.zeros((0, 3), dtype=torch.int32), kind).numel() == 0
    e = amr.from_numpy(np.zeros((0, 3), np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    e.build_sorted_index()
    out = torch.ones(2, dtype=torch.int64, device=e.device)
    e.snap_count_into(out, amr.INDEX_SORTED)
    assert out.tolist() == [0, 0]
    assert (e.locate(far, amr.INDEX_SORTED) == -1).all()


def test_index_two_million_cells(amr):
    """The ~2M-cell octree: 20,000 random points against the oracle's
    locator, and the snap counts of all 2M cells equal through both."""
    cs = amrgen.octree_shell_2m()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    s.build_sorted_index()
    pts = _points(cs, 20000, 9)
    tp = torch.from_numpy(pts)
    h = s.locate(tp, amr.INDEX_HASH).cpu().numpy()
    q = s.locate(tp, amr.INDEX_SORTED).cpu().numpy()
    o = oracle.Oracle(cs.xyz, cs.level, cs.value, validate=False)
    want = np.array([o.locate(p) for p in pts.tolist()], np.int32)
    assert np.array_equal(h, want) and np.array_equal(q, want)
    out = torch.zeros(2, dtype=torch.int64, device=s.device)
    res = []
    for kind in (amr.INDEX_HASH, amr.INDEX_SORTED):
        s.snap_count_into(out, kind)
        res.append(tuple(out.cpu().tolist()))
    _say("2M cells: snaps found %d" % res[0][0])
    assert res[0] == res[1] and res[0][0] > 27 * cs.n // 2


def test_index_block_vortex_full_size(amr):
    """The 50.8M-cell block-structured set with a hole: snap counts equal
    through both indexes; 200,000 points near cells (inside and around the
    obstacle) located alike by both."""
    cs = amrgen.block_vortex(device="cuda")
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    s.build_sorted_index()
    out = torch.zeros(2, dtype=torch.int64, device=s.device)
    res = []
    for kind in (amr.INDEX_HASH, amr.INDEX_SORTED):
        s.snap_count_into(out, kind)
        res.append(tuple(out.cpu().tolist()))
    _say("block-vortex: snaps found %d of %d" % (res[0][0], 27 * cs.n))
    assert res[0] == res[1]
    rng = np.random.default_rng(13)
    pick = rng.integers(0, cs.n, 100000)
    near = cs.xyz[pick] + rng.integers(-9, 10, (100000, 3)).astype(np.int32)
    (ox0, ox1), (oy0, oy1), (oz0, oz1) = cs.meta["obstacle"]
    hole = rng.integers([ox0 - 4, oy0 - 4, oz0 - 4], [ox1 + 4, oy1 + 4, oz1 + 4], (100000, 3)).astype(np.int32)
    tp = torch.from_numpy(np.concatenate([near, hole]))
    h = s.locate(tp, amr.INDEX_HASH)
    q = s.locate(tp, amr.INDEX_SORTED)
    assert torch.equal(h, q)
    # each found cell contains its point
    hc = h.cpu().numpy()
    pts = tp.numpy()
    f = hc >= 0
    lo = cs.xyz[hc[f]]
    w = (1 << cs.level[hc[f]].astype(np.int64))[:, None]
    assert np.all((lo <= pts[f]) & (pts[f] < lo + w))
