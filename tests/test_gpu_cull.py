"""Range culling of iso-surface passes gives the same outputs as full passes.

The second extraction after a build records, per 2x2x2 group, the value
range of the group's 4x4x4 neighbourhood and the set's dual count; later iso
calls that do not ask for dual indices skip groups whose range cannot
straddle iso.  Full passes are the reference here: a call that asks for dual
indices never culls, nor do the first two calls after a build.  Bar:
triangles and cell pairs bit for bit equal, dual counts equal, and the
oracle's triangle and dual counts at the set's own iso.
"""
import os
import sys

import numpy as np
import pytest

import amrgen
import oracle

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _util import canon_by_cells  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amr():
    import paper_2004_08475_amd as amr

    amr.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return amr


CASES = {
    # 530 tiles: the fused single pass
    "octree-shell-256": lambda: amrgen.octree_shell(),
    # 2,879 tiles: count / scan / write passes
    "octree-sized-647k": lambda: amrgen.octree_sized(800_000, seed=9),
    "random-octree-holes": lambda: amrgen.random_octree(7, roots=4, root_level=4, p_split=0.45, p_hole=0.15,
                                                        values="smooth", origin=(-64, 32, -16)),
}


def _isos(value):
    v = np.sort(np.asarray(value, np.float32))
    mid = v[len(v) // 2]
    return [
        float(v[0]) - 1.0,       # below every cell: nothing survives the cull
        float(v[0]),             # the minimum itself (cells equal to iso count as >= iso)
        float(np.quantile(v, 0.01)),
        float(np.quantile(v, 0.3)),
        float(mid),              # exactly a cell's value
        float(np.nextafter(mid, np.float32(np.inf))),
        float(np.quantile(v, 0.9)),
        float(v[-1]),            # the maximum itself
        float(v[-1]) + 1.0,
    ]


def _full(s, iso):
    """A full pass: asking for dual indices turns the cull off."""
    r = s.isosurface(iso, cells=True, dual=True)
    return r["tris"], r["cells"], r["n_duals"]


@pytest.mark.parametrize("name", list(CASES))
def test_culled_passes_equal_full_passes(amr, name):
    cs = CASES[name]()
    print("cull %s: %d cells" % (name, cs.n), flush=True)
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    # first call after the build: a full pass (the next one records the ranges)
    t0, d0 = s.count(cs.iso)
    ro = oracle.Oracle(cs.xyz, cs.level, cs.value).isosurface(cs.iso)
    assert t0 == len(ro["tris"]) and d0 == ro["n_duals"]
    for iso in _isos(cs.value):
        tf, cf, df = _full(s, iso)
        # culled count, culled count + write (two-pass), culled single pass
        assert s.count(iso) == (len(tf), d0)
        r = s.isosurface(iso, cells=True)
        assert r["n_duals"] == df == d0
        assert torch.equal(r["tris"], tf) and torch.equal(r["cells"], cf)
        r1 = s.isosurface(iso, cap=len(tf) + 5)
        assert torch.equal(r1["tris"], tf)
    # at the set's own iso the culled count still matches the oracle
    assert s.count(cs.iso) == (len(ro["tris"]), ro["n_duals"])


def test_ranges_recorded_by_dual_cells(amr):
    cs = amrgen.octree_sized(800_000, seed=9)
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    pl, _ = s.dual_cells()  # a counting call, then the recording one
    iso = float(np.quantile(cs.value, 0.6))
    r = s.isosurface(iso, cells=True)
    tf, cf, df = _full(s, iso)
    assert r["n_duals"] == df == len(pl)
    assert torch.equal(r["tris"], tf) and torch.equal(r["cells"], cf)


@pytest.mark.parametrize("name", ["octree-shell-256", "octree-sized-647k"])
def test_rebuild_forgets_ranges(amr, name):
    # same cells, negated values: every recorded range is wrong for the new
    # field, so a culled pass on stale ranges would lose triangles
    cs = CASES[name]()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    for _ in range(3):
        s.count(cs.iso)  # full, recording, culled
    dev = s.device
    xyz = torch.from_numpy(np.ascontiguousarray(cs.xyz, np.int32)).to(dev)
    lvl = torch.from_numpy(np.ascontiguousarray(cs.level, np.int32)).to(dev)
    neg = torch.from_numpy(np.ascontiguousarray(-cs.value, np.float32)).to(dev)
    s.upload(xyz, lvl, neg)
    s.build_index()
    fresh = amr.from_numpy(cs.xyz, cs.level, -cs.value)
    for iso in (-cs.iso, float(np.quantile(-cs.value, 0.2))):
        a = s.isosurface(iso, cells=True)
        b = fresh.isosurface(iso, cells=True, dual=True)
        assert a["n_duals"] == b["n_duals"]
        # two builds may order their groups differently: compare by topology
        ta, ca, _ = canon_by_cells(a["tris"].cpu().numpy(), a["cells"].cpu().numpy())
        tb, cb, _ = canon_by_cells(b["tris"].cpu().numpy(), b["cells"].cpu().numpy())
        assert np.array_equal(ca, cb)
        assert np.array_equal(ta.view(np.uint32), tb.view(np.uint32))


@pytest.mark.parametrize("name", ["octree-sized-647k"])
def test_first_writes_over_groups_with_triangles(amr, name):
    # Right after a build (nothing recorded yet) a write on a set of more
    # than 2048 tiles counts over all groups, lists the groups with
    # triangles and writes over that list only: same bits, same order as the
    # full write pass (the one that also names each triangle's dual).
    cs = CASES[name]()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    for q in (0.1, 0.5, 0.93):
        iso = float(np.quantile(cs.value, q))
        s.build_index()  # forget everything recorded
        n, d = s.count(iso)
        r = s.isosurface(iso, cap=n + 3, cells=True)  # second extraction: also records
        f = s.isosurface(iso, cells=True, dual=True)
        assert r["n_duals"] == f["n_duals"] == d
        assert torch.equal(r["tris"], f["tris"]) and torch.equal(r["cells"], f["cells"])
        s.build_index()
        r1 = s.isosurface(iso, cap=n, cells=True)  # the very first extraction
        f1 = s.isosurface(iso, cells=True, dual=True)  # same build (a rebuild may order groups differently)
        assert r1["n_duals"] == f1["n_duals"] == d
        assert torch.equal(r1["tris"], f1["tris"]) and torch.equal(r1["cells"], f1["cells"])
    # no triangles at all: an empty list, an empty scan, nothing written
    s.build_index()
    buf = torch.full((5, 9), -7.0, dtype=torch.float32, device=s.device)
    counts = s.isosurface_into(float(np.min(cs.value)) - 1.0, buf, 5)
    assert counts.tolist() == [0, d]
    assert torch.all(buf == -7.0)
