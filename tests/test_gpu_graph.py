"""Whole steps in HIP graphs, and the build's verdict on the device.

amr_upload, amr_build_index and amr_isosurface do no host synchronisation
(the build decides its verdict on the device, and extraction kernels read
the group count and geometry from there), so one graph can hold a whole
step.  Replays with new cell values or moved cells must equal eager runs and
the oracle.  A failed build makes extractions report -1, and the host learns
why from amr_build_status.  A recording call captured and never replayed
must not make later calls cull with ranges that were never written.
"""
import os
import sys

import numpy as np
import pytest

import amrgen
import oracle

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _util import same_positions  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amr():
    import paper_2004_08475_amd as amr

    amr.load_library()
    assert torch.cuda.is_available()
    return amr


def _say(msg):
    print(msg, flush=True)


def _as_set(tris):
    """Triangles in a canonical order by position (build-independent)."""
    return oracle.canonical_triangles(np.asarray(tris, np.float32))[0]


@pytest.mark.parametrize("name", ["octree-shell-256", "octree-sized-647k"])
def test_upload_build_iso_in_one_graph(amr, name):
    cs = amrgen.octree_shell() if name == "octree-shell-256" else amrgen.octree_sized(800_000, seed=9)
    _say("graph step %s: %d cells" % (name, cs.n))
    dev = torch.device("cuda", 0)
    xyz = torch.from_numpy(cs.xyz).to(dev)
    lvl = torch.from_numpy(cs.level).to(dev)
    val = torch.from_numpy(cs.value).to(dev)
    s = amr.AmrSet(0)
    s.upload(xyz, lvl, val)
    s.build_index()  # sizes the table and the grid bound, eagerly
    cap = 4 * s.count(cs.iso)[0] + 4096
    tris = torch.zeros((cap, 9), dtype=torch.float32, device=dev)

    def step():
        s.upload(xyz, lvl, val)
        s.build_index(wait=False)
        s.isosurface_into(cs.iso, tris, cap)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    # new values, moved cells (a shift by a multiple of the coarsest width
    # keeps every corner aligned), and the original set again
    shift = np.array([1, -2, 3], np.int32) * (1 << (int(cs.level.max()) + 1))
    variants = [("values x1.04", cs.xyz, (cs.value * np.float32(1.04)).astype(np.float32)),
                ("values x0.97", cs.xyz, (cs.value * np.float32(0.97)).astype(np.float32)),
                ("cells moved", (cs.xyz + shift).astype(np.int32), cs.value),
                ("original", cs.xyz, cs.value)]
    for what, vx, vv in variants:
        xyz.copy_(torch.from_numpy(vx))
        val.copy_(torch.from_numpy(vv))
        g.replay()
        torch.cuda.synchronize()
        n = int(s.counts[0].item())
        _say("replay (%s): %d triangles" % (what, n))
        assert 0 < n <= cap
        got = tris[:n].cpu().numpy()
        # eager run of the same step on a fresh set
        e = amr.from_numpy(vx, cs.level, vv)
        want = e.isosurface(cs.iso)["tris"].cpu().numpy()
        assert len(want) == n
        assert same_positions(_as_set(got), _as_set(want))
        # the oracle
        ro = oracle.Oracle(vx, cs.level, vv, validate=False).isosurface(cs.iso)
        assert int(s.counts[1].item()) == ro["n_duals"]
        assert same_positions(_as_set(got), _as_set(ro["tris"]))
    s.build_status()  # the verdict of the last replayed build: no error


def test_failed_build_counts_minus_one(amr):
    """A duplicate cell in a re-upload of as many cells: the build is
    enqueued without waiting, extraction writes -1, amr_build_status names
    the overlap, and later extractions are refused on the host."""
    cs = amrgen.random_octree(11, roots=3, root_level=3, p_split=0.5, values="smooth")
    dev = torch.device("cuda", 0)
    s = amr.AmrSet(0)
    xyz = torch.from_numpy(cs.xyz).to(dev)
    lvl = torch.from_numpy(cs.level).to(dev)
    val = torch.from_numpy(cs.value).to(dev)
    s.upload(xyz, lvl, val)
    s.build_index()
    good = s.count(cs.iso)
    assert good[0] > 0
    bad = cs.xyz.copy()
    same = np.nonzero(cs.level == cs.level[0])[0]
    bad[same[1]] = bad[same[0]]  # two cells of one level at one corner
    xyz2 = torch.from_numpy(bad).to(dev)
    s.upload(xyz2, lvl, val)
    s.build_index(wait=False)
    tris = torch.zeros((16, 9), dtype=torch.float32, device=dev)
    counts = s.isosurface_into(cs.iso, tris, 16)
    torch.cuda.synchronize()
    assert counts.tolist() == [-1, -1]
    assert torch.all(tris == 0)
    with pytest.raises(amr.AmrError) as ei:
        s.build_status()
    assert ei.value.code == amr.AMR_EOVERLAP
    with pytest.raises(amr.AmrError) as ei:
        s.count(cs.iso)
    assert ei.value.code == amr.AMR_ESTATE
    # the good cells again: the set works as before
    s.upload(xyz, lvl, val)
    s.build_index()
    assert s.count(cs.iso) == good


@pytest.mark.parametrize("name", ["octree-shell-256", "octree-sized-647k"])
def test_captured_recording_call_never_replayed(amr, name):
    """The second extraction after a build records the group value ranges.
    Captured and never replayed, it records nothing, so the eager calls after
    it must not cull (they run full passes and give the same output); once
    the graph has run, they cull and still give the same output."""
    cs = amrgen.octree_shell() if name == "octree-shell-256" else amrgen.octree_sized(800_000, seed=9)
    _say("uncaptured ranges %s: %d cells" % (name, cs.n))
    iso = float(np.quantile(cs.value, 0.6))
    cap = 2 * amr.from_numpy(cs.xyz, cs.level, cs.value).count(iso)[0] + 1024  # on another set
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    first = torch.zeros((cap, 9), dtype=torch.float32, device=s.device)
    s.isosurface_into(iso, first, cap)  # extraction 1: no ranges yet
    torch.cuda.synchronize()
    n = int(s.counts[0].item())
    assert 0 < n <= cap
    ref = first[:n].clone()
    rec = torch.zeros((cap, 9), dtype=torch.float32, device=s.device)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.isosurface_into(iso, rec, cap)  # would record the ranges
    torch.cuda.synchronize()
    for k in range(2):
        out = torch.zeros((cap, 9), dtype=torch.float32, device=s.device)
        s.isosurface_into(iso, out, cap)  # the host asks for culling
        torch.cuda.synchronize()
        assert int(s.counts[0].item()) == n
        assert torch.equal(out[:n], ref)
    g.replay()  # now the ranges are recorded
    torch.cuda.synchronize()
    assert torch.equal(rec[:n], ref)
    for v in (iso, float(np.quantile(cs.value, 0.3))):
        out = torch.zeros((cap, 9), dtype=torch.float32, device=s.device)
        s.isosurface_into(v, out, cap)
        torch.cuda.synchronize()
        m = int(s.counts[0].item())
        assert 0 < m <= cap
        want = s.isosurface(v, cells=True, dual=True)  # a full pass (dual indices: no culling)
        assert torch.equal(out[:m], want["tris"])
