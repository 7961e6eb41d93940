"""Indexed face set on the GPU (the weld of fat triangles, paper sec. 5.2)
against the oracle's weld of the oracle's own triangles.

Bar: vertex count exact; connectivity exact as triples of edge cell pairs;
vertex positions within the iso-surface position tolerance; and on the GPU
output alone: every corner expands back to its fat-triangle position bit for
bit, corner key <-> vertex index is a bijection, vertices are numbered in
order of first appearance.
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return amr


def _keys(cells):
    c = np.asarray(cells, np.int64).reshape(-1, 2)
    return (c[:, 0] << 32) | c[:, 1]


def check_valid(tris, cells, verts, idx):
    """Properties that hold for any correct weld of this triangle list."""
    t = np.asarray(tris, np.float32).reshape(-1, 3)
    f = np.asarray(idx).reshape(-1)
    v = np.asarray(verts, np.float32)
    nv = len(v)
    # every corner expands back to its own position, bit for bit
    assert np.array_equal(v[f].view(np.uint32), t.view(np.uint32))
    # one vertex per distinct edge cell pair
    k = _keys(cells)
    assert len(np.unique(k)) == nv
    assert len(np.unique(np.stack([k, f.astype(np.int64)], 1), axis=0)) == nv
    # numbered by first appearance
    u, first = np.unique(f, return_index=True)
    assert np.array_equal(u, np.arange(nv))
    assert np.all(np.diff(first) > 0)


def check_against_oracle(tris_g, cells_g, verts_g, idx_g, ro):
    ov, oi = oracle.indexed_mesh(ro["tris"], ro["cells"])
    assert len(verts_g) == len(ov)
    kg = _keys(cells_g)
    ko = _keys(ro["cells"])
    # vertex key tables (first corner of each vertex)
    vk_g = np.empty(len(verts_g), np.int64)
    vk_g[np.asarray(idx_g).reshape(-1)] = kg
    vk_o = np.empty(len(ov), np.int64)
    vk_o[oi.reshape(-1)] = ko
    # connectivity as key triples, each rotated to start at its smallest key
    def triples(vk, ix):
        tk = vk[np.asarray(ix).reshape(-1, 3)]
        r = np.argmin(tk, axis=1)
        tk = np.take_along_axis(tk, (r[:, None] + np.arange(3)[None]) % 3, 1)
        return tk[np.lexsort((tk[:, 2], tk[:, 1], tk[:, 0]))]
    assert np.array_equal(triples(vk_g, idx_g), triples(vk_o, oi))
    # positions of the same vertex agree
    og = np.argsort(vk_g)
    oo = np.argsort(vk_o)
    assert np.array_equal(vk_g[og], vk_o[oo])
    assert same_positions(np.asarray(verts_g)[og], ov[oo])


CASES = {
    "two-level-sphere-16": lambda: amrgen.two_level_sphere(),
    "octree-shell-256": lambda: amrgen.octree_shell(),
    "random-octree-holes": lambda: amrgen.random_octree(7, roots=4, root_level=4, p_split=0.45, p_hole=0.15,
                                                        values="smooth", origin=(-64, 32, -16)),
    "random-octree-values": lambda: amrgen.random_octree(8, roots=5, root_level=3, p_split=0.6, p_hole=0.0,
                                                         values="random", origin=(0, 0, 0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_indexed_mesh_matches_oracle(amr, name):
    cs = CASES[name]()
    print("indexed mesh %s: %d cells, iso %r" % (name, cs.n, cs.iso), flush=True)
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    r = s.isosurface(cs.iso, cells=True)
    verts, idx = amr.indexed_mesh(r["tris"], r["cells"])
    tg, cg = r["tris"].cpu().numpy(), r["cells"].cpu().numpy()
    vg, ig = verts.cpu().numpy(), idx.cpu().numpy()
    check_valid(tg, cg, vg, ig)
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    check_against_oracle(tg, cg, vg, ig, o.isosurface(cs.iso))


def test_indexed_mesh_many_tiles_properties(amr):
    # ~1.5M cells, ~220k corners: dozens of scan tiles and a ragged last tile
    cs = amrgen.octree_sized(2_000_000, seed=11)
    print("indexed mesh octree-sized: %d cells" % cs.n, flush=True)
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    r = s.isosurface(cs.iso, cells=True)
    n = int(r["tris"].shape[0])
    assert 3 * n > 4096 * 40 and (3 * n) % 4096 != 0
    verts, idx = amr.indexed_mesh(r["tris"], r["cells"])
    check_valid(r["tris"].cpu().numpy(), r["cells"].cpu().numpy(), verts.cpu().numpy(), idx.cpu().numpy())
    # same input twice: same output (first-appearance numbering is deterministic)
    v2, i2 = amr.indexed_mesh(r["tris"], r["cells"])
    assert torch.equal(idx, i2) and torch.equal(verts, v2)


def test_indexed_mesh_empty_and_capacity(amr):
    dev = torch.device("cuda", 0)
    tris = torch.empty((0, 9), dtype=torch.float32, device=dev)
    cells = torch.empty((0, 6), dtype=torch.int32, device=dev)
    v, i = amr.indexed_mesh(tris, cells)
    assert v.shape[0] == 0 and i.shape[0] == 0
    cs = amrgen.octree_shell()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    r = s.isosurface(cs.iso, cells=True)
    full_v, full_i = amr.indexed_mesh(r["tris"], r["cells"])
    cap = len(full_v) // 3
    n = int(r["tris"].shape[0])
    verts = torch.full((cap + 4, 3), -7.0, dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
    nv = torch.zeros(1, dtype=torch.int64, device=dev)
    # verts past cap are not written, the count and every index still are
    lib = amr.load_library()
    b = amr.C.c_size_t(0)
    amr._check(lib.amr_indexed_mesh_bytes(n, amr.C.byref(b)))
    ws = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
    amr._check(lib.amr_indexed_mesh(amr._ptr(r["tris"]), amr._ptr(r["cells"]), n, amr._ptr(verts), amr._ptr(idx),
                                    cap, amr._ptr(nv), amr._ptr(ws), ws.numel(), amr._stream(dev)))
    torch.cuda.synchronize()
    assert int(nv.item()) == len(full_v)
    assert torch.equal(idx, full_i)
    assert torch.equal(verts[:cap], full_v[:cap])
    assert torch.all(verts[cap:] == -7.0)
    # too small a workspace is an error, not a fault
    with pytest.raises(amr.AmrError):
        amr._check(lib.amr_indexed_mesh(amr._ptr(r["tris"]), amr._ptr(r["cells"]), n, amr._ptr(verts),
                                        amr._ptr(idx), cap, amr._ptr(nv), amr._ptr(ws), 1024, amr._stream(dev)))
