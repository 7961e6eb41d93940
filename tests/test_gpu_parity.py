"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar: dual cells bit-exact (corner, level, 8 cell indices), triangle topology
bit-exact (per-vertex cell pairs, per-dual triangle sets), triangle counts
exact, vertex positions equal bit for bit (tighter than 1e-5 of the finest
width: both sides place vertices with the same float32 operations).
"""
import os
import sys

import numpy as np
import pytest

import amrgen
import oracle

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _util import canon_by_cells, directed_edges, same_positions  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amr():
    import paper_2004_08475_amd as amr

    amr.load_library()  # raises if the library is not built: no silent fallback
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return amr


def _say(msg):
    print(msg, flush=True)


def gpu_set(amr, cs):
    return amr.from_numpy(cs.xyz, cs.level, cs.value)


def check_duals(s, o):
    pl_g, ids_g, vals_g = s.dual_cells(values=True)
    # the values written beside the duals are the cells' values
    assert np.array_equal(vals_g.cpu().numpy(), o.value[ids_g.cpu().numpy()])
    pl_o, ids_o = o.dual_cells()
    a = oracle.canonical_duals(pl_g.cpu().numpy(), ids_g.cpu().numpy())
    b = oracle.canonical_duals(pl_o, ids_o)
    assert len(a[0]) == len(b[0])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    return pl_g.cpu().numpy(), ids_g.cpu().numpy()


def check_iso(s, o, iso, pl_g=None):
    r = s.isosurface(iso, cells=True, dual=True)
    ro = o.isosurface(iso)
    tg, cg, dg = r["tris"].cpu().numpy(), r["cells"].cpu().numpy(), r["dual"].cpu().numpy()
    assert len(tg) == len(ro["tris"])
    assert r["n_duals"] == ro["n_duals"]
    A, AC, AD = canon_by_cells(tg, cg, dg)
    B, BC, BD = canon_by_cells(ro["tris"], ro["cells"], ro["dual"])
    assert np.array_equal(AC, BC)
    assert same_positions(A, B)
    if pl_g is not None and len(AD):
        # per-dual triangle sets: the generating dual of each triangle agrees
        pl_o, _ = o.dual_cells()
        kg = [tuple(pl_g[d]) for d in AD]
        ko = [tuple(pl_o[d]) for d in BD]
        assert kg == ko
    return r, A


CASES = {
    "two-level-sphere-16": lambda: amrgen.two_level_sphere(),
    "octree-shell-256": lambda: amrgen.octree_shell(),
    "random-octree-holes": lambda: amrgen.random_octree(7, roots=4, root_level=4, p_split=0.45, p_hole=0.15,
                                                        values="smooth", origin=(-64, 32, -16)),
    "random-octree-dense": lambda: amrgen.random_octree(8, roots=5, root_level=3, p_split=0.6, p_hole=0.0,
                                                        values="random", origin=(0, 0, 0)),
    "grid-33-level1": lambda: amrgen.uniform_grid(33, 1, 3, origin=(-40, 10, 6)),
    "grid-17-level0": lambda: amrgen.uniform_grid(17, 0, 4, origin=(5, -3, 100)),
    # 92,118 groups = 2,879 tiles: past the fused single-pass limit (2,048
    # tiles), so this one runs the count / scan / write passes
    "octree-sized-647k": lambda: amrgen.octree_sized(800_000, seed=9),
}


@pytest.mark.parametrize("name", list(CASES))
def test_parity(amr, name):
    cs = CASES[name]()
    _say("parity %s: %d cells" % (name, cs.n))
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    s = gpu_set(amr, cs)
    pl_g, _ = check_duals(s, o)
    check_iso(s, o, cs.iso, pl_g)
    # a second iso on the same index
    iso2 = float(np.quantile(cs.value, 0.3))
    check_iso(s, o, iso2, pl_g)


def test_two_level_closed_surface_on_gpu(amr):
    cs = amrgen.two_level_sphere()
    s = gpu_set(amr, cs)
    pl, _ = s.dual_cells()
    assert len(pl) == 947
    r = s.isosurface(cs.iso, cells=True)
    cnt = directed_edges(r["cells"].cpu().numpy())
    assert all(cnt.get((b, a), 0) == c for (a, b), c in cnt.items())


def test_deterministic_and_capacity_contract(amr):
    cs = amrgen.octree_shell()
    s = gpu_set(amr, cs)
    full = s.isosurface(cs.iso)["tris"].clone()
    again = s.isosurface(cs.iso, cap=len(full))["tris"]
    assert torch.equal(full, again)
    # too small: counts report the full number, only cap triangles written
    cap = len(full) // 3
    buf = torch.full((cap + 16, 9), -7.0, dtype=torch.float32, device=s.device)
    counts = s.isosurface_into(cs.iso, buf, cap)
    torch.cuda.synchronize()
    assert int(counts[0]) == len(full)
    assert torch.equal(buf[:cap], full[:cap])
    assert torch.all(buf[cap:] == -7.0)
    # count-only pass
    assert s.count(cs.iso)[0] == len(full)


@pytest.mark.parametrize("name", ["octree-shell-256", "octree-sized-647k"])
def test_isosurface_graph_replays(amr, name):
    # amr_isosurface does no host synchronisation, so it can be captured in a
    # HIP graph; replays with new isos (eager work in between) must equal the
    # eager calls.  octree-shell-256 runs the fused pass, the 647k set the
    # count / scan / write passes.
    cs = CASES[name]()
    _say("graph replay %s: %d cells" % (name, cs.n))
    s = gpu_set(amr, cs)
    isos = np.quantile(cs.value, [0.3, 0.5, 0.7, 0.5]).astype(np.float32)
    cap = 2 * max(s.count(float(v))[0] for v in isos) + 64
    tris = torch.zeros((cap, 9), dtype=torch.float32, device=s.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.isosurface_into(float(isos[0]), tris, cap)  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graphs = []
    for v in isos[:3]:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s.isosurface_into(float(v), tris, cap)
        graphs.append((g, float(v)))
    torch.cuda.synchronize()
    for g, v in graphs + graphs[::-1]:
        g.replay()
        torch.cuda.synchronize()
        n = int(s.counts[0].item())
        got = tris[:n].clone()
        want = s.isosurface(v)["tris"]  # eager work between the replays
        assert n == len(want)
        assert torch.equal(got, want)


def test_tri_dual_points_at_generating_dual(amr):
    cs = amrgen.random_octree(9, roots=4, root_level=3, p_split=0.5, p_hole=0.1, values="smooth")
    s = gpu_set(amr, cs)
    pl, ids = s.dual_cells()
    r = s.isosurface(cs.iso, cells=True, dual=True)
    ids = ids.cpu().numpy()
    cells = r["cells"].cpu().numpy()
    for tcell, d in zip(cells, r["dual"].cpu().numpy()):
        assert set(tcell.tolist()) <= set(ids[d].tolist())


def test_edge_cases(amr):
    # empty set
    s = amr.AmrSet()
    e = torch.empty((0, 3), dtype=torch.int32, device="cuda")
    s.upload(e, torch.empty(0, dtype=torch.int32, device="cuda"), torch.empty(0, dtype=torch.float32, device="cuda"))
    s.build_index()
    assert s.count(0.5) == (0, 0)
    assert len(s.dual_cells()[0]) == 0
    # one cell: no dual has all 8 vertices
    one = amr.from_numpy(np.array([[8, 8, 8]]), np.array([3]), np.array([1.0], np.float32))
    assert len(one.dual_cells()[0]) == 0
    # 2x2x2 level-3 cells: exactly one dual
    xyz = np.array([[x, y, z] for z in (0, 8) for y in (0, 8) for x in (0, 8)])
    eight = amr.from_numpy(xyz, np.full(8, 3), np.arange(8, dtype=np.float32))
    pl, ids = eight.dual_cells()
    assert pl.cpu().tolist() == [[8, 8, 8, 3]]
    assert ids.cpu().tolist() == [list(range(8))]
    # coordinates near the limits
    cs = amrgen.random_octree(5, roots=2, root_level=3, p_split=0.5, values="smooth", origin=(-(1 << 22), (1 << 22), 0))
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    s2 = gpu_set(amr, cs)
    check_duals(s2, o)
    check_iso(s2, o, cs.iso)


def test_sparse_set_grows_index(amr):
    """One cell per sibling block: more groups than the first table size
    allows, so the build reports ENOSPACE and the binding retries."""
    g = np.arange(0, 64, 2)
    xyz = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    val = amrgen.uniform(3, 1, np.arange(len(xyz), dtype=np.uint64)).astype(np.float32)
    s = amr.from_numpy(xyz, np.zeros(len(xyz)), val)
    assert len(s.dual_cells()[0]) == 0  # isolated cells: no dual is covered
    # now fill in the odd cells too: every dual inside is a unit cube
    g1 = np.arange(0, 16)
    xyz1 = np.stack(np.meshgrid(g1, g1, g1, indexing="ij"), -1).reshape(-1, 3)
    keep = np.any(xyz1 % 2 == 1, axis=1)
    xyz2 = np.concatenate([xyz1[~keep][::1], xyz1[keep]])
    v2 = amrgen.uniform(4, 1, np.arange(len(xyz2), dtype=np.uint64)).astype(np.float32)
    o = oracle.Oracle(xyz2, np.zeros(len(xyz2)), v2)
    s2 = amr.from_numpy(xyz2, np.zeros(len(xyz2)), v2)
    check_duals(s2, o)


def test_error_codes(amr):
    def up(xyz, lvl, val, build=True):
        # the upload's verdict is read by the build (or amr_index_bytes)
        s = amr.AmrSet()
        s.upload(torch.tensor(np.asarray(xyz), dtype=torch.int32, device="cuda").reshape(-1, 3),
                 torch.tensor(np.asarray(lvl), dtype=torch.int32, device="cuda"),
                 torch.tensor(np.asarray(val), dtype=torch.float32, device="cuda"))
        if build:
            s.build_index()
        return s

    with pytest.raises(amr.AmrError) as ei:
        up([[1, 0, 0]], [1], [0.0])
    assert ei.value.code == amr.AMR_EINVAL
    with pytest.raises(amr.AmrError) as ei:
        up([[0, 0, 0]], [21], [0.0])
    assert ei.value.code == amr.AMR_EINVAL
    with pytest.raises(amr.AmrError) as ei:
        up([[0, 0, 0]], [0], [float("nan")])
    assert ei.value.code == amr.AMR_EINVAL
    with pytest.raises(amr.AmrError) as ei:
        up([[1 << 23, 0, 0]], [0], [0.0])
    assert ei.value.code == amr.AMR_ERANGE
    with pytest.raises(amr.AmrError) as ei:
        up([[0, 0, 0], [1 << 20, 0, 0]], [0, 0], [0.0, 0.0])
    assert ei.value.code == amr.AMR_ERANGE
    with pytest.raises(amr.AmrError) as ei:
        up([[0, 0, 0], [0, 0, 0]], [0, 0], [0.0, 1.0])
    assert ei.value.code == amr.AMR_EOVERLAP
    with pytest.raises(amr.AmrError) as ei:
        up([[0, 0, 0], [2, 2, 2]], [2, 0], [0.0, 1.0])
    assert ei.value.code == amr.AMR_EOVERLAP
    # a bad upload after a good one on the same set and workspace (the build
    # does not wait for the verdict then) still reports the bad cell
    s = up([[0, 0, 0], [2, 0, 0]], [1, 1], [0.0, 1.0])
    s.upload(torch.tensor([[0, 0, 0], [3, 0, 0]], dtype=torch.int32, device="cuda"),
             torch.tensor([1, 1], dtype=torch.int32, device="cuda"),
             torch.tensor([0.0, 1.0], dtype=torch.float32, device="cuda"))
    with pytest.raises(amr.AmrError) as ei:
        s.build_index()
    assert ei.value.code == amr.AMR_EINVAL
    s = up([[0, 0, 0]], [0], [0.0], build=False)
    with pytest.raises(amr.AmrError) as ei:
        s.count(0.5)
    assert ei.value.code == amr.AMR_ESTATE
    s.build_index()
    with pytest.raises(amr.AmrError) as ei:
        s.count(float("nan"))
    assert ei.value.code == amr.AMR_EINVAL


def _owner_of_duals(pl, ids, level):
    """Generating cell of each dual under rule 3: the cell in the lowest slot
    whose level equals the dual's level."""
    lv = level[ids]
    same = lv == pl[:, 3:4]
    first = np.argmax(same, axis=1)
    return ids[np.arange(len(ids)), first]


def test_block_vortex_full_size_sampled(amr):
    """~50M-cell block-structured set with a hole, at full size: all GPU duals
    and triangles whose generating cell lies in a sample of cells equal the
    oracle's for that sample.  Samples: two contiguous ranges of 60,000 cells
    of the shuffled input (random cells anywhere), and every cell with its
    lower corner in a 24-unit slab along one edge of the obstacle box (cells
    beside the hole, on both of its faces there); the oracle gets that slab's
    cells plus every cell meeting the slab grown by 2^(Lmax+1), which holds
    every point their duals snap."""
    cs = amrgen.block_vortex(device="cuda")
    _say("block-vortex: %d cells" % cs.n)
    s = gpu_set(amr, cs)
    pl, ids = s.dual_cells()
    pl, ids = pl.cpu().numpy(), ids.cpu().numpy()
    r = s.isosurface(cs.iso, cells=True, dual=True)
    tg, cg, dg = r["tris"].cpu().numpy(), r["cells"].cpu().numpy(), r["dual"].cpu().numpy()
    _say("gpu: %d duals, %d triangles" % (len(pl), len(tg)))
    assert r["n_duals"] == len(pl) and len(tg) > 0
    owner = _owner_of_duals(pl, ids, cs.level)

    def check(sel, opl, oids, ro, back):
        a = oracle.canonical_duals(pl[sel], ids[sel])
        b = oracle.canonical_duals(opl, back[oids].astype(np.int32))
        assert len(a[0]) == len(b[0]) > 0
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        tsel = sel[dg]
        assert int(tsel.sum()) == len(ro["tris"])
        if len(ro["tris"]) == 0:
            return len(a[0]), 0
        A, AC, _ = canon_by_cells(tg[tsel], cg[tsel])
        B, BC, _ = canon_by_cells(ro["tris"], back[ro["cells"]])
        assert np.array_equal(AC, BC)
        assert same_positions(A, B)
        return len(a[0]), len(A)

    # the slab beside the hole, on its own small oracle
    (ox0, ox1), (oy0, oy1), (oz0, oz1) = cs.meta["obstacle"]
    lo = np.array([ox0 - 12, oy0 - 12, oz0 - 12])
    hi = np.array([ox0 + 12, oy0 + 12, oz1 + 12])
    in_slab = np.all((cs.xyz >= lo) & (cs.xyz < hi), axis=1)
    halo = 2 << int(cs.level.max())
    w = (1 << cs.level.astype(np.int64))[:, None]
    near = np.all((cs.xyz + w > lo - halo) & (cs.xyz < hi + halo), axis=1)
    sub = np.concatenate([np.nonzero(in_slab)[0], np.nonzero(near & ~in_slab)[0]])
    n_slab = int(in_slab.sum())
    o = oracle.Oracle(cs.xyz[sub], cs.level[sub], cs.value[sub], validate=False)
    opl, oids = o.dual_cells(0, n_slab)
    nd, nt = check(in_slab[owner], opl, oids, o.isosurface(cs.iso, 0, n_slab), sub)
    _say("slab beside the hole: %d cells, %d duals, %d triangles" % (n_slab, nd, nt))
    del o

    # the set has no overlaps by construction (and the GPU build checked);
    # the oracle's own overlap check takes minutes at this size
    o = oracle.Oracle(cs.xyz, cs.level, cs.value, validate=False)
    _say("oracle index built")
    everyone = np.arange(cs.n, dtype=np.int64)
    for c0 in (cs.n // 3, 2 * cs.n // 3):
        c1 = c0 + 60000
        opl, oids = o.dual_cells(c0, c1)
        nd, nt = check((owner >= c0) & (owner < c1), opl, oids, o.isosurface(cs.iso, c0, c1), everyone)
        _say("input range [%d, %d): %d duals, %d triangles" % (c0, c1, nd, nt))


def _sweep_case(k):
    """Seeded variety of small AMR sets: root levels 2..5, split and hole
    rates, smooth or random values, origins with negative coordinates."""
    rng = np.random.default_rng(1000 + k)
    root_level = int(rng.integers(2, 6))
    roots = int(rng.integers(2, 5))
    origin = tuple(int(v) * (1 << (root_level + 1)) for v in rng.integers(-6, 7, 3))
    return amrgen.random_octree(2000 + k, roots=roots, root_level=root_level, p_split=float(rng.uniform(0.2, 0.7)),
                                p_hole=float(rng.choice([0.0, 0.0, 0.1, 0.3])),
                                values=str(rng.choice(["smooth", "random"])), origin=origin)


@pytest.mark.parametrize("k", range(24))
def test_parity_sweep_random_octrees(amr, k):
    cs = _sweep_case(k)
    if cs.n == 0:
        pytest.skip("empty draw")
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    s = gpu_set(amr, cs)
    pl_g, _ = check_duals(s, o)
    q = float(np.random.default_rng(3000 + k).uniform(0.05, 0.95))
    check_iso(s, o, float(np.quantile(cs.value, q)), pl_g)
