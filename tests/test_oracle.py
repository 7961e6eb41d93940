"""Pins for the CPU oracle (no GPU).

Each test ties the oracle to something other than itself: closed forms of a
hand-checkable workload, brute force, the vertex-centric characterization of
the dual mesh that the paper reformulates, plain Marching Cubes on a regular
lattice, and invariants of the Marching Cubes polygonisation.
"""
import itertools
import os
from collections import Counter, defaultdict

import numpy as np
import pytest

import amrgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            parts = line.split()
            out[parts[0]] = parts[1:]
    return out


# ---------------------------------------------------------------------------
# helpers written independently of the oracle
# ---------------------------------------------------------------------------

def brute_locate(xyz, lvl, q):
    w = (1 << lvl.astype(np.int64))[:, None]
    lo = xyz.astype(np.int64)
    hit = np.all((lo <= np.asarray(q)) & (np.asarray(q) < lo + w), axis=1)
    idx = np.nonzero(hit)[0]
    assert len(idx) <= 1
    return int(idx[0]) if len(idx) else -1


def vertex_centric_duals(xyz, lvl):
    """Dual mesh by the vertex-centric characterization (sec. 2, Moran et al.):
    one dual per distinct corner P of an actual cell whose 8 octants around P
    are all covered; its vertices are the covering cells and its level the
    finest of theirs.  Octant e of P is probed at the unit cube P + (e-1)."""
    corners = set()
    for c in range(len(lvl)):
        w = 1 << int(lvl[c])
        for d in itertools.product((0, 1), repeat=3):
            corners.add(tuple(int(xyz[c, a]) + d[a] * w for a in range(3)))
    out = {}
    for P in corners:
        ids = []
        for s in range(8):
            e = (s & 1, (s >> 1) & 1, (s >> 2) & 1)
            v = brute_locate(xyz, lvl, [P[a] + e[a] - 1 for a in range(3)])
            if v < 0:
                break
            ids.append(v)
        else:
            m = min(int(lvl[v]) for v in ids)
            out[(P, m)] = tuple(ids)
    return out


def trilinear_volume(pts):
    """Volume of the trilinear map of a hexahedron (8 points in slot order),
    2-point Gauss rule per axis (exact: det J has degree <= 2 per variable)."""
    g = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    vol = 0.0
    for u, v, w in itertools.product(g, g, g):
        J = np.zeros((3, 3))
        for s in range(8):
            e = (s & 1, (s >> 1) & 1, (s >> 2) & 1)
            fu = [u if e[0] else 1 - u, v if e[1] else 1 - v, w if e[2] else 1 - w]
            for a in range(3):
                d = [fu[0], fu[1], fu[2]]
                d[a] = 1.0 if e[a] else -1.0
                J[:, a] += pts[s] * d[0] * d[1] * d[2]
        vol += np.linalg.det(J) / 8.0
    return vol


def directed_edges(cells):
    """Directed edges between welded vertices; a vertex is its cell pair."""
    cnt = Counter()
    for t in np.asarray(cells).reshape(-1, 3, 2):
        ks = [tuple(sorted(map(int, v))) for v in t]
        for i in range(3):
            cnt[(ks[i], ks[(i + 1) % 3])] += 1
    return cnt


def unbalanced(cnt):
    return {k: c - cnt.get((k[1], k[0]), 0) for k, c in cnt.items() if c != cnt.get((k[1], k[0]), 0)}


# ---------------------------------------------------------------------------
# cell location
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_sorted_locate_matches_brute(seed):
    cs = amrgen.random_octree(seed, roots=2, root_level=3, p_split=0.4, p_hole=0.15, origin=(-8, 0, 16))
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    rng = np.random.default_rng(seed)
    qs = rng.integers(-14, 36, size=(3000, 3))
    for q in qs:
        assert o.locate(q) == brute_locate(cs.xyz, cs.level, q)


def test_locate_negative_coordinates_floor():
    # a single level-2 cell at (-4,-4,-4) covers [-4,0)^3 (floor semantics)
    o = oracle.Oracle(np.array([[-4, -4, -4]]), np.array([2]), np.array([1.0], np.float32))
    assert o.locate((-1, -4, -3)) == 0
    assert o.locate((0, -1, -1)) == -1
    assert o.locate((-5, -1, -1)) == -1


# ---------------------------------------------------------------------------
# validation
# ---------------------------------------------------------------------------

def test_validation_rejects_bad_input():
    with pytest.raises(ValueError):  # misaligned level-1 corner
        oracle.Oracle(np.array([[1, 0, 0]]), np.array([1]), np.array([0.0], np.float32))
    with pytest.raises(ValueError):  # NaN value
        oracle.Oracle(np.array([[0, 0, 0]]), np.array([0]), np.array([np.nan], np.float32))
    with pytest.raises(ValueError):  # nested cells
        oracle.Oracle(np.array([[0, 0, 0], [2, 2, 2]]), np.array([2, 0]), np.zeros(2, np.float32))
    with pytest.raises(ValueError):  # duplicate
        oracle.Oracle(np.array([[0, 0, 0], [0, 0, 0]]), np.array([0, 0]), np.zeros(2, np.float32))
    for loc in ("brute", "sorted"):
        with pytest.raises(ValueError):
            oracle.Oracle(np.array([[0, 0, 0], [4, 4, 0], [6, 6, 2]]), np.array([0, 2, 0]), np.zeros(3, np.float32),
                          locator=loc)


# ---------------------------------------------------------------------------
# two-level workload: closed forms
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sphere16():
    cs = amrgen.two_level_sphere()
    return cs, oracle.Oracle(cs.xyz, cs.level, cs.value, locator="brute")


def test_two_level_closed_form(sphere16):
    cs, o = sphere16
    g = _golden("two_level_sphere_16.txt")
    assert cs.n == int(g["n_cells"][0])
    assert int((cs.level == 0).sum()) == int(g["n_level0"][0])
    pl, ids = o.dual_cells()
    assert len(pl) == int(g["duals"][0])
    assert int((pl[:, 3] == 0).sum()) == int(g["duals_level0"][0])
    assert int((pl[:, 3] == 1).sum()) == int(g["duals_level1"][0])
    distinct = np.array([len(set(r)) for r in ids])
    lv = cs.level[ids]
    unit = (pl[:, 3] == 0) & (distinct == 8) & np.all(lv == 0, axis=1)
    assert int(unit.sum()) == int(g["duals_level0_unit_cubes"][0])
    assert int(((pl[:, 3] == 0) & ~unit).sum()) == int(g["duals_level0_transition"][0])
    assert np.all(distinct[pl[:, 3] == 1] == 8) and np.all(lv[pl[:, 3] == 1] == 1)
    # no dual emitted twice
    assert len({tuple(r) for r in pl}) == len(pl)
    # the duals tile the hull of the cell centres
    ctr = cs.centres()
    vol = sum(trilinear_volume(ctr[r]) for r in ids)
    assert abs(vol - float(g["dual_volume"][0])) < 1e-6


def test_two_level_surface_closed(sphere16):
    cs, o = sphere16
    g = _golden("two_level_sphere_16.txt")
    r = o.isosurface(cs.iso)
    cnt = directed_edges(r["cells"])
    assert not unbalanced(cnt)
    # every undirected edge used by exactly two triangles
    und = Counter()
    for (a, b), c in cnt.items():
        und[frozenset((a, b))] += c
    assert set(und.values()) == {2}
    V = len({tuple(sorted(v)) for t in r["cells"].reshape(-1, 3, 2) for v in t})
    assert V - len(und) + len(r["tris"]) == int(g["euler_characteristic"][0])


def test_two_level_symmetry(sphere16):
    """The cell set and field are symmetric under the 48 symmetries of the cube
    about (8,8,8): the set of cut dual edges (as pairs of cell corners) must be
    too, and surface vertices must mirror within one fp32 ulp."""
    cs, o = sphere16
    r = o.isosurface(cs.iso)
    corner = {i: (tuple(cs.xyz[i]), int(cs.level[i])) for i in range(cs.n)}
    edges = set()
    pos = {}
    for t, cc in zip(r["tris"].reshape(-1, 3, 3), r["cells"].reshape(-1, 3, 2)):
        for v in range(3):
            k = frozenset((corner[int(cc[v, 0])], corner[int(cc[v, 1])]))
            edges.add(k)
            pos[k] = t[v].astype(np.float64)

    def img(ck, perm, flip):
        (x, l) = ck
        w = 1 << l
        lo = [x[perm[a]] for a in range(3)]
        lo = [16 - lo[a] - w if flip[a] else lo[a] for a in range(3)]
        return (tuple(lo), l)

    for perm in itertools.permutations(range(3)):
        for flip in itertools.product((0, 1), repeat=3):
            mapped = {frozenset(img(c, perm, flip) for c in k) for k in edges}
            assert mapped == edges
            for k in list(edges)[:200]:
                p = pos[k]
                q = np.array([p[perm[a]] for a in range(3)])
                q = np.where(np.array(flip) == 1, 16.0 - q, q)
                k2 = frozenset(img(c, perm, flip) for c in k)
                assert np.all(np.abs(pos[k2] - q) <= 2 * np.spacing(np.float32(16.0)))


# ---------------------------------------------------------------------------
# exactly once == vertex-centric characterization
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,p_hole,origin", [(11, 0.0, (0, 0, 0)), (12, 0.2, (-16, 8, 0)), (13, 0.1, (0, -8, -8)),
                                                (14, 0.3, (8, 8, 8)), (15, 0.0, (-8, -8, -8))])
def test_exactly_once_matches_vertex_centric(seed, p_hole, origin):
    cs = amrgen.random_octree(seed, roots=2, root_level=3, p_split=0.5, p_hole=p_hole, origin=origin)
    for loc in ("brute", "sorted"):
        o = oracle.Oracle(cs.xyz, cs.level, cs.value, locator=loc)
        pl, ids = o.dual_cells()
        got = {}
        for p, v in zip(pl, ids):
            key = (tuple(int(a) for a in p[:3]), int(p[3]))
            assert key not in got, "dual emitted twice"
            got[key] = tuple(int(a) for a in v)
        want = vertex_centric_duals(cs.xyz, cs.level)
        assert got == want


def test_exactly_once_level_jumps_of_three():
    """A level-3 cell next to level-0 cells (jump of three levels)."""
    xyz, lvl = [], []
    for x in range(0, 32, 8):
        for y in range(0, 16, 8):
            for z in range(0, 16, 8):
                if (x, y, z) == (8, 0, 0):
                    for a in range(8):
                        for b in range(8):
                            for c in range(8):
                                xyz.append((x + a, y + b, z + c))
                                lvl.append(0)
                else:
                    xyz.append((x, y, z))
                    lvl.append(3)
    xyz = np.array(xyz)
    lvl = np.array(lvl)
    o = oracle.Oracle(xyz, lvl, np.zeros(len(lvl), np.float32))
    pl, ids = o.dual_cells()
    got = {(tuple(int(a) for a in p[:3]), int(p[3])): tuple(int(a) for a in v) for p, v in zip(pl, ids)}
    assert len(got) == len(pl)
    assert got == vertex_centric_duals(xyz, lvl)


# ---------------------------------------------------------------------------
# single level == plain Marching Cubes on the cell-centre lattice
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,level,origin,seed", [(9, 0, (0, 0, 0), 1), (7, 1, (-6, 4, 10), 2), (6, 2, (-24, -24, 8), 3),
                                                 (10, 0, (-5, 3, -7), 4)])
def test_single_level_is_plain_mc(n, level, origin, seed):
    cs = amrgen.uniform_grid(n, level, seed, origin=origin)
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    pl, ids = o.dual_cells()
    assert len(pl) == (n - 1) ** 3
    r = o.isosurface(cs.iso)
    w = 1 << level
    # lattice: vals[k, j, i] of the cell at origin + (i, j, k) * w
    lat = np.zeros((n, n, n), np.float32)
    lid = np.zeros((n, n, n), np.int64)
    ijk = (cs.xyz - np.asarray(origin)) // w
    lat[ijk[:, 2], ijk[:, 1], ijk[:, 0]] = cs.value
    lid[ijk[:, 2], ijk[:, 1], ijk[:, 0]] = np.arange(cs.n)
    h0 = np.asarray(origin, np.float64) + 0.5 * w
    gt, gp = oracle.grid_mc(lat, h0, float(w), cs.iso)
    assert len(gt) == len(r["tris"]) > 0
    gcells = lid.reshape(-1)[gp]
    a, ac = oracle.canonical_triangles(r["tris"], r["cells"])
    b, bc = oracle.canonical_triangles(gt, gcells)
    assert np.array_equal(a, b)
    assert np.array_equal(ac, bc)


# ---------------------------------------------------------------------------
# Marching Cubes polygonisation
# ---------------------------------------------------------------------------

CORNER = np.array([[s & 1, (s >> 1) & 1, (s >> 2) & 1] for s in range(8)], np.float64)
EDGES = [(s, s | (1 << a)) for a in range(3) for s in range(8) if not (s >> a) & 1]
MID = np.array([(CORNER[a] + CORNER[b]) / 2 for a, b in EDGES])


def _components(case, positive):
    """Components of the corners of one sign: cube edges connect; a face
    diagonal connects two corners < iso exactly when their face is ambiguous."""
    parent = list(range(8))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    sgn = [(case >> s) & 1 for s in range(8)]
    mine = [s for s in range(8) if sgn[s] == positive]
    for a, b in EDGES:
        if sgn[a] == positive and sgn[b] == positive:
            parent[find(a)] = find(b)
    if not positive:
        for axis in range(3):
            for side in (0, 1):
                f = [s for s in range(8) if ((s >> axis) & 1) == side]
                for a, b in itertools.combinations(f, 2):
                    if bin(a ^ b).count("1") == 2:
                        others = [s for s in f if s not in (a, b)]
                        if sgn[a] == sgn[b] == 0 and sgn[others[0]] == sgn[others[1]] == 1:
                            parent[find(a)] = find(b)
    return len({find(s) for s in mine})


def _segments(tris):
    cnt = Counter()
    for t in tris:
        for i in range(3):
            cnt[(int(t[i]), int(t[(i + 1) % 3]))] += 1
    segs = set()
    for (a, b), c in cnt.items():
        d = c - cnt.get((b, a), 0)
        assert d in (0, 1, -1)
        if d == 1:
            segs.add((a, b))
    return segs


def test_polygonize_counts_and_cut_edges():
    g = _golden("mc_case_counts.txt")
    maxt = 0
    for case in range(256):
        tris = oracle.polygonize(case)
        maxt = max(maxt, len(tris))
        sgn = [(case >> s) & 1 for s in range(8)]
        cut = {k for k, (a, b) in enumerate(EDGES) if sgn[a] != sgn[b]}
        assert {int(e) for e in tris.reshape(-1)} == cut
        if case in (0, 255):
            assert len(tris) == 0
            continue
        loops = _components(case, 1) + _components(case, 0) - 1
        assert len(tris) == len(cut) - 2 * loops, case
    assert maxt == int(g["max_per_case"][1])
    for name, vals in g.items():
        if name == "max_per_case":
            continue
        case = sum(1 << int(s) for s in vals[0].split(","))
        assert len(oracle.polygonize(case)) == int(vals[1]), name


def test_polygonize_face_segments_cut_off_positive_runs():
    """The boundary of each case's triangle fan consists of segments lying on
    cube faces; looking at a face from outside, each segment has corners >= iso
    on its left and only those, and every face carries one segment per run of
    corners >= iso."""
    for case in range(1, 255):
        segs = _segments(oracle.polygonize(case))
        sgn = [(case >> s) & 1 for s in range(8)]
        per_face = Counter()
        for a, b in segs:
            ca, cb = set(EDGES[a]), set(EDGES[b])
            faces = [(ax, sd) for ax in range(3) for sd in (0, 1)
                     if all(((s >> ax) & 1) == sd for s in ca | cb)]
            assert len(faces) == 1, (case, a, b)
            ax, sd = faces[0]
            per_face[faces[0]] += 1
            n = np.zeros(3)
            n[ax] = 1.0 if sd else -1.0
            d = MID[b] - MID[a]
            left = []
            for s in range(8):
                if ((s >> ax) & 1) != sd:
                    continue
                side = np.dot(np.cross(d, CORNER[s] - MID[a]), n)
                if side > 1e-12:
                    left.append(s)
            assert left and all(sgn[s] for s in left), (case, a, b, left)
        for ax in range(3):
            for sd in (0, 1):
                cyc = [s for s in range(8) if ((s >> ax) & 1) == sd]
                # order the face cycle geometrically
                u, v = (ax + 1) % 3, (ax + 2) % 3
                cyc.sort(key=lambda s: np.arctan2(CORNER[s][v] - 0.5, CORNER[s][u] - 0.5))
                p = [sgn[s] for s in cyc]
                runs = sum(1 for i in range(4) if p[i] and not p[i - 1])
                if all(p):
                    runs = 0
                assert per_face[(ax, sd)] == runs, (case, ax, sd)


def test_polygonize_symmetric_under_cube_group():
    """The face rule is invariant under the 48 symmetries of the cube, so the
    boundary segments of case g(c) are the images of those of c (reversed for
    reflections)."""
    segs = {c: _segments(oracle.polygonize(c)) for c in range(256)}
    eidx = {frozenset(e): k for k, e in enumerate(EDGES)}
    for perm in itertools.permutations(range(3)):
        for flip in itertools.product((0, 1), repeat=3):
            det = np.linalg.det(np.eye(3)[list(perm)]) * np.prod([-1 if f else 1 for f in flip])

            def gs(s):
                c = [CORNER[s][perm[a]] for a in range(3)]
                c = [1 - c[a] if flip[a] else c[a] for a in range(3)]
                return int(c[0]) + 2 * int(c[1]) + 4 * int(c[2])

            def ge(k):
                a, b = EDGES[k]
                return eidx[frozenset((gs(a), gs(b)))]

            for c in range(256):
                gc = sum(1 << gs(s) for s in range(8) if (c >> s) & 1)
                img = {(ge(a), ge(b)) if det > 0 else (ge(b), ge(a)) for a, b in segs[c]}
                assert img == segs[gc], (perm, flip, c)


# ---------------------------------------------------------------------------
# crack-freeness on sets with holes and level jumps
# ---------------------------------------------------------------------------

def _dual_faces(ids):
    """Faces of each dual as (axis, cells at face slots (0,0),(1,0),(0,1),(1,1))."""
    faces = Counter()
    per_dual = []
    for v in ids:
        fl = []
        for ax in range(3):
            u, w = (ax + 1) % 3, (ax + 2) % 3
            for sd in (0, 1):
                sl = [(sd << ax) | (i << u) | (j << w) for j in (0, 1) for i in (0, 1)]
                key = (ax, tuple(int(v[s]) for s in sl))
                faces[key] += 1
                fl.append((key, set(sl)))
        per_dual.append(fl)
    return faces, per_dual


@pytest.mark.parametrize("seed,p_hole", [(21, 0.0), (22, 0.15), (23, 0.3), (24, 0.1)])
def test_crack_free_open_surfaces(seed, p_hole):
    cs = amrgen.random_octree(seed, roots=3, root_level=3, p_split=0.45, p_hole=p_hole, values="smooth")
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    pl, ids = o.dual_cells()
    r = o.isosurface(cs.iso)
    assert r["n_duals"] == len(pl)
    assert len(r["tris"]) > 0
    faces, per_dual = _dual_faces(ids)
    # faces with area (three or four distinct cells) are shared by at most 2 duals
    assert max(c for k, c in faces.items() if len(set(k[1])) >= 3) <= 2
    ub = unbalanced(directed_edges(r["cells"]))
    # Every unbalanced edge lies on a boundary face of the dual mesh (a face with
    # area that only one dual has): both of its welded vertices are edges of that
    # face's corner cycle.  (A zero-volume sliver dual can pass a segment from one
    # of its faces to the opposite one, so the face is not always the generating
    # dual's own.)
    boundary_edges = set()
    for (ax, cells4), c in faces.items():
        if c == 1 and len(set(cells4)) >= 3:
            cyc = [cells4[0], cells4[1], cells4[3], cells4[2]]
            fe = {tuple(sorted((cyc[i], cyc[(i + 1) % 4]))) for i in range(4)}
            for e1 in fe:
                for e2 in fe:
                    boundary_edges.add((e1, e2))
    assert ub, "an open surface must have a boundary"
    for e in ub:
        assert e in boundary_edges, e


def test_permutation_and_translation_invariance():
    cs = amrgen.random_octree(31, roots=2, root_level=3, p_split=0.5, p_hole=0.1, values="smooth")
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    a = oracle.canonical_triangles(o.isosurface(cs.iso)["tris"])[0]
    perm = np.random.default_rng(0).permutation(cs.n)
    o2 = oracle.Oracle(cs.xyz[perm], cs.level[perm], cs.value[perm])
    b = oracle.canonical_triangles(o2.isosurface(cs.iso)["tris"])[0]
    assert np.array_equal(a, b)
    shift = np.array([-64, 32, 128])
    o3 = oracle.Oracle(cs.xyz + shift, cs.level, cs.value)
    c = oracle.canonical_triangles(o3.isosurface(cs.iso)["tris"])[0]
    assert np.allclose(c - np.tile(shift, 3), a, atol=1e-4)


def test_vertex_placement_within_fp32_bound():
    cs = amrgen.random_octree(41, roots=3, root_level=3, p_split=0.45, p_hole=0.1, values="smooth")
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    r = o.isosurface(cs.iso)
    ctr = cs.centres()
    v = cs.value.astype(np.float64)
    A = r["cells"].reshape(-1, 3, 2)[:, :, 0].reshape(-1)
    B = r["cells"].reshape(-1, 3, 2)[:, :, 1].reshape(-1)
    assert np.all(v[A] < cs.iso) and np.all(v[B] >= cs.iso)
    t = (cs.iso - v[A]) / (v[B] - v[A])
    exact = ctr[A] + t[:, None] * (ctr[B] - ctr[A])
    got = r["tris"].reshape(-1, 3).astype(np.float64)
    eps = 2.0 ** -24
    bound = 4 * eps * np.abs(ctr[B] - ctr[A]) + 2 * eps * np.abs(exact) + 1e-30
    assert np.all(np.abs(got - exact) <= bound)


def test_indexed_mesh_reproduces_fat_triangles_and_counts_vertices(sphere16):
    cs, o = sphere16
    r = o.isosurface(cs.iso)
    verts, idx = oracle.indexed_mesh(r["tris"], r["cells"])
    # every fat triangle is recovered exactly from the indexed one
    assert np.array_equal(verts[idx].reshape(-1, 9), r["tris"])
    # one vertex per distinct cut edge; closed genus-0 surface: V - E + F = 2
    keys = {tuple(v) for v in r["cells"].reshape(-1, 2)}
    assert len(verts) == len(keys)
    edges = {frozenset((int(a), int(b))) for tri in idx for a, b in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0]))}
    assert len(verts) - len(edges) + len(idx) == 2
    # numbering by first appearance
    seen = []
    for v in idx.reshape(-1):
        if v not in seen:
            seen.append(v)
    assert seen == list(range(len(verts)))


# ---------------------------------------------------------------------------
# Dual-mesh interpolant (oracle.dual_mesh_sample): each dual as a trilinear
# hexahedron over its cells' centres carrying the trilinear interpolant of
# their values.  Pinned to textbook trilinear interpolation, to exact
# reproduction of linear fields, to the cells' own values at their centres,
# and to a partition of the covered volume where level jumps are small.
# ---------------------------------------------------------------------------

def _centres(cs):
    return cs.xyz.astype(np.float64) + 0.5 * (1 << cs.level.astype(np.int64))[:, None]


def _duals(cs):
    """(pl, ids) of the oracle's dual cells."""
    return oracle.Oracle(cs.xyz, cs.level, cs.value).dual_cells()


def test_dual_interpolant_is_trilinear_on_single_level_grids():
    for level in (0, 1):
        cs = amrgen.uniform_grid(6, level, 7, origin=(-8, 4, 12))
        w = 1 << level
        c = _centres(cs)
        c0 = c.min(0)
        lattice = np.full((6, 6, 6), np.nan)
        ijk = np.rint((c - c0) / w).astype(int)
        lattice[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = cs.value
        rng = np.random.default_rng(11 + level)
        pts = c0 + rng.uniform(0, 5 * w, (150, 3))
        got, _, hits = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, *_duals(cs), pts)
        assert np.all(hits == 1)
        # textbook trilinear interpolation on the cell-centre lattice
        g = (pts - c0) / w
        i0 = np.minimum(np.floor(g).astype(int), 4)
        f = g - i0
        want = np.zeros(len(pts))
        for dx, dy, dz in itertools.product((0, 1), repeat=3):
            wt = (f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) * (f[:, 2] if dz else 1 - f[:, 2])
            want += wt * lattice[i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz]
        assert np.max(np.abs(got - want)) < 1e-12


def test_dual_interpolant_reproduces_linear_fields():
    a, b = np.array([0.3, -1.2, 0.7]), 2.5
    rng = np.random.default_rng(5)
    sets = [amrgen.two_level_sphere(),
            amrgen.random_octree(50, roots=2, root_level=3, p_split=0.5, values="smooth"),
            amrgen.random_octree(51, roots=3, root_level=3, p_split=0.45, p_hole=0.1, values="smooth")]
    for cs in sets:
        lin = _centres(cs) @ a + b
        ext = cs.xyz.max(0) + (1 << cs.level.max())
        pts = rng.uniform(cs.xyz.min(0), ext, (300, 3))
        got, _, hits = oracle.dual_mesh_sample(cs.xyz, cs.level, lin, *_duals(cs), pts)
        inside = hits > 0
        assert inside.sum() > 15
        assert np.all(np.isnan(got[~inside]))
        assert np.max(np.abs(got[inside] - (pts[inside] @ a + b))) < 1e-9


def test_dual_interpolant_gives_cell_values_at_centres():
    cs = amrgen.random_octree(52, roots=2, root_level=3, p_split=0.5, values="random")
    c = _centres(cs)
    got, _, hits = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, *_duals(cs), c)
    inside = hits > 0
    assert inside.sum() > 20
    # at a collapsed vertex of a degenerate dual the inverse map is ill
    # conditioned: a 1e-9 position residual moves the value by up to ~1e-7
    assert np.max(np.abs(got[inside] - cs.value[inside].astype(np.float64))) < 1e-6


def test_dual_mesh_partitions_the_two_level_sphere():
    # the dual volumes sum to 14^3 over [1,15]^3 (pinned above); each point
    # inside lies in exactly one dual, each point outside in none
    cs = amrgen.two_level_sphere()
    pl, ids = _duals(cs)
    rng = np.random.default_rng(9)
    inside = rng.uniform(1.0, 15.0, (300, 3))
    _, _, hits = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, pl, ids, inside)
    assert np.all(hits == 1)
    outside = rng.uniform(0.0, 16.0, (400, 3))
    outside = outside[np.any((outside < 1.0) | (outside > 15.0), 1)]
    _, _, hits = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, pl, ids, outside)
    assert np.all(hits == 0)


def test_dual_hexahedra_overlap_under_large_level_jumps():
    # Level-0 cells beside level-4 cells: two duals around the corner
    # (16, 16, 16) both reach this point, with interpolants 1.3% apart, so the
    # dual mesh is no partition there and an interpolant over it needs a rule
    # for overlaps.
    cs = amrgen.random_octree(52, roots=2, root_level=4, p_split=0.6, values="smooth")
    p = np.array([[15.68839305, 13.50619197, 16.97884438]])
    pl, ids = _duals(cs)
    v, which, hits = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, pl, ids, p)
    assert hits[0] == 2
    # each of the two alone: the overlap rule picks the finer dual's value
    alone = []
    for d in range(len(ids)):
        lo = np.min(_centres(cs)[ids[d]], 0)
        hi = np.max(_centres(cs)[ids[d]], 0)
        if np.all(lo <= p[0]) and np.all(p[0] <= hi):
            vd, _, hd = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, pl[d:d + 1], ids[d:d + 1], p)
            if hd[0]:
                key = (int(pl[d, 3]), int(pl[d, 2]), int(pl[d, 1]), int(pl[d, 0]))
                alone.append((key, float(vd[0]), d))
    # two level-0 duals whose cells span levels 0..4 (the rule's tie-break
    # by centre vertex decides), interpolants 1.3% apart
    assert len(alone) == 2 and alone[0][0][0] == alone[1][0][0] == 0
    first = min(alone)
    assert which[0] == first[2] and v[0] == first[1]
    assert abs(alone[0][1] - alone[1][1]) > 1e-2 * abs(first[1])


def test_dual_interpolant_on_shared_faces_of_a_grid():
    # points on the faces, edges and vertices shared by the duals of a
    # single-level grid are reached by 2, 4 or 8 duals, whose interpolants
    # agree there: the value is the textbook trilinear one whichever wins
    cs = amrgen.uniform_grid(5, 0, 3, origin=(2, -3, 7))
    c = _centres(cs)
    c0 = c.min(0)
    lattice = np.full((5, 5, 5), np.nan)
    ijk = np.rint(c - c0).astype(int)
    lattice[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = cs.value
    rng = np.random.default_rng(4)
    g = rng.uniform(0, 4, (120, 3))
    k = np.arange(len(g))
    on = rng.integers(1, 4, (len(g), 3)).astype(float)
    g[k % 3 == 0, 0] = on[k % 3 == 0, 0]                 # faces
    g[k % 3 == 1, :2] = on[k % 3 == 1, :2]               # edges
    g[k % 3 == 2] = on[k % 3 == 2]                       # vertices
    got, _, hits = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, *_duals(cs), c0 + g)
    assert np.all(hits[k % 3 == 0] == 2) and np.all(hits[k % 3 == 1] == 4) and np.all(hits[k % 3 == 2] == 8)
    i0 = np.minimum(np.floor(g).astype(int), 3)
    f = g - i0
    want = np.zeros(len(g))
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        wt = (f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) * (f[:, 2] if dz else 1 - f[:, 2])
        want += wt * lattice[i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz]
    assert np.max(np.abs(got - want)) < 1e-12
