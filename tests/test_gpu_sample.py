"""GPU parity of the dual-mesh interpolant (amr_sampler_build / amr_sample)
against the oracle's brute-force sampler (oracle.dual_mesh_sample: every
dual of the set is a candidate, fp64 Newton, the smallest (level, P.z, P.y,
P.x) among the duals reaching a point wins).

Bar, per point: NaN on both sides or neither; the winning dual is the same
(compared by its centre vertex P and level, since the two sides number
their duals differently); the value agrees to one float32 unit in the last
place.  Both sides evaluate the same interpolant in float64 (the GPU solves
the Newton steps by Cramer's rule, the oracle by LU, which moves the result
by about 1e-15 relative) and the GPU rounds it to float32 once, so the only
difference left is that rounding.

The oracle gets all duals of small sets.  On large sets it gets, per point,
the duals whose centre vertex P lies within 2^(Lmax+1) of the point on every
axis: a dual's vertex cells contain points within 2^l <= 2^Lmax of P, so
their centres (and the whole hexahedron, their convex hull contains the
trilinear image of the unit cube) lie within 1.5 * 2^Lmax of P per axis, and
no other dual can reach the point.
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


def _points(cs, k, seed, pad=1.0):
    """k seeded uniform points over the set's bounding box grown by pad."""
    w = (1 << cs.level.astype(np.int64))[:, None]
    lo = cs.xyz.min(0) - pad
    hi = (cs.xyz + w).max(0) + pad
    return np.random.default_rng(seed).uniform(lo, hi, (k, 3)).astype(np.float32)


def _gpu_sample(amr, s, pts):
    smp = amr.DualSampler(s)
    v, d = smp.sample(torch.from_numpy(pts))
    torch.cuda.synchronize()
    return v.cpu().numpy(), d.cpu().numpy(), smp.corner_level.cpu().numpy()


def _compare(vals_g, dual_g, pl_g, vals_o, which_o, pl_o):
    nan_g, nan_o = np.isnan(vals_g), np.isnan(vals_o)
    assert np.array_equal(nan_g, nan_o), "points covered differently: %d vs %d" % (int((~nan_g).sum()),
                                                                                   int((~nan_o).sum()))
    assert np.array_equal(dual_g < 0, which_o < 0)
    hit = ~nan_o
    assert np.array_equal(pl_g[dual_g[hit]], pl_o[which_o[hit]]), "a different dual wins"
    ref = vals_o[hit]
    tol = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    err = np.abs(vals_g[hit].astype(np.float64) - ref)
    assert np.all(err <= tol), "max error %g (ulp there %g)" % (err.max(), tol[np.argmax(err - tol)])
    return int(hit.sum())


def _oracle_all(cs, pts):
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    pl, ids = o.dual_cells()
    vals, which, _ = oracle.dual_mesh_sample(cs.xyz, cs.level, cs.value, pl, ids, pts.astype(np.float64))
    return vals, which, pl


CASES = {
    "two-level-sphere-16": lambda: amrgen.two_level_sphere(),
    "random-octree-holes": lambda: amrgen.random_octree(7, roots=3, root_level=4, p_split=0.45, p_hole=0.15,
                                                        values="smooth", origin=(-64, 32, -16)),
    "random-octree-deep": lambda: amrgen.random_octree(104, roots=2, root_level=5, p_split=0.4, p_hole=0.0),
    "random-octree-deep-holes": lambda: amrgen.random_octree(111, roots=2, root_level=5, p_split=0.46,
                                                             p_hole=0.15),
    "grid-9-level1": lambda: amrgen.uniform_grid(9, level=1, origin=(-6, 10, 2)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sampler_matches_oracle(amr, name):
    cs = CASES[name]()
    pts = _points(cs, 800, 11)
    # the cells' own centres too: every dual around a centre reaches it, the
    # tie goes to the smallest key, and the value there is the cell's
    ctr = (cs.xyz + 0.5 * (1 << cs.level.astype(np.int64))[:, None]).astype(np.float32)
    pts = np.concatenate([pts, ctr[np.random.default_rng(12).permutation(len(ctr))[:200]]])
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    vals_g, dual_g, pl_g = _gpu_sample(amr, s, pts)
    vals_o, which_o, pl_o = _oracle_all(cs, pts)
    n = _compare(vals_g, dual_g, pl_g, vals_o, which_o, pl_o)
    _say("%s: %d of %d points inside the dual mesh" % (name, n, len(pts)))
    assert n > len(pts) // 4


def test_sampler_edge_cases(amr):
    cs = amrgen.two_level_sphere()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    smp = amr.DualSampler(s)
    # no points
    v, d = smp.sample(torch.zeros((0, 3)))
    assert v.numel() == 0
    # outside the coordinate limits, NaN coordinates, far away: NaN, no dual
    far = torch.tensor([[1e9, 0, 0], [float("nan"), 4, 4], [-4e6, 8, 8], [8, 8, 1e7]], dtype=torch.float32)
    v, d = smp.sample(far)
    torch.cuda.synchronize()
    assert torch.isnan(v).all() and (d == -1).all()
    # a rebuild invalidates the sampler
    s.build_index()
    with pytest.raises(amr.AmrError):
        smp.sample(far)
    # an empty set samples nothing
    e = amr.from_numpy(np.zeros((0, 3), np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    v, d = amr.DualSampler(e).sample(far)
    torch.cuda.synchronize()
    assert torch.isnan(v).all() and (d == -1).all()


def _oracle_local(xyz, lvl, val, pl, ids, pts, lmax):
    """oracle.dual_mesh_sample per point over the duals whose P lies within
    2^(lmax+1) of it (see the module docstring)."""
    reach = float(2 << lmax)
    P = pl[:, :3].astype(np.float64)
    vals = np.full(len(pts), np.nan)
    which = np.full(len(pts), -1, np.int64)
    for q, p in enumerate(pts.astype(np.float64)):
        near = np.nonzero(np.all(np.abs(P - p) <= reach, 1))[0]
        if len(near) == 0:
            continue
        v, w, _ = oracle.dual_mesh_sample(xyz, lvl, val, pl[near], ids[near], p[None])
        vals[q] = v[0]
        which[q] = near[w[0]] if w[0] >= 0 else -1
    return vals, which


def test_sampler_two_million_cell_octree_sampled(amr):
    """The ~2M-cell octree at full size: 300 points, the oracle's duals of the
    whole set."""
    cs = amrgen.octree_shell_2m()
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    pts = _points(cs, 300, 21, pad=0.0)
    vals_g, dual_g, pl_g = _gpu_sample(amr, s, pts)
    o = oracle.Oracle(cs.xyz, cs.level, cs.value, validate=False)
    pl, ids = o.dual_cells()
    _say("octree 2M: %d cells, %d duals" % (cs.n, len(pl)))
    vals_o, which_o = _oracle_local(cs.xyz, cs.level, cs.value, pl, ids, pts, int(cs.level.max()))
    n = _compare(vals_g, dual_g, pl_g, vals_o, which_o, pl)
    assert n > 200


def test_sampler_block_vortex_sampled(amr):
    """The 50.8M-cell block-structured set with a hole at full size: points
    in two boxes (one across a corner of the obstacle, one around a surface
    point among refined bricks); the oracle gets the cells meeting each box
    grown by 2^(Lmax+3) (every cell a reaching dual depends on)."""
    dev = torch.device("cuda", 0)
    cs = amrgen.block_vortex(device="cuda")
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    r = s.isosurface(cs.iso)
    v0 = r["tris"][:, :3].double()
    target = torch.tensor([300.0, 500.0, 500.0], dtype=torch.float64, device=dev)
    near_v = v0[torch.argmin(((v0 - target) ** 2).sum(1))].cpu().numpy()
    del r, v0
    (ox0, _), (oy0, _), (oz0, _) = cs.meta["obstacle"]
    boxes = [np.array([ox0, oy0, oz0], np.float64), np.floor(near_v)]
    smp = amr.DualSampler(s)
    lmax = int(cs.level.max())
    halo = 8 << lmax
    w = (1 << cs.level.astype(np.int64))[:, None]
    for bi, c in enumerate(boxes):
        lo, hi = c - 20.0, c + 20.0
        pts = np.random.default_rng(31 + bi).uniform(lo, hi, (250, 3)).astype(np.float32)
        v, d = smp.sample(torch.from_numpy(pts))
        torch.cuda.synchronize()
        vals_g, dual_g = v.cpu().numpy(), d.cpu().numpy()
        pl_g = smp.corner_level[torch.from_numpy(np.maximum(dual_g, 0)).to(dev)].cpu().numpy()
        sub = np.nonzero(np.all((cs.xyz + w > lo - halo) & (cs.xyz < hi + halo), 1))[0]
        o = oracle.Oracle(cs.xyz[sub], cs.level[sub], cs.value[sub], validate=False)
        pl, ids = o.dual_cells()
        _say("block-vortex box %d at %s: oracle on %d cells, %d duals" % (bi, c.tolist(), len(sub), len(pl)))
        vals_o, which_o = _oracle_local(cs.xyz[sub], cs.level[sub], cs.value[sub], pl, ids, pts, lmax)
        nan_g, nan_o = np.isnan(vals_g), np.isnan(vals_o)
        assert np.array_equal(nan_g, nan_o)
        hit = ~nan_o
        assert np.array_equal(pl_g[hit], pl[which_o[hit]])
        ref = vals_o[hit]
        tol = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(vals_g[hit].astype(np.float64) - ref) <= tol)
        _say("box %d: %d of %d points inside the dual mesh" % (bi, int(hit.sum()), len(pts)))
        assert hit.sum() > 50
