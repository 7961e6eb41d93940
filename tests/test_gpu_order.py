"""The output order is a function of the cells alone.

The group list is ordered by (home slot, key): the home slot is a function
of the key and the table size, which the build takes from the cells, so
which of two colliding keys won a slot -- a race -- no longer shows.
Repeated builds of the same cells, and a build of the same cells in another
input order, must emit duals and triangles in the same order with the same
bits (cell references map through the permutation)."""
import numpy as np
import pytest

import amrgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amr():
    import paper_2004_08475_amd as amr

    amr.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return amr


CASES = {
    "octree-shell-256": amrgen.octree_shell,
    "random-octree-holes": lambda: amrgen.random_octree(7, roots=3, root_level=4, p_split=0.45, p_hole=0.15,
                                                        values="smooth", origin=(-64, 32, -16)),
    "octree-shell-256-2m": amrgen.octree_shell_2m,
}


@pytest.mark.parametrize("name", list(CASES))
def test_repeated_and_permuted_builds_emit_identical_bits(amr, name):
    cs = CASES[name]()
    perm = np.random.default_rng(3).permutation(cs.n)
    inputs = [(cs.xyz, cs.level, cs.value)] * 3 + [(cs.xyz[perm], cs.level[perm], cs.value[perm])]
    tris, cells, duals = [], [], []
    for k, (xyz, lvl, val) in enumerate(inputs):
        s = amr.from_numpy(np.ascontiguousarray(xyz), np.ascontiguousarray(lvl), np.ascontiguousarray(val))
        r = s.isosurface(float(cs.iso), cells=True)
        cl, vv = s.dual_cells()
        back = torch.from_numpy(perm).to(r["cells"].device) if k == 3 else None
        tris.append(r["tris"])
        # cell references in the original input numbering
        cells.append(back[r["cells"].long()].int() if back is not None else r["cells"])
        duals.append((cl, back[vv.long()].int() if back is not None else vv))
        s.close()
    print("%s: %d triangles, %d duals" % (name, len(tris[0]), len(duals[0][0])), flush=True)
    assert len(tris[0]) > 0
    for k in range(1, len(inputs)):
        assert torch.equal(tris[k], tris[0]), "build %d: triangle order or bits differ" % k
        assert torch.equal(cells[k], cells[0])
        assert torch.equal(duals[k][0], duals[0][0])
        assert torch.equal(duals[k][1], duals[0][1])
