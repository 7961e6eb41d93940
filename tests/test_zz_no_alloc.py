"""The allocation-free weld (amr_indexed_mesh_noalloc) against the weld with
a caller workspace (amr_indexed_mesh), through the C ABI: two calls in a
row, the second with a smaller input, each equal to the workspace path bit
for bit (vertex count, vertices, corner indices); sizes past the scratch
are refused."""
import ctypes as C

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


def _surface(amr, cs):
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    r = s.isosurface(cs.iso, cells=True)
    return r["tris"].contiguous(), r["cells"].contiguous()


def _noalloc(amr, tris, cells):
    n = int(tris.shape[0])
    dev = tris.device
    verts = torch.full((3 * n + 1, 3), -7.0, dtype=torch.float32, device=dev)
    idx = torch.full((n + 1, 3), -7, dtype=torch.int32, device=dev)
    nv = torch.full((1,), -7, dtype=torch.int64, device=dev)
    lib = amr.load_library()
    code = lib.amr_indexed_mesh_noalloc(C.c_void_p(tris.data_ptr()), C.c_void_p(cells.data_ptr()), n,
                                        C.c_void_p(verts.data_ptr()), C.c_void_p(idx.data_ptr()), 3 * n + 1,
                                        C.c_void_p(nv.data_ptr()),
                                        C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    assert code == 0, lib.amr_last_error()
    torch.cuda.synchronize(dev)
    v = int(nv.item())
    return verts[:v], idx[:n]


def test_noalloc_weld_equals_workspace_weld(amr):
    big = _surface(amr, amrgen.octree_shell_2m())
    small = _surface(amr, amrgen.octree_shell())
    assert big[0].shape[0] > small[0].shape[0] > 0
    for tris, cells in (big, small):
        vw, iw = amr.indexed_mesh(tris, cells)
        va, ia = _noalloc(amr, tris, cells)
        assert va.shape == vw.shape
        assert torch.equal(va.view(torch.int32), vw.view(torch.int32))
        assert torch.equal(ia, iw)
        print("noalloc weld: %d triangles, %d vertices" % (tris.shape[0], va.shape[0]), flush=True)


def test_noalloc_weld_limits(amr):
    lib = amr.load_library()
    dev = torch.device("cuda", 0)
    nv = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    # past the scratch: refused before anything runs
    assert lib.amr_indexed_mesh_noalloc(None, None, (1 << 18) + 1, None, None, 0, C.c_void_p(nv.data_ptr()),
                                        stream) == amr.AMR_ERANGE
    # no triangles: zero vertices
    nv.fill_(5)
    assert lib.amr_indexed_mesh_noalloc(None, None, 0, None, None, 0, C.c_void_p(nv.data_ptr()), stream) == 0
    torch.cuda.synchronize()
    assert nv.item() == 0
