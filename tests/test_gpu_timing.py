"""Kernel timing hooks (amr_time_kernel, amr_timed_kernel_name): an armed
timing brackets the next launch of its kernel slot with the caller's events
and names the kernel that ran, as rocprofv3 names it; a slot the call does
not launch stays unnamed and its events unrecorded by the library."""
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


def _timed(amr, s, kernel, call):
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    e1.record(stream)
    s.time_kernel(kernel, e0, e1)
    call()
    torch.cuda.synchronize()
    name = s.timed_kernel_name()
    s.time_kernel(0, e0, e1)
    return name, e0.elapsed_time(e1)


def test_timed_kernel_names(amr):
    small = amrgen.two_level_sphere()
    s = amr.from_numpy(small.xyz, small.level, small.value)
    cap = s.count(small.iso)[0]
    tris = torch.empty((cap, 9), dtype=torch.float32, device=s.device)
    iso = lambda: s.isosurface_into(small.iso, tris, cap)  # noqa: E731
    # a small set extracts in one fused pass: no write pass
    assert _timed(amr, s, amr.KERNEL_EXTRACT, iso)[0] == "k_extract<false, 2>"
    assert _timed(amr, s, amr.KERNEL_WRITE, iso)[0] == ""
    name, ms = _timed(amr, s, amr.KERNEL_INSERT, lambda: s.build_index())
    assert name == "k_index_insert" and ms > 0.0
    # 175,616 groups (5,488 tiles): count pass, list of groups with
    # triangles, write pass over the list
    g = amrgen.uniform_grid(112)
    t = amr.from_numpy(g.xyz, g.level, g.value)
    cap = t.count(g.iso)[0]
    tris = torch.empty((max(cap, 1), 9), dtype=torch.float32, device=t.device)
    iso = lambda: t.isosurface_into(g.iso, tris, cap)  # noqa: E731
    assert _timed(amr, t, amr.KERNEL_EXTRACT, iso)[0] == "k_extract<false, 0>"
    assert _timed(amr, t, amr.KERNEL_WRITE, iso)[0] == "k_extract_list<1>"
