"""Parity on the resident serving set at full size: octree-shell-2048, 608.9M
cells on levels 0..5.  The GPU runs the whole set; the duals and triangles
owned by a spatially compact sample of at least 1M cells must equal the
oracle's for those cells.

The oracle only gets the sample plus a halo: every point a cell snaps lies
within one of its own widths (at most 2^Lmax) of the cell, so the cells
meeting the sample box grown by 2^(Lmax+1) contain every point the sample's
duals and triangles depend on, and the oracle's index stays small.

Bar: dual cells bit-exact (corner, level, 8 global cell indices); triangle
topology exact (per-vertex cell pairs); positions equal bit for bit.  A serving mix against the same resident
set must give each request's result as it is alone.
"""
import os
import sys

import numpy as np
import pytest

import amrgen
import oracle

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _util import canon_by_cells, same_positions  # noqa: E402

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


def _owned(pl, ids, level, sample_mask, chunk=1 << 26):
    """Per dual: is its generating cell (under rule 3, the cell in the lowest
    slot whose level equals the dual's) in the sample?  On the device, in
    chunks."""
    out = torch.empty(pl.shape[0], dtype=torch.bool, device=pl.device)
    for a in range(0, pl.shape[0], chunk):
        b = min(a + chunk, pl.shape[0])
        i = ids[a:b].long()
        same = level[i] == pl[a:b, 3:4]
        first = torch.argmax(same.to(torch.uint8), dim=1, keepdim=True)
        owner = torch.gather(i, 1, first).squeeze(1)
        out[a:b] = sample_mask[owner]
    return out


@pytest.fixture(scope="module")
def big(amr):
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    xyz, lv, val, iso = amrgen.octree_shell_torch(2048, 5, (480.0, 560.0), 0.6, 0.575, 5, dev,
                                                  sigma=(80.0, 320.0))
    n = int(lv.numel())
    _say("serving set: %d cells, iso %r" % (n, iso))
    assert n > 600_000_000
    s = amr.AmrSet(0)
    s.upload(xyz, lv, val)
    s.build_index()
    return xyz, lv, val, iso, s


def test_serving_set_sampled(amr, big):
    dev = torch.device("cuda", 0)
    xyz, lv, val, iso, s = big

    # GPU: the whole set
    pl, ids = s.dual_cells()
    r = s.isosurface(iso, cells=True, dual=True)
    assert r["n_duals"] == pl.shape[0]

    # the sample: cells whose lower corner lies in a box around the surface
    # point nearest a fixed point on the shell (whatever the triangle order),
    # grown until it holds at least 1M cells
    v0 = r["tris"][:, :3].double()
    target = torch.tensor([1024.0 + 520.0, 1024.0, 1024.0], dtype=torch.float64, device=dev)
    near_v = v0[torch.argmin(((v0 - target) ** 2).sum(1))]
    centre = torch.floor(near_v).to(torch.int32)
    half = 32
    while True:
        lo, hi = centre - half, centre + half
        in_box = ((xyz >= lo) & (xyz < hi)).all(1)
        n_sample = int(in_box.sum().item())
        if n_sample >= 1_000_000:
            break
        half += 16
    lmax = int(lv.max().item())
    halo = 2 << lmax
    width = (torch.ones_like(lv) << lv).unsqueeze(1)
    near = ((xyz + width > lo - halo) & (xyz < hi + halo)).all(1)
    sub = torch.cat([in_box.nonzero().squeeze(1), (near & ~in_box).nonzero().squeeze(1)])
    _say("sample: %d cells in a box of side %d around %s, oracle input %d cells"
         % (n_sample, 2 * half, centre.tolist(), len(sub)))

    owned = _owned(pl, ids, lv, in_box)
    tsel = owned[r["dual"].long()]
    pl_g, ids_g = pl[owned].cpu().numpy(), ids[owned].cpu().numpy()
    tg, cg = r["tris"][tsel].cpu().numpy(), r["cells"][tsel].cpu().numpy()
    _say("gpu: %d duals, %d triangles in all; %d duals, %d triangles owned by the sample"
         % (pl.shape[0], r["tris"].shape[0], len(pl_g), len(tg)))
    del pl, ids, owned, r, tsel
    torch.cuda.empty_cache()

    # oracle: the sample (first n_sample cells of its input) and the halo
    sub_np = sub.cpu().numpy().astype(np.int64)
    o = oracle.Oracle(xyz[sub].cpu().numpy(), lv[sub].cpu().numpy(), val[sub].cpu().numpy(), validate=False)
    opl, oids = o.dual_cells(0, n_sample)
    _say("oracle: %d duals" % len(opl))
    a = oracle.canonical_duals(pl_g, ids_g)
    b = oracle.canonical_duals(opl, sub_np[oids].astype(np.int32))
    assert len(a[0]) == len(b[0]) > 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    ro = o.isosurface(iso, 0, n_sample)
    _say("oracle: %d triangles" % len(ro["tris"]))
    A, AC, _ = canon_by_cells(tg, cg)
    B, BC, _ = canon_by_cells(ro["tris"], sub_np[ro["cells"]])
    assert len(A) == len(B) > 0
    assert np.array_equal(AC, BC)
    assert same_positions(A, B)


def test_serving_mix_on_the_resident_set(amr, big):
    """Requests served against the 608.9M-cell resident set, mixed with
    uploads, give what each gives alone: the same bits in the same order
    (an upload's index is built afresh, and a build's output order depends
    on its cells alone)."""
    from paper_2004_08475_amd import serve

    xyz, lv, val, iso, s = big
    sample = val[torch.randint(0, val.numel(), (1 << 20,), device=val.device,
                               generator=torch.Generator(val.device).manual_seed(7))]
    isos = torch.quantile(sample.double(), torch.linspace(0.1, 0.9, 9, device=val.device,
                                                          dtype=torch.float64)).float().cpu().numpy()
    uploads = [amrgen.random_octree(400 + k, roots=3, root_level=3, p_split=0.5, p_hole=0.05, values="smooth")
               for k in range(3)]

    def up(k):
        u = uploads[k % len(uploads)]
        return serve.UploadRequest(u.xyz, u.level, u.value, u.iso)

    trace = serve.poisson_trace(20.0, 2.0, 17, lambda k: isos[k % len(isos)], up, p_upload=0.3)
    _say("mix on the resident set: %d requests" % len(trace))
    srv = serve.IsoServer(s, upload_slots=2)
    out = srv.serve(trace)
    _say("served; checking each request alone")
    assert len(out) == len(trace)
    for (at, req), r in zip(trace, out):
        if isinstance(req, serve.IsoRequest):
            want = s.isosurface(req.iso)["tris"]
            assert r.triangles == want.shape[0]
            assert torch.equal(r.tris, want)
        else:
            alone = amr.from_numpy(req.xyz, req.level, req.value).isosurface(req.iso)["tris"]
            assert torch.equal(r.tris, alone)
