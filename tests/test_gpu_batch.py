"""Batched iso-surfaces (one persistent launch over many (set, iso) jobs):
every job's output must equal, bit for bit and in order, the plain
single-iso path on the same set and iso; graph replays must too."""
import numpy as np
import pytest

import amrgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amr():
    import paper_2004_08475_amd as amr

    amr.load_library()
    assert torch.cuda.is_available()
    return amr


def _plain(s, iso):
    return s.isosurface(float(np.float32(iso)))["tris"]


@pytest.fixture(scope="module")
def shell(amr):
    cs = amrgen.octree_shell()
    return cs, amr.from_numpy(cs.xyz, cs.level, cs.value)


@pytest.mark.parametrize("block,per", [(256, 1), (128, 2), (512, 1), (64, 4)])
def test_many_isos_one_set_equal_plain(amr, shell, block, per):
    cs, s = shell
    isos = np.quantile(cs.value, np.linspace(0.05, 0.95, 16)).astype(np.float32)
    print("batch %d isos, block %d x %d" % (len(isos), block, per), flush=True)
    b = amr.AmrBatch([s])
    outs = b.isosurface([0] * len(isos), isos, block, per)
    for iso, got in zip(isos, outs):
        want = _plain(s, iso)
        assert got.shape == want.shape
        assert torch.equal(got, want)


def test_many_sets_own_iso_equal_plain(amr):
    sets, css = [], []
    for k, (roots, p) in enumerate([(2, 0.5), (4, 0.45), (3, 0.6), (6, 0.4), (1, 0.0), (5, 0.5)]):
        cs = amrgen.random_octree(100 + k, roots=roots, root_level=3, p_split=p, p_hole=0.1 * (k % 2),
                                  values="smooth", origin=(8 * k, -16 * k, 0))
        css.append(cs)
        sets.append(amr.from_numpy(cs.xyz, cs.level, cs.value))
    print("batch over %d sets: %s cells" % (len(sets), [c.n for c in css]), flush=True)
    b = amr.AmrBatch(sets)
    jobs_set = list(range(len(sets))) + [1, 3]
    jobs_iso = [c.iso for c in css] + [float(np.quantile(css[1].value, 0.2)), float(np.quantile(css[3].value, 0.8))]
    outs = b.isosurface(jobs_set, jobs_iso, 256, 1)
    for si, iso, got in zip(jobs_set, jobs_iso, outs):
        assert torch.equal(got, _plain(sets[si], iso))


def test_batch_capacity_contract(amr, shell):
    cs, s = shell
    b = amr.AmrBatch([s])
    iso = [cs.iso, float(np.quantile(cs.value, 0.3))]
    full = [_plain(s, v) for v in iso]
    caps = [len(full[0]) // 2, 0]
    tris = torch.full((caps[0] + 8, 9), -3.0, dtype=torch.float32, device=s.device)
    counts = torch.zeros(2, dtype=torch.int64, device=s.device)
    jobs = b.jobs_tensor([0, 0], iso, [0, caps[0]], caps)
    b.run_into(jobs, 2, tris, counts)
    torch.cuda.synchronize()
    assert counts.tolist() == [len(full[0]), len(full[1])]
    assert torch.equal(tris[:caps[0]], full[0][:caps[0]])
    assert torch.all(tris[caps[0]:] == -3.0)


def test_batch_graph_replay_with_new_isos(amr, shell):
    cs, s = shell
    b = amr.AmrBatch([s])
    rounds = [np.quantile(cs.value, q).astype(np.float32) for q in ([0.2, 0.5, 0.8], [0.3, 0.6, 0.9], [0.1, 0.4, 0.7])]
    cap = 4 * max(len(_plain(s, v)) for r in rounds for v in r)
    n = 3
    tris = torch.zeros((n * cap, 9), dtype=torch.float32, device=s.device)
    counts = torch.zeros(n, dtype=torch.int64, device=s.device)
    jobs = b.jobs_tensor([0] * n, rounds[0], [k * cap for k in range(n)], [cap] * n)
    ws = b.workspace(n, 256, 1)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run_into(jobs, n, tris, counts, 256, 1, ws)  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_into(jobs, n, tris, counts, 256, 1, ws)
    for r in rounds + rounds[:1]:
        new = b.jobs_tensor([0] * n, r, [k * cap for k in range(n)], [cap] * n)
        jobs.copy_(new)
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays
        want = [_plain(s, v) for v in r]
        c = counts.tolist()
        for k in range(n):
            assert c[k] == len(want[k])
            assert torch.equal(tris[k * cap:k * cap + c[k]], want[k])
    assert not b.barrier_timed_out(256, 1)


def test_batched_configurations_at_full_size(amr, shell):
    """The two batched workloads bench.py times, at full size, in the launch
    shapes the autotuner picks for them (512 x 1 and 256 x 2) and the default
    one: octree-shell-256 with 64 isos at percentiles 5 + 90 k / 63, and 32
    octree sets of log-uniform sizes in [10k, 5M] cells (seed 4), each at its
    median iso.  Every job equals the plain path bit for bit."""
    cs, s = shell
    isos = np.quantile(cs.value, 0.05 + 0.90 * np.arange(64) / 63).astype(np.float32)
    b = amr.AmrBatch([s])
    want = [_plain(s, iso) for iso in isos]
    for block, per in ((512, 1), (256, 1)):
        outs = b.isosurface([0] * len(isos), isos, block, per)
        for w, got in zip(want, outs):
            assert torch.equal(got, w)
    sizes = np.exp(np.random.default_rng(4).uniform(np.log(1e4), np.log(5e6), 32)).astype(int)
    css = [amrgen.octree_sized(int(n), seed=200 + k) for k, n in enumerate(sizes)]
    print("32 sets, %d cells in all" % sum(c.n for c in css), flush=True)
    sets = [amr.from_numpy(c.xyz, c.level, c.value) for c in css]
    b = amr.AmrBatch(sets)
    want = [_plain(st, c.iso) for st, c in zip(sets, css)]
    for block, per in ((256, 2), (256, 1)):
        outs = b.isosurface(list(range(len(sets))), [c.iso for c in css], block, per)
        for w, got in zip(want, outs):
            assert torch.equal(got, w)
