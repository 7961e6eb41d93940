"""Batched iso-surfaces (one batched run over many (set, iso) jobs).

Every job's output must equal the CPU oracle's iso-surface of its set at its
iso: the triangle count, the triangle positions bit for bit, and (through
the plain single-iso path, which the job equals bit for bit and in order,
and which also names each vertex's cell pair) the cell-pair topology.  Sets
above a million cells are checked on windows of owner cells (all triangles
of the duals those cells generate).  Graph replays must equal eager runs."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import amrgen
import oracle

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _util import canon_by_cells, same_positions, window_matches_oracle  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ORACLE_THREADS = 8


def _say(msg):
    print(msg, flush=True)


def _check_job_against_oracle(s, iso, got, ro):
    """One batched job (float32 [T, 9]) against the oracle's output for the
    whole set: count and positions directly, topology through the plain path."""
    g = got.cpu().numpy()
    assert len(g) == len(ro["tris"])
    A, _ = oracle.canonical_triangles(g)
    B, _ = oracle.canonical_triangles(ro["tris"])
    assert same_positions(A, B)
    r = s.isosurface(float(iso), cells=True)
    assert torch.equal(r["tris"], got)
    AT, AC, _ = canon_by_cells(r["tris"].cpu().numpy(), r["cells"].cpu().numpy())
    BT, BC, _ = canon_by_cells(ro["tris"], ro["cells"])
    assert np.array_equal(AC, BC)
    assert same_positions(AT, BT)


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


@pytest.mark.parametrize("block,unit", [(256, 256), (128, 128), (256, 64), (128, 1024)])
def test_many_isos_one_set_equal_plain(amr, shell, block, unit):
    cs, s = shell
    isos = np.quantile(cs.value, np.linspace(0.05, 0.95, 16)).astype(np.float32)
    print("batch %d isos, block %d, unit %d" % (len(isos), block, unit), flush=True)
    b = amr.AmrBatch([s])
    outs = b.isosurface([0] * len(isos), isos, block, unit)
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
    outs = b.isosurface(jobs_set, jobs_iso, 256, 256)
    for si, iso, got in zip(jobs_set, jobs_iso, outs):
        assert torch.equal(got, _plain(sets[si], iso))


def test_batch_edge_cases(amr, shell):
    """A job with a NaN iso or naming no set of the batch counts -1 and writes
    nothing; a job on an empty set, or at an iso outside the values, counts 0;
    two equal jobs both equal the plain path; a set no job names costs
    nothing; launch shapes outside the documented ones are errors."""
    cs, s = shell
    e = amr.from_numpy(np.zeros((0, 3), np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    sm = amrgen.two_level_sphere()
    t = amr.from_numpy(sm.xyz, sm.level, sm.value)
    u = amr.from_numpy(sm.xyz, sm.level, sm.value)  # named by no job
    b = amr.AmrBatch([s, e, t, u])
    jobs_set = [0, 0, 0, 1, 0, 0, 7, 2, -1]
    jobs_iso = [cs.iso, cs.iso, float("nan"), 5.0, 1e30, -1e30, 5.0, sm.iso, cs.iso]
    want = {0: _plain(s, cs.iso), 1: _plain(s, cs.iso), 7: _plain(t, sm.iso)}
    n = len(jobs_iso)
    caps = [len(want[k]) if k in want else 16 for k in range(n)]
    off = np.concatenate([[0], np.cumsum(caps)[:-1]])
    tris = torch.full((int(sum(caps)), 9), -3.0, dtype=torch.float32, device=s.device)
    counts = torch.zeros(n, dtype=torch.int64, device=s.device)
    for block, unit in ((256, 256), (128, 64)):
        tris.fill_(-3.0)
        jobs = b.jobs_tensor(jobs_set, jobs_iso, off, caps)
        b.run_into(jobs, n, tris, counts, block, unit)
        torch.cuda.synchronize()
        c = counts.tolist()
        assert c == [len(want[0]), len(want[1]), -1, 0, 0, 0, -1, len(want[7]), -1]
        for k in range(n):
            got = tris[int(off[k]):int(off[k]) + caps[k]]
            if k in want:
                assert torch.equal(got, want[k])
            else:
                assert torch.all(got == -3.0)
    for block, unit in ((256, 100), (192, 256), (256, 2048), (128, 32)):
        with pytest.raises(amr.AmrError):
            b.workspace(n, block, unit)


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
    ws = b.workspace(n, 256, 128)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run_into(jobs, n, tris, counts, 256, 128, ws)  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_into(jobs, n, tris, counts, 256, 128, ws)
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


def test_batched_launch_shapes_agree(amr, shell):
    """octree-shell-256 with 64 isos at percentiles 5 + 90 k / 63 in the
    launch shapes (256 threads, 256 groups) and (128, 64): every job equals the plain path bit
    for bit (the oracle tests below cover the jobs themselves)."""
    cs, s = shell
    isos = np.quantile(cs.value, 0.05 + 0.90 * np.arange(64) / 63).astype(np.float32)
    b = amr.AmrBatch([s])
    want = [_plain(s, iso) for iso in isos]
    for block, unit in ((256, 256), (128, 64)):
        outs = b.isosurface([0] * len(isos), isos, block, unit)
        for w, got in zip(want, outs):
            assert torch.equal(got, w)


def test_many_isos_equal_oracle(amr, shell):
    """octree-shell-256 at 64 isos (percentiles 5 + 90 k / 63), one launch,
    every job against the oracle on the whole set."""
    cs, s = shell
    isos = np.quantile(cs.value, 0.05 + 0.90 * np.arange(64) / 63).astype(np.float32)
    b = amr.AmrBatch([s])
    outs = b.isosurface([0] * len(isos), isos, 256, 256)
    o = oracle.Oracle(cs.xyz, cs.level, cs.value)
    with ThreadPoolExecutor(ORACLE_THREADS) as ex:
        ros = list(ex.map(lambda v: o.isosurface(float(v)), isos))
    _say("64 isos: %d triangles in all" % sum(len(r["tris"]) for r in ros))
    for iso, got, ro in zip(isos, outs, ros):
        _check_job_against_oracle(s, iso, got, ro)


def test_many_isos_two_million_cells_equal_oracle(amr):
    """The ~2M-cell octree at 64 isos in one launch; each job is checked on
    its own window of 40,000 owner cells of the shuffled input."""
    cs = amrgen.octree_shell_2m()
    _say("octree-shell-256-2m: %d cells" % cs.n)
    s = amr.from_numpy(cs.xyz, cs.level, cs.value)
    isos = np.quantile(cs.value, 0.05 + 0.90 * np.arange(64) / 63).astype(np.float32)
    b = amr.AmrBatch([s])
    outs = b.isosurface([0] * len(isos), isos, 256, 128)
    pl, ids = (t.cpu().numpy() for t in s.dual_cells())
    o = oracle.Oracle(cs.xyz, cs.level, cs.value, validate=False)
    win = 40_000
    jobs = []
    for k, (iso, got) in enumerate(zip(isos, outs)):
        r = s.isosurface(float(iso), cells=True, dual=True)
        assert torch.equal(r["tris"], got)
        c0 = (k * 29_989) % (cs.n - win)
        jobs.append((iso, r["tris"].cpu().numpy(), r["cells"].cpu().numpy(), r["dual"].cpu().numpy(), c0))
    with ThreadPoolExecutor(ORACLE_THREADS) as ex:
        n = list(ex.map(lambda j: window_matches_oracle(o, j[0], pl, ids, j[1], j[2], j[3], j[4], j[4] + win), jobs))
    _say("2M-cell set: %d triangles compared over 64 windows" % sum(n))
    assert sum(n) > 0


def test_multiset_batch_equal_oracle(amr):
    """The 32 octree sets of log-uniform sizes in [10k, 5M] cells (seed 4),
    each at its median iso, in one launch: sets up to 1M cells against the
    oracle on the whole set, larger ones on two windows of 60,000 owner
    cells each."""
    sizes = np.exp(np.random.default_rng(4).uniform(np.log(1e4), np.log(5e6), 32)).astype(int)
    css = [amrgen.octree_sized(int(n), seed=200 + k) for k, n in enumerate(sizes)]
    _say("32 sets, %d cells in all" % sum(c.n for c in css))
    sets = [amr.from_numpy(c.xyz, c.level, c.value) for c in css]
    b = amr.AmrBatch(sets)
    outs = b.isosurface(list(range(len(sets))), [c.iso for c in css], 256, 256)
    for a, c in zip(outs, b.isosurface(list(range(len(sets))), [c.iso for c in css], 128, 512)):
        assert torch.equal(a, c)  # another launch shape, the same bits
    small = [k for k, c in enumerate(css) if c.n <= 1_000_000]
    large = [k for k, c in enumerate(css) if c.n > 1_000_000]
    orcs = {k: oracle.Oracle(css[k].xyz, css[k].level, css[k].value, validate=(css[k].n <= 1_000_000))
            for k in range(len(css))}
    with ThreadPoolExecutor(ORACLE_THREADS) as ex:
        ros = dict(zip(small, ex.map(lambda k: orcs[k].isosurface(float(css[k].iso)), small)))
    for k in small:
        _check_job_against_oracle(sets[k], css[k].iso, outs[k], ros[k])
    _say("%d sets checked whole, %d on windows" % (len(small), len(large)))
    win = 60_000
    jobs = []
    for k in large:
        cs, s = css[k], sets[k]
        r = s.isosurface(float(cs.iso), cells=True, dual=True)
        assert torch.equal(r["tris"], outs[k])
        pl, ids = (t.cpu().numpy() for t in s.dual_cells())
        for c0 in (cs.n // 5, (3 * cs.n) // 5):
            jobs.append((k, pl, ids, r["tris"].cpu().numpy(), r["cells"].cpu().numpy(), r["dual"].cpu().numpy(), c0))
    with ThreadPoolExecutor(ORACLE_THREADS) as ex:
        n = list(ex.map(lambda j: window_matches_oracle(orcs[j[0]], css[j[0]].iso, j[1], j[2], j[3], j[4], j[5],
                                                        j[6], j[6] + win), jobs))
    assert all(x >= 0 for x in n)
