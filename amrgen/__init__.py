"""Seeded synthetic AMR cell sets.

This module only *produces inputs*: flat, unsorted lists of AMR cells
(int32 lower corner, int32 level, float32 value) plus an iso-value.  It holds
none of the dual-mesh / iso-surface arithmetic; both the CPU oracle and the
HIP library consume its arrays.

Cell convention (paper, section 3.1): level 0 is the finest level, a level-l
cell has width 2^l and a lower corner that is a multiple of 2^l.

Randomness is counter based: every random number is a pure function of
(seed, stream, key) through the SplitMix64 output function (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), so a
cell's random draw does not depend on the order in which cells are visited.
The final cell order is a seeded shuffle (sort by a hash of the cell key).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_U64 = np.uint64
_MASK = (1 << 64) - 1


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
    return z ^ (z >> _U64(31))


def hash64(seed: int, stream: int, key) -> np.ndarray:
    """64-bit hash of (seed, stream, key); key is a uint64 array."""
    s = ((seed * 0x9E3779B97F4A7C15) ^ (stream * 0xD1B54A32D192ED03)) & _MASK
    s = int(_mix64(np.array([s], dtype=np.uint64))[0])
    return _mix64(np.asarray(key, dtype=np.uint64) ^ _U64(s))


def uniform(seed: int, stream: int, key) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of hash64."""
    return (hash64(seed, stream, key) >> _U64(11)).astype(np.float64) * (1.0 / (1 << 53))


def cell_key(x, y, z, level) -> np.ndarray:
    """Unique uint64 label of a cell (x, y, z >= -2^19 and < 2^19 assumed)."""
    off = 1 << 19
    ux = (np.asarray(x, np.int64) + off).astype(np.uint64)
    uy = (np.asarray(y, np.int64) + off).astype(np.uint64)
    uz = (np.asarray(z, np.int64) + off).astype(np.uint64)
    lv = np.asarray(level, np.int64).astype(np.uint64)
    return (lv << _U64(60)) | (uz << _U64(40)) | (uy << _U64(20)) | ux


@dataclass
class CellSet:
    """A flat AMR cell list in structure-of-arrays form."""
    xyz: np.ndarray          # int32 [n, 3], lower corners
    level: np.ndarray        # int32 [n]
    value: np.ndarray        # float32 [n]
    iso: float = 0.0         # default iso-value for this workload
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.level.shape[0])

    def shuffled(self, seed: int) -> "CellSet":
        key = cell_key(self.xyz[:, 0], self.xyz[:, 1], self.xyz[:, 2], self.level)
        order = np.argsort(hash64(seed, 99, key), kind="stable")
        return CellSet(np.ascontiguousarray(self.xyz[order]), np.ascontiguousarray(self.level[order]),
                       np.ascontiguousarray(self.value[order]), self.iso, self.name, dict(self.meta))

    def centres(self) -> np.ndarray:
        w = (1 << self.level.astype(np.int64)).astype(np.float64)
        return self.xyz.astype(np.float64) + 0.5 * w[:, None]


def _make(xyz, level, value, iso, name, seed, **meta) -> CellSet:
    cs = CellSet(np.ascontiguousarray(np.asarray(xyz, np.int32).reshape(-1, 3)),
                 np.ascontiguousarray(np.asarray(level, np.int32)),
                 np.ascontiguousarray(np.asarray(value, np.float32)), float(np.float32(iso)), name, meta)
    return cs.shuffled(seed)


_CHILD = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.int64)


# ---------------------------------------------------------------------------
# Workload 1: tiny two-level set, 16^3 domain
# ---------------------------------------------------------------------------

def two_level_sphere(seed: int = 1) -> CellSet:
    """512 level-0 cells filling [4,12)^3 and 448 level-1 cells filling the rest
    of [0,16)^3; value = |centre - (8,8,8)| (computed in float64, stored as
    float32); iso 5.0."""
    r = np.arange(4, 12)
    fine = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    r2 = np.arange(0, 16, 2)
    coarse = np.stack(np.meshgrid(r2, r2, r2, indexing="ij"), -1).reshape(-1, 3)
    inside = np.all((coarse >= 4) & (coarse < 12), axis=1)
    coarse = coarse[~inside]
    xyz = np.concatenate([fine, coarse])
    lvl = np.concatenate([np.zeros(len(fine), np.int32), np.ones(len(coarse), np.int32)])
    c = xyz.astype(np.float64) + 0.5 * (1 << lvl)[:, None]
    val = np.sqrt(((c - 8.0) ** 2).sum(1))
    return _make(xyz, lvl, val, 5.0, "two-level-sphere-16", seed)


# ---------------------------------------------------------------------------
# Octree sets: random refinement concentrated on a spherical shell
# ---------------------------------------------------------------------------

def _box_hits_shell(lo, w, c, r0, r1):
    lo = lo.astype(np.float64)
    hi = lo + w
    d = np.maximum(np.maximum(lo - c, 0.0), c - hi)
    dmin = np.sqrt((d * d).sum(1))
    far = np.maximum(np.abs(lo - c), np.abs(hi - c))
    dmax = np.sqrt((far * far).sum(1))
    return (dmin < r1) & (dmax > r0)


def _gaussian_field(pts, seed, domain, n_g=8, sig=(10.0, 40.0), amp=(0.5, 1.5)):
    k = np.arange(n_g, dtype=np.uint64)
    mu = np.stack([uniform(seed, 10 + a, k) * domain for a in range(3)], 1)
    sg = sig[0] + (sig[1] - sig[0]) * uniform(seed, 13, k)
    am = amp[0] + (amp[1] - amp[0]) * uniform(seed, 14, k)
    out = np.zeros(len(pts), np.float64)
    for g in range(n_g):
        d2 = ((pts - mu[g]) ** 2).sum(1)
        out += am[g] * np.exp(-d2 / (2.0 * sg[g] ** 2))
    return out, dict(mu=mu, sigma=sg, amp=am)


def octree_shell(domain: int = 256, root_level: int = 4, shell=(60.0, 70.0), p_in: float = 0.6,
                 p_out: float = 0.1, seed: int = 2, sigma=(10.0, 40.0), n_gauss: int = 8,
                 name: str | None = None) -> CellSet:
    """Octree AMR without 2:1 balance.  Roots are level-`root_level` cells tiling
    [0, domain)^3; every cell above level 0 is split into its 8 children with
    probability p_in if its box meets the shell r0 < |x - c| < r1 around the
    domain centre, else p_out.  Value: sum of `n_gauss` seeded isotropic
    Gaussians at the cell centre; iso: the lower median of the cell values."""
    w0 = 1 << root_level
    assert domain % w0 == 0
    n = domain // w0
    r = np.arange(n, dtype=np.int64) * w0
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    c = domain / 2.0
    leaves, lvls = [], []
    lvl = root_level
    while True:
        w = 1 << lvl
        if lvl == 0 or len(g) == 0:
            leaves.append(g)
            lvls.append(np.full(len(g), lvl, np.int32))
            break
        hit = _box_hits_shell(g, w, c, shell[0], shell[1])
        u = uniform(seed, 1, cell_key(g[:, 0], g[:, 1], g[:, 2], np.full(len(g), lvl)))
        split = u < np.where(hit, p_in, p_out)
        leaves.append(g[~split])
        lvls.append(np.full(int((~split).sum()), lvl, np.int32))
        g = (g[split][:, None, :] + _CHILD[None] * (w // 2)).reshape(-1, 3)
        lvl -= 1
    xyz = np.concatenate(leaves)
    lv = np.concatenate(lvls)
    ctr = xyz.astype(np.float64) + 0.5 * (1 << lv.astype(np.int64))[:, None]
    val, gp = _gaussian_field(ctr, seed, float(domain), n_gauss, sigma)
    v32 = val.astype(np.float32)
    iso = np.sort(v32)[(len(v32) - 1) // 2]
    nm = name or f"octree-shell-{domain}"
    return _make(xyz, lv, v32, float(iso), nm, seed, domain=domain, root_level=root_level,
                 shell=tuple(shell), p_in=p_in, p_out=p_out, **gp)


def octree_shell_2m(seed: int = 2) -> CellSet:
    """The octree-shell recipe on 256^3 (levels 0..4, split probability 0.6
    for cells meeting the shell 60 < r < 70) with the probability elsewhere
    raised from 0.1 to 0.565, which gives the ~2M cells the workload states
    (2,017,464 cells at seed 2; with 0.1 the recipe gives 136,935)."""
    return octree_shell(p_out=0.565, seed=seed, name="octree-shell-256-2m")


def octree_sized(target_cells: int, seed: int) -> CellSet:
    """Octree-shell set whose domain is scaled (shell radii with it) so that the
    cell count lands near `target_cells`; used for batches of uneven sets."""
    base = 136_669.0  # cells of the 256^3 recipe at seed 2
    s = (max(target_cells, 1000) / base) ** (1.0 / 3.0)
    domain = max(32, int(round(256 * s / 16.0)) * 16)
    k = domain / 256.0
    return octree_shell(domain=domain, shell=(60.0 * k, 70.0 * k), seed=seed,
                        sigma=(10.0 * k, 40.0 * k), name=f"octree-shell-{domain}-s{seed}")


# ---------------------------------------------------------------------------
# Small sets for property tests
# ---------------------------------------------------------------------------

def uniform_grid(n: int, level: int = 0, seed: int = 5, origin=(0, 0, 0), field_kind: str = "gauss") -> CellSet:
    """n^3 cells on one level; value from a smooth seeded field."""
    w = 1 << level
    r = np.arange(n, dtype=np.int64) * w
    xyz = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3) + np.asarray(origin, np.int64)
    ctr = xyz.astype(np.float64) + 0.5 * w
    if field_kind == "gauss":
        val, _ = _gaussian_field(ctr - np.asarray(origin, np.float64), seed, float(n * w), 4,
                                 (0.15 * n * w, 0.4 * n * w))
    else:
        val = uniform(seed, 7, cell_key(xyz[:, 0], xyz[:, 1], xyz[:, 2], np.full(len(xyz), level)))
    v32 = val.astype(np.float32)
    iso = np.sort(v32)[(len(v32) - 1) // 2]
    return _make(xyz, np.full(len(xyz), level, np.int32), v32, float(iso), f"grid-{n}-l{level}", seed)


def random_octree(seed: int, roots: int = 2, root_level: int = 3, p_split: float = 0.45,
                  p_hole: float = 0.0, origin=(0, 0, 0), values: str = "random") -> CellSet:
    """Tiny random octree: roots^3 root cells, each cell split with probability
    p_split, leaves dropped (holes) with probability p_hole.  Level jumps are
    unrestricted.  Values are seeded uniforms (or a smooth field)."""
    w0 = 1 << root_level
    r = np.arange(roots, dtype=np.int64) * w0
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3) + np.asarray(origin, np.int64)
    leaves, lvls = [], []
    lvl = root_level
    while len(g):
        w = 1 << lvl
        key = cell_key(g[:, 0], g[:, 1], g[:, 2], np.full(len(g), lvl))
        split = (uniform(seed, 1, key) < p_split) if lvl > 0 else np.zeros(len(g), bool)
        keep = ~split
        leaves.append(g[keep])
        lvls.append(np.full(int(keep.sum()), lvl, np.int32))
        g = (g[split][:, None, :] + _CHILD[None] * (w // 2)).reshape(-1, 3)
        lvl -= 1
    xyz = np.concatenate(leaves)
    lv = np.concatenate(lvls)
    if p_hole > 0:
        u = uniform(seed, 2, cell_key(xyz[:, 0], xyz[:, 1], xyz[:, 2], lv))
        m = u >= p_hole
        xyz, lv = xyz[m], lv[m]
    key = cell_key(xyz[:, 0], xyz[:, 1], xyz[:, 2], lv)
    if values == "random":
        val = uniform(seed, 3, key)
    else:
        ctr = xyz.astype(np.float64) + 0.5 * (1 << lv.astype(np.int64))[:, None]
        ext = float(roots * w0)
        val, _ = _gaussian_field(ctr - np.asarray(origin, np.float64), seed, ext, 3, (0.2 * ext, 0.5 * ext))
    v32 = val.astype(np.float32)
    iso = np.sort(v32)[(len(v32) - 1) // 2] if len(v32) else 0.0
    return _make(xyz, lv, v32, float(iso), f"random-octree-s{seed}", seed)


WORKLOADS = {
    "two-level-sphere-16": two_level_sphere,
    "octree-shell-256": octree_shell,
    "octree-shell-256-2m": octree_shell_2m,
}


# ---------------------------------------------------------------------------
# Block-structured set with holes: 8^3-cell bricks on 4 levels around
# synthetic vortex tubes
# ---------------------------------------------------------------------------

def _helices(seed, n, domain):
    k = np.arange(n, dtype=np.uint64)
    rnd = lambda st: uniform(seed, st, k)
    c = np.stack([domain * (0.3 + 0.4 * rnd(20 + a)) for a in range(3)], 1)
    # axis from a uniform direction
    zc = 2.0 * rnd(23) - 1.0
    ph = 2.0 * np.pi * rnd(24)
    ax = np.stack([np.sqrt(1 - zc * zc) * np.cos(ph), np.sqrt(1 - zc * zc) * np.sin(ph), zc], 1)
    tmp = np.where(np.abs(ax[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    u = np.cross(ax, tmp)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(ax, u)
    R = 40.0 + 100.0 * rnd(25)
    P = 150.0 + 250.0 * rnd(26)
    # circulation: log-normal spread, core radius uniform
    z = np.sqrt(-2.0 * np.log(np.maximum(rnd(27), 1e-300))) * np.cos(2 * np.pi * rnd(28))
    gamma = np.exp(z)
    rc = 8.0 + 24.0 * rnd(29)
    return dict(c=c, a=ax, u=u, v=v, R=R, P=P, gamma=gamma, rc=rc)


def _helix_dist(pts, H, i):
    """Distance from pts [n,3] to helix i and the unit tangent at the nearest
    of three candidate turns (nearest in axial position)."""
    d = pts - H["c"][i]
    z = d @ H["a"][i]
    th = np.arctan2(d @ H["v"][i], d @ H["u"][i])
    R, P = H["R"][i], H["P"][i]
    k0 = np.round((2 * np.pi * z / P - th) / (2 * np.pi))
    best = np.full(len(pts), np.inf)
    best_s = np.zeros(len(pts))
    for dk in (-1.0, 0.0, 1.0):
        s = th + 2 * np.pi * (k0 + dk)
        h = (R * np.cos(s))[:, None] * H["u"][i] + (R * np.sin(s))[:, None] * H["v"][i] + \
            (P * s / (2 * np.pi))[:, None] * H["a"][i]
        dd = ((d - h) ** 2).sum(1)
        better = dd < best
        best = np.where(better, dd, best)
        best_s = np.where(better, s, best_s)
    t = (-R * np.sin(best_s))[:, None] * H["u"][i] + (R * np.cos(best_s))[:, None] * H["v"][i] + \
        (P / (2 * np.pi)) * H["a"][i]
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return np.sqrt(best), t


def _vortex_values_torch(xyz, lv, H, n_helix, device, chunk):
    """Same field as the numpy path, evaluated with torch (float64) on
    `device`; used to generate large sets quickly.  Results can differ from
    the numpy path in the last bit of some values."""
    import torch

    out = np.empty(len(xyz), np.float32)
    Ht = {k: torch.as_tensor(np.asarray(v), dtype=torch.float64, device=device) for k, v in H.items()}
    for s0 in range(0, len(xyz), chunk):
        p = torch.as_tensor(xyz[s0:s0 + chunk], device=device).to(torch.float64)
        w = torch.as_tensor(lv[s0:s0 + chunk], device=device).to(torch.int64)
        p = p + 0.5 * torch.pow(2.0, w.to(torch.float64))[:, None]
        om = torch.zeros_like(p)
        for i in range(n_helix):
            d = p - Ht["c"][i]
            z = d @ Ht["a"][i]
            th = torch.atan2(d @ Ht["v"][i], d @ Ht["u"][i])
            R, P = Ht["R"][i], Ht["P"][i]
            k0 = torch.round((2 * np.pi * z / P - th) / (2 * np.pi))
            best = torch.full_like(z, float("inf"))
            best_s = torch.zeros_like(z)
            for dk in (-1.0, 0.0, 1.0):
                sp = th + 2 * np.pi * (k0 + dk)
                h = (R * torch.cos(sp))[:, None] * Ht["u"][i] + (R * torch.sin(sp))[:, None] * Ht["v"][i] + \
                    (P * sp / (2 * np.pi))[:, None] * Ht["a"][i]
                dd = ((d - h) ** 2).sum(1)
                better = dd < best
                best = torch.where(better, dd, best)
                best_s = torch.where(better, sp, best_s)
            t = (-R * torch.sin(best_s))[:, None] * Ht["u"][i] + (R * torch.cos(best_s))[:, None] * Ht["v"][i] + \
                (P / (2 * np.pi)) * Ht["a"][i]
            t = t / torch.linalg.norm(t, dim=1, keepdim=True)
            rc = Ht["rc"][i]
            om += (Ht["gamma"][i] / (np.pi * rc * rc) * torch.exp(-best / (rc * rc)))[:, None] * t
        out[s0:s0 + chunk] = torch.sqrt((om * om).sum(1)).to(torch.float32).cpu().numpy()
    return out


def block_vortex(domain: int = 1024, tube: float = 13.5, n_helix: int = 5, seed: int = 3,
                 obstacle=((560, 720), (380, 540), (400, 560)), chunk: int = 1 << 22, device=None) -> CellSet:
    """Block-structured AMR: 8^3-cell bricks on levels 0..3 (a level-l brick
    spans 8*2^l units); level-3 bricks tile [0, domain)^3 and a brick of level
    l > 0 is replaced by its 8 half-size bricks when it comes within
    tube * 2^(l-1) of one of `n_helix` seeded helices.  Every cell meeting the
    axis-aligned obstacle box is removed (a hole, no parent structure).
    Value: |sum of Lamb-Oseen tube vorticities| (log-normal circulations);
    iso: 90th percentile of the cell values."""
    H = _helices(seed, n_helix, float(domain))
    top = 3
    wb = 8 << top
    r = np.arange(domain // wb, dtype=np.int64) * wb
    b = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    leaves = []
    for lvl in range(top, -1, -1):
        span = 8 << lvl
        if lvl == 0 or len(b) == 0:
            leaves.append((b, lvl))
            break
        ctr = b.astype(np.float64) + span / 2.0
        dmin = np.full(len(b), np.inf)
        for i in range(n_helix):
            dmin = np.minimum(dmin, _helix_dist(ctr, H, i)[0])
        refine = dmin - np.sqrt(3.0) * span / 2.0 < tube * (1 << (lvl - 1))
        leaves.append((b[~refine], lvl))
        half = span // 2
        b = (b[refine][:, None, :] + _CHILD[None] * half).reshape(-1, 3)
    cell8 = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    xyz_parts, lv_parts = [], []
    (ox0, ox1), (oy0, oy1), (oz0, oz1) = obstacle
    for bb, lvl in leaves:
        if len(bb) == 0:
            continue
        w = 1 << lvl
        cells = (bb[:, None, :] + cell8[None] * w).reshape(-1, 3)
        hit = ((cells[:, 0] < ox1) & (cells[:, 0] + w > ox0) & (cells[:, 1] < oy1) & (cells[:, 1] + w > oy0) &
               (cells[:, 2] < oz1) & (cells[:, 2] + w > oz0))
        cells = cells[~hit]
        xyz_parts.append(cells.astype(np.int32))
        lv_parts.append(np.full(len(cells), lvl, np.int32))
    xyz = np.concatenate(xyz_parts)
    lv = np.concatenate(lv_parts)
    if device is not None:
        val = _vortex_values_torch(xyz, lv, H, n_helix, device, chunk)
    else:
        val = np.empty(len(xyz), np.float32)
        for s0 in range(0, len(xyz), chunk):
            p = xyz[s0:s0 + chunk].astype(np.float64) + 0.5 * (1 << lv[s0:s0 + chunk].astype(np.int64))[:, None]
            om = np.zeros((len(p), 3))
            for i in range(n_helix):
                d, t = _helix_dist(p, H, i)
                rc = H["rc"][i]
                om += (H["gamma"][i] / (np.pi * rc * rc) * np.exp(-(d * d) / (rc * rc)))[:, None] * t
            val[s0:s0 + chunk] = np.sqrt((om * om).sum(1)).astype(np.float32)
    iso = np.sort(val)[int(0.9 * (len(val) - 1))]
    return _make(xyz, lv, val, float(iso), "block-vortex-%d" % domain, seed, domain=domain, tube=tube,
                 obstacle=obstacle, n_helix=n_helix)


# ---------------------------------------------------------------------------
# torch port of the octree generator for very large sets (same draws, same
# cells; values may differ from the numpy path in the last bit)
# ---------------------------------------------------------------------------

def _i64(u: int) -> int:
    u &= _MASK
    return u - (1 << 64) if u >= (1 << 63) else u


def _lsr_t(z, k: int):
    import torch

    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix64_t(z):
    z = z ^ _lsr_t(z, 30)
    z = z * _i64(0xBF58476D1CE4E5B9)
    z = z ^ _lsr_t(z, 27)
    z = z * _i64(0x94D049BB133111EB)
    return z ^ _lsr_t(z, 31)


def _uniform_t(seed: int, stream: int, key):
    s = ((seed * 0x9E3779B97F4A7C15) ^ (stream * 0xD1B54A32D192ED03)) & _MASK
    s = int(_mix64(np.array([s], dtype=np.uint64))[0])
    h = _mix64_t(key ^ _i64(s))
    return _lsr_t(h, 11).double() * (1.0 / (1 << 53))


def _cell_key_t(g, lvl: int):
    off = 1 << 19
    return ((lvl << 60) | ((g[:, 2] + off) << 40) | ((g[:, 1] + off) << 20) | (g[:, 0] + off))


def octree_shell_torch(domain: int, root_level: int, shell, p_in: float, p_out: float, seed: int, device,
                       sigma=(10.0, 40.0), n_gauss: int = 8, name: str | None = None):
    """octree_shell on a torch device.  Returns (xyz int32 [n,3], level int32
    [n], value float32 [n]) device tensors, shuffled by the same seeded hash
    order as the numpy path, and the iso (lower median)."""
    import torch

    w0 = 1 << root_level
    n = domain // w0
    r = torch.arange(n, dtype=torch.int64, device=device) * w0
    gx, gy, gz = torch.meshgrid(r, r, r, indexing="ij")
    g = torch.stack([gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)], 1)
    c = domain / 2.0
    child = torch.as_tensor(_CHILD, device=device)
    xs, ls = [], []
    lvl = root_level
    while True:
        w = 1 << lvl
        if lvl == 0 or len(g) == 0:
            xs.append(g.to(torch.int32))
            ls.append(torch.full((len(g),), lvl, dtype=torch.int32, device=device))
            break
        lo = g.double()
        hi = lo + w
        d = torch.maximum(torch.maximum(lo - c, torch.zeros_like(lo)), c - hi)
        dmin = torch.sqrt((d * d).sum(1))
        far = torch.maximum((lo - c).abs(), (hi - c).abs())
        dmax = torch.sqrt((far * far).sum(1))
        hit = (dmin < shell[1]) & (dmax > shell[0])
        u = _uniform_t(seed, 1, _cell_key_t(g, lvl))
        split = u < torch.where(hit, torch.full_like(u, p_in), torch.full_like(u, p_out))
        keep = g[~split]
        xs.append(keep.to(torch.int32))
        ls.append(torch.full((len(keep),), lvl, dtype=torch.int32, device=device))
        g = (g[split][:, None, :] + child[None] * (w // 2)).reshape(-1, 3)
        del lo, hi, d, dmin, far, dmax, hit, u, split, keep
        lvl -= 1
    xyz = torch.cat(xs)
    lv = torch.cat(ls)
    del xs, ls, g
    k = np.arange(n_gauss, dtype=np.uint64)
    mu = np.stack([uniform(seed, 10 + a, k) * float(domain) for a in range(3)], 1)
    sg = sigma[0] + (sigma[1] - sigma[0]) * uniform(seed, 13, k)
    am = 0.5 + 1.0 * uniform(seed, 14, k)
    val = torch.empty(len(xyz), dtype=torch.float32, device=device)
    step = 1 << 25
    for s0 in range(0, len(xyz), step):
        ctr = xyz[s0:s0 + step].double() + 0.5 * torch.pow(2.0, lv[s0:s0 + step].double())[:, None]
        acc = torch.zeros(len(ctr), dtype=torch.float64, device=device)
        for gi in range(n_gauss):
            d2 = ((ctr - torch.as_tensor(mu[gi], device=device)) ** 2).sum(1)
            acc += am[gi] * torch.exp(-d2 / (2.0 * sg[gi] ** 2))
        val[s0:s0 + step] = acc.float()
        del ctr, acc
    key = _cell_key_t(xyz.long(), 0) ^ (lv.long() << 60)
    h = _mix64_t(key ^ _i64(int(_mix64(np.array([((seed * 0x9E3779B97F4A7C15) ^ (99 * 0xD1B54A32D192ED03)) & _MASK],
                                                   dtype=np.uint64))[0])))
    order = torch.argsort(h ^ _i64(1 << 63), stable=True)  # unsigned order of the hash
    del h, key
    xyz, lv, val = xyz[order].contiguous(), lv[order].contiguous(), val[order].contiguous()
    iso = float(torch.kthvalue(val.cpu(), (len(val) - 1) // 2 + 1).values) if len(val) < (1 << 27) else \
        float(torch.sort(val).values[(len(val) - 1) // 2])
    return xyz, lv, val, iso
