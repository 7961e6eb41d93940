"""CPU oracle for AMR dual cells and crack-free iso-surfaces.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this package.  The product path (the HIP library and its
Python binding) never imports it, and it imports nothing from the product.

The arithmetic lives in ``amr_oracle.c`` (plain C, fp32 placement with an
explicit fma, no fast-math, no FP contraction); this module compiles it with
gcc, loads it through ctypes and adds numpy conveniences: canonical ordering
of duals and triangles, a thread-split driver for the CPU baseline, the weld
of an indexed face set, and the dual-mesh interpolant at query points (fp64,
brute force over the duals).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amr_oracle.c")
# ORACLE_LIB names another build of amr_oracle.c to load (the sanitizer
# test runs the pins against an AddressSanitizer + UBSan build)
LIB = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liborc.so")

OK, EINVAL, ERANGE, EOVERLAP, ENOSPACE = 0, -1, -2, -3, -4

_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liborc.so."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.environ.get("ORACLE_LIB") and (not os.path.exists(LIB) or
                                                  os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = C.CDLL(LIB)
        i64, i32p, f32p, i64p, vp = C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_float), C.POINTER(C.c_int64), C.c_void_p
        L.orc_check_fields.argtypes = [i64, i32p, i32p, f32p, i64p]
        L.orc_check_fields.restype = C.c_int
        L.orc_index_new.argtypes = [i64, i32p, i32p]
        L.orc_index_new.restype = vp
        L.orc_index_free.argtypes = [vp]
        L.orc_index_free.restype = None
        L.orc_locate.argtypes = [vp, i64, i64, i64]
        L.orc_locate.restype = i64
        L.orc_locate_brute.argtypes = [i64, i32p, i32p, i64, i64, i64]
        L.orc_locate_brute.restype = i64
        L.orc_check_overlap.argtypes = [vp, i64, i32p, i32p, i64p]
        L.orc_check_overlap.restype = C.c_int
        L.orc_dual_cells.argtypes = [vp, i64, i32p, i32p, i64, i64, i32p, i32p, i64]
        L.orc_dual_cells.restype = i64
        L.orc_polygonize.argtypes = [C.c_int, C.POINTER(C.c_int8)]
        L.orc_polygonize.restype = C.c_int
        L.orc_isosurface.argtypes = [vp, i64, i32p, i32p, f32p, C.c_float, i64, i64, f32p, i32p, i64p, i64, i64p]
        L.orc_isosurface.restype = i64
        L.orc_grid_mc.argtypes = [C.c_int, C.c_int, C.c_int, f32p, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_float, f32p, i32p, i64]
        L.orc_grid_mc.restype = i64
        _lib = L
        return L


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def polygonize(case: int) -> np.ndarray:
    """Triangles of MC case `case` as an int8 [T, 3] array of hex edge ids."""
    L = _load()
    out = np.zeros((16, 3), np.int8)
    nt = L.orc_polygonize(int(case), _p(out, C.c_int8))
    if nt < 0:
        raise RuntimeError("polygonize failed for case %d" % case)
    return out[:nt].copy()


def grid_mc(vals: np.ndarray, origin, h: float, iso: float):
    """Plain Marching Cubes over a regular lattice vals[k, j, i]."""
    L = _load()
    vals = np.ascontiguousarray(vals, np.float32)
    nz, ny, nx = vals.shape
    n = L.orc_grid_mc(nx, ny, nz, _p(vals, C.c_float), float(origin[0]), float(origin[1]), float(origin[2]),
                      float(h), C.c_float(iso), None, None, 0)
    tris = np.zeros((max(n, 1), 9), np.float32)
    pts = np.zeros((max(n, 1), 6), np.int32)
    L.orc_grid_mc(nx, ny, nz, _p(vals, C.c_float), float(origin[0]), float(origin[1]), float(origin[2]), float(h),
                  C.c_float(iso), _p(tris, C.c_float), _p(pts, C.c_int32), n)
    return tris[:n], pts[:n]


class Oracle:
    """Oracle over one cell set.  `locator` is "sorted" (the paper's sorted
    corners + binary search per level) or "brute" (linear scan)."""

    def __init__(self, xyz, level, value=None, locator: str = "sorted", validate: bool = True):
        self.L = _load()
        self.xyz = np.ascontiguousarray(np.asarray(xyz, np.int32).reshape(-1, 3))
        self.level = np.ascontiguousarray(np.asarray(level, np.int32))
        self.value = None if value is None else np.ascontiguousarray(np.asarray(value, np.float32))
        self.n = int(self.level.shape[0])
        self.locator = locator
        if validate:
            bad = C.c_int64(-1)
            st = self.L.orc_check_fields(self.n, _p(self.xyz, C.c_int32), _p(self.level, C.c_int32),
                                         _p(self.value, C.c_float), C.byref(bad))
            if st != OK:
                raise ValueError("invalid cell %d (status %d)" % (bad.value, st))
        self._ix = self.L.orc_index_new(self.n, _p(self.xyz, C.c_int32), _p(self.level, C.c_int32))
        if not self._ix:
            raise MemoryError("oracle index")
        if validate:
            bad = C.c_int64(-1)
            ix = self._ix if (locator == "sorted" or self.n > 4000) else None
            st = self.L.orc_check_overlap(ix, self.n, _p(self.xyz, C.c_int32), _p(self.level, C.c_int32),
                                          C.byref(bad))
            if st != OK:
                raise ValueError("overlapping cells near %d" % bad.value)

    def __del__(self):
        try:
            if getattr(self, "_ix", None):
                self.L.orc_index_free(self._ix)
                self._ix = None
        except Exception:
            pass

    @property
    def _ixp(self):
        return self._ix if self.locator == "sorted" else None

    def locate(self, q) -> int:
        q = [int(v) for v in q]
        if self.locator == "sorted":
            return int(self.L.orc_locate(self._ix, *q))
        return int(self.L.orc_locate_brute(self.n, _p(self.xyz, C.c_int32), _p(self.level, C.c_int32), *q))

    def dual_cells(self, c0: int = 0, c1: int | None = None):
        """(pl [M,4] int32 = P.xyz + level, ids [M,8] int32) in emission order."""
        c1 = self.n if c1 is None else c1
        a = (self._ixp, self.n, _p(self.xyz, C.c_int32), _p(self.level, C.c_int32), c0, c1)
        m = self.L.orc_dual_cells(*a, None, None, 0)
        pl = np.zeros((max(m, 1), 4), np.int32)
        ids = np.zeros((max(m, 1), 8), np.int32)
        self.L.orc_dual_cells(*a, _p(pl, C.c_int32), _p(ids, C.c_int32), m)
        return pl[:m], ids[:m]

    def isosurface(self, iso: float, c0: int = 0, c1: int | None = None, want_cells: bool = True):
        """dict(tris [T,9] f32, cells [T,6] i32 (A,B per vertex), dual [T] i64,
        n_duals)."""
        if self.value is None:
            raise ValueError("no values")
        c1 = self.n if c1 is None else c1
        a = (self._ixp, self.n, _p(self.xyz, C.c_int32), _p(self.level, C.c_int32), _p(self.value, C.c_float),
             C.c_float(iso), c0, c1)
        nd = C.c_int64(0)
        t = self.L.orc_isosurface(*a, None, None, None, 0, C.byref(nd))
        tris = np.zeros((max(t, 1), 9), np.float32)
        cells = np.zeros((max(t, 1), 6), np.int32) if want_cells else None
        dual = np.zeros(max(t, 1), np.int64) if want_cells else None
        self.L.orc_isosurface(*a, _p(tris, C.c_float), _p(cells, C.c_int32), _p(dual, C.c_int64), t, C.byref(nd))
        return dict(tris=tris[:t], cells=None if cells is None else cells[:t],
                    dual=None if dual is None else dual[:t], n_duals=int(nd.value))

    def count_range(self, iso: float, c0: int, c1: int):
        """(triangles, duals) of cells [c0, c1) without storing anything."""
        nd = C.c_int64(0)
        t = self.L.orc_isosurface(self._ixp, self.n, _p(self.xyz, C.c_int32), _p(self.level, C.c_int32),
                                  _p(self.value, C.c_float), C.c_float(iso), c0, c1, None, None, None, 0,
                                  C.byref(nd))
        return int(t), int(nd.value)

    def isosurface_threaded(self, iso: float, threads: int, c0: int = 0, c1: int | None = None):
        """Split [c0, c1) over `threads` threads (ctypes drops the GIL);
        returns (triangles, duals)."""
        c1 = self.n if c1 is None else c1
        edges = np.linspace(c0, c1, threads + 1).astype(np.int64)
        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(lambda k: self.count_range(iso, int(edges[k]), int(edges[k + 1])), range(threads)))
        return sum(r[0] for r in res), sum(r[1] for r in res)


# ---------------------------------------------------------------------------
# Canonical forms for comparisons
# ---------------------------------------------------------------------------

def canonical_duals(pl: np.ndarray, ids: np.ndarray):
    """Sort duals by (level, P.z, P.y, P.x)."""
    pl = np.asarray(pl)
    order = np.lexsort((pl[:, 0], pl[:, 1], pl[:, 2], pl[:, 3]))
    return pl[order], np.asarray(ids)[order]


def canonical_triangles(tris: np.ndarray, cells: np.ndarray | None = None):
    """Rotate every triangle (winding kept) so that its smallest vertex, by
    (z, y, x) and then by the cell pair, comes first; then sort the triangles.
    Returns (tris [T,9], cells [T,6] or None)."""
    t = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    n = t.shape[0]
    if n == 0:
        return t.reshape(0, 9), (None if cells is None else np.asarray(cells).reshape(0, 6))
    cc = None if cells is None else np.asarray(cells).reshape(-1, 3, 2)
    # rank the 3 vertices of each triangle
    keys = []
    for v in range(3):
        keys.append((t[:, v, 2], t[:, v, 1], t[:, v, 0]))
    best = np.zeros(n, np.int64)
    for v in (1, 2):
        z, y, x = keys[v]
        bz, by, bx = (np.choose(best, [keys[0][0], keys[1][0], keys[2][0]]),
                      np.choose(best, [keys[0][1], keys[1][1], keys[2][1]]),
                      np.choose(best, [keys[0][2], keys[1][2], keys[2][2]]))
        less = (z < bz) | ((z == bz) & ((y < by) | ((y == by) & (x < bx))))
        best = np.where(less, v, best)
    idx = (best[:, None] + np.arange(3)[None]) % 3
    t = np.take_along_axis(t, idx[:, :, None], 1)
    if cc is not None:
        cc = np.take_along_axis(cc, idx[:, :, None], 1)
    flat = t.reshape(n, 9)
    # primary key: first vertex x, then y, z, then the other vertices
    order = np.lexsort(tuple(flat[:, i] for i in range(8, -1, -1)))
    flat = flat[order]
    if cc is not None:
        cc = cc.reshape(n, 6)[order]
    return flat, cc


# ---------------------------------------------------------------------------
# Indexed face set (paper sec. 5.2): shared vertices of the fat triangles get
# one index.  A vertex is identified by the cell pair of its edge; vertices
# are numbered in order of first appearance (triangle-major, corner-minor).
# ---------------------------------------------------------------------------

def indexed_mesh(tris: np.ndarray, cells: np.ndarray):
    """(verts float32 [V,3], idx int32 [T,3]) for fat triangles tris [T,9]
    with per-corner cell pairs cells [T,6]."""
    t = np.asarray(tris, np.float32).reshape(-1, 3)
    c = np.asarray(cells, np.int64).reshape(-1, 2)
    key = (c[:, 0] << 32) | c[:, 1]
    _, first, inv = np.unique(key, return_index=True, return_inverse=True)
    # renumber unique keys by their first corner
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(len(order))
    idx = rank[inv].reshape(-1, 3).astype(np.int32)
    verts = t[np.sort(first)]
    return verts, idx


# ---------------------------------------------------------------------------
# Dual-mesh interpolant (paper sec. 5 names the dual mesh, as Moran et al.
# use it, as an interpolant for volume rendering; sec. 7 lists that as
# future work; neither defines one).
# Reading: each emitted dual is the trilinear hexahedron over its 8 vertex
# cells' centres, slot s = ex + 2 ey + 4 ez at parameter u = (ex, ey, ez),
# and carries the trilinear interpolant of their values.  A point's value
# comes from a dual whose map reaches it with u in [0,1]^3; points no dual
# reaches get NaN.  The map sends each corner of the unit cube to its slot's
# cell centre exactly, so a dual reaches the centres of its vertex cells
# (u = that corner, value = that cell's value); elsewhere Newton on the
# trilinear map (fp64) finds u.  (Newton alone cannot settle a centre where
# a degenerate dual's map is singular: there its outcome is decided by
# rounding.)  Degenerate duals whose map has no volume reach no other
# point.  Where several duals reach a
# point (on shared faces, and inside overlapping duals, which exist when
# the levels of a dual's cells span three or more), the one with the
# smallest (level, P.z, P.y, P.x) wins: the finest dual, then the lowest
# centre vertex P in (z, y, x) order.  Brute force over all duals: small
# sets only.
# ---------------------------------------------------------------------------

def _trilinear(u):
    """Weights B_s(u) [K,8] and their derivatives dB_s/du_a [K,3,8]."""
    ux, uy, uz = u[:, 0:1], u[:, 1:2], u[:, 2:3]
    s = np.arange(8)
    ex, ey, ez = (s & 1)[None], ((s >> 1) & 1)[None], (s >> 2)[None]
    fx = np.where(ex, ux, 1 - ux)
    fy = np.where(ey, uy, 1 - uy)
    fz = np.where(ez, uz, 1 - uz)
    dx = np.where(ex, 1.0, -1.0)
    dy = np.where(ey, 1.0, -1.0)
    dz = np.where(ez, 1.0, -1.0)
    w = fx * fy * fz
    dw = np.stack([dx * fy * fz, fx * dy * fz, fx * fy * dz], 1)
    return w, dw


def _invert(V, p, iters=40):
    """u [K,3] with X(u) = p for the hexahedra V [K,8,3] (Newton from the
    centre), and whether it converged."""
    u = np.full((len(V), 3), 0.5)
    ok = np.ones(len(V), bool)
    for _ in range(iters):
        w, dw = _trilinear(u)
        x = np.einsum("ks,ksa->ka", w, V)
        J = np.einsum("kbs,ksa->kab", dw, V)  # J[k, a, b] = dX_a / du_b
        r = p - x
        det = np.linalg.det(J)
        good = np.abs(det) > 1e-14
        ok &= good
        step = np.zeros_like(u)
        if good.any():
            step[good] = np.linalg.solve(J[good], r[good][:, :, None])[:, :, 0]
        u = np.clip(u + step, -0.5, 1.5)
    w, _ = _trilinear(u)
    resid = np.abs(np.einsum("ks,ksa->ka", w, V) - p).max(1)
    return u, ok & (resid < 1e-9)


def dual_mesh_sample(xyz, level, value, pl, ids, points, eps: float = 1e-9):
    """Interpolated values at points [Q,3] from the duals (pl [M,4] = centre
    vertex P and level, ids [M,8] = cell indices per slot) of the cells
    (xyz, level, value).  Returns (values float64 [Q] (NaN outside the dual
    mesh), dual index int64 [Q] (the reaching dual with the smallest
    (level, P.z, P.y, P.x), -1 if none), number of duals that reach the
    point int64 [Q])."""
    xyz = np.asarray(xyz, np.float64).reshape(-1, 3)
    lvl = np.asarray(level, np.int64)
    val = np.asarray(value, np.float64)
    pl = np.asarray(pl, np.int64).reshape(-1, 4)
    ids = np.asarray(ids, np.int64).reshape(-1, 8)
    pts = np.asarray(points, np.float64).reshape(-1, 3)
    centre = xyz + 0.5 * (1 << lvl)[:, None].astype(np.float64)
    V = centre[ids]  # [M,8,3]
    F = val[ids]     # [M,8]
    lo, hi = V.min(1) - eps, V.max(1) + eps
    out = np.full(len(pts), np.nan)
    which = np.full(len(pts), -1, np.int64)
    hits = np.zeros(len(pts), np.int64)
    corner = np.array([[s & 1, (s >> 1) & 1, s >> 2] for s in range(8)], np.float64)
    for q, p in enumerate(pts):
        cand = np.nonzero(np.all((lo <= p) & (p <= hi), 1))[0]
        if len(cand) == 0:
            continue
        u, ok = _invert(V[cand], np.broadcast_to(p, (len(cand), 3)))
        # a dual with a vertex cell centred exactly at p reaches it at that
        # slot's corner (the first such slot)
        at = np.all(V[cand] == p, axis=2)  # [K, 8]
        has = at.any(1)
        u[has] = corner[np.argmax(at[has], axis=1)]
        ok = ok | has
        inside = np.nonzero(ok & np.all((u >= -eps) & (u <= 1 + eps), 1))[0]
        hits[q] = len(inside)
        if len(inside):
            key = pl[cand[inside]]
            # smallest (level, z, y, x): lexsort takes its last key as the primary one
            k = int(inside[np.lexsort((key[:, 0], key[:, 1], key[:, 2], key[:, 3]))[0]])
            w, _ = _trilinear(np.clip(u[k:k + 1], 0.0, 1.0))
            out[q] = float(w[0] @ F[cand[k]])
            which[q] = int(cand[k])
    return out, which, hits
