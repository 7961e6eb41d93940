/*
 * amr_oracle.c -- CPU oracle for dual-mesh and iso-surface extraction from
 * AMR cells (I. Wald, "A Simple, General, and GPU Friendly Method for
 * Computing Dual Mesh and Iso-Surfaces of Adaptive Mesh Refinement (AMR)
 * Data", arXiv 2004.08475).
 *
 * TEST INFRASTRUCTURE.  This is the plain, slow, obviously correct reference
 * that the GPU library is checked against.  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg load it.  It shares no code, header,
 * table or generator with the HIP library.
 *
 * Conventions (each restated from the paper):
 *  - Cells (sec. 3.1): level 0 is finest; a level-l cell has width w = 2^l,
 *    lower corner (i,j,k) a multiple of w, and spans [lo, lo + w) per axis.
 *    Its centre is lo + w/2.
 *  - snap / cell location (sec. 3.2): the actual cell containing an integer
 *    point q.  The sorted variant sorts cells by their integer lower corner,
 *    then for every level m clears the low m bits of q (a floor, also for
 *    negative q) and binary-searches for a cell with exactly that corner and
 *    level m.  The brute-force variant scans all cells.
 *  - Dual cells (sec. 4.2-4.4): every cell generates the 8 logical level-l
 *    duals centred on its 8 corners P = lo + delta*w, delta in {0,1}^3.  The
 *    dual's vertex in slot s = ex + 2 ey + 4 ez is snap(P + (e - 1) * w).
 *    Rule 1: any vertex missing -> reject.  Rule 2: any vertex on a finer
 *    level -> reject.  Rule 3: any vertex on the same level whose lower corner
 *    precedes the generating cell's (lexicographic in z, then y, then x) ->
 *    reject.  What remains is emitted exactly once.
 *  - Iso-surface (sec. 5): every emitted dual, degenerate or not, is treated
 *    as a hexahedron with vertices at the centres of its 8 cells and fed to
 *    Marching Cubes; triangles that do not have three distinct vertices are
 *    dropped.  Vertices are identified by the unordered pair of cells at the
 *    ends of their hexahedron edge.
 *  - Marching Cubes polygonisation is computed procedurally (no stored
 *    table): on each hexahedron face the cut edges are paired so that every
 *    run of corners >= iso along the face cycle is cut off on its own; the
 *    segments chain into closed loops and each loop is fan-triangulated
 *    from its lowest-numbered edge.
 *  - Vertex placement: on a cut edge, A is the endpoint with value < iso and
 *    B the one with value >= iso; t = (iso - vA) / (vB - vA) and
 *    p = fma(t, cB - cA, cA), all in IEEE binary32.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -2, ORC_EOVERLAP = -3, ORC_ENOSPACE = -4 };

#define ORC_MAX_LEVEL 30

/* ------------------------------------------------------------------------ */
/* Cells                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const int32_t* xyz; /* [n][3] lower corners */
    const int32_t* lvl; /* [n] */
    int64_t* order;     /* cell indices sorted by lower corner (z, y, x) */
    int maxlevel;
} orc_index;

/* lexicographic order on (z, y, x) */
static int corner_cmp3(int64_t ax, int64_t ay, int64_t az, int64_t bx, int64_t by, int64_t bz) {
    if (az != bz) return az < bz ? -1 : 1;
    if (ay != by) return ay < by ? -1 : 1;
    if (ax != bx) return ax < bx ? -1 : 1;
    return 0;
}

static int cell_before(const int32_t* xyz, int64_t a, int64_t b) {
    return corner_cmp3(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], xyz[3 * b], xyz[3 * b + 1], xyz[3 * b + 2]) < 0;
}

static int sort_cmp(const void* pa, const void* pb, void* ctx) {
    const int32_t* xyz = (const int32_t*)ctx;
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    return corner_cmp3(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], xyz[3 * b], xyz[3 * b + 1], xyz[3 * b + 2]);
}

/* Field checks: level range, lower corner aligned to 2^level, finite value. */
int orc_check_fields(int64_t n, const int32_t* xyz, const int32_t* lvl, const float* val, int64_t* bad) {
    for (int64_t i = 0; i < n; ++i) {
        int l = lvl[i];
        if (l < 0 || l > ORC_MAX_LEVEL) { if (bad) *bad = i; return ORC_EINVAL; }
        int64_t w = (int64_t)1 << l;
        for (int a = 0; a < 3; ++a) {
            int64_t c = xyz[3 * i + a];
            if (((c % w) + w) % w != 0) { if (bad) *bad = i; return ORC_EINVAL; }
        }
        if (val && !isfinite(val[i])) { if (bad) *bad = i; return ORC_EINVAL; }
    }
    return ORC_OK;
}

orc_index* orc_index_new(int64_t n, const int32_t* xyz, const int32_t* lvl) {
    orc_index* ix = (orc_index*)calloc(1, sizeof(orc_index));
    if (!ix) return NULL;
    ix->n = n;
    ix->xyz = xyz;
    ix->lvl = lvl;
    ix->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!ix->order) { free(ix); return NULL; }
    ix->maxlevel = 0;
    for (int64_t i = 0; i < n; ++i) {
        ix->order[i] = i;
        if (lvl[i] > ix->maxlevel) ix->maxlevel = lvl[i];
    }
    qsort_r(ix->order, (size_t)n, sizeof(int64_t), sort_cmp, (void*)xyz);
    return ix;
}

void orc_index_free(orc_index* ix) {
    if (!ix) return;
    free(ix->order);
    free(ix);
}

/* First position in the sorted order whose corner is not below (cx,cy,cz). */
static int64_t lower_bound_corner(const orc_index* ix, int64_t cx, int64_t cy, int64_t cz) {
    int64_t lo = 0, hi = ix->n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int64_t c = ix->order[mid];
        const int32_t* p = ix->xyz + 3 * c;
        if (corner_cmp3(p[0], p[1], p[2], cx, cy, cz) < 0) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* snap, sorted variant: loop over levels, clear the low bits, binary search,
   and accept only a cell that has exactly that corner *and* that level. */
int64_t orc_locate(const orc_index* ix, int64_t qx, int64_t qy, int64_t qz) {
    for (int m = 0; m <= ix->maxlevel; ++m) {
        int64_t mask = ~(((int64_t)1 << m) - 1);
        int64_t cx = qx & mask, cy = qy & mask, cz = qz & mask;
        int64_t pos = lower_bound_corner(ix, cx, cy, cz);
        if (pos < ix->n) {
            int64_t c = ix->order[pos];
            const int32_t* p = ix->xyz + 3 * c;
            if (p[0] == cx && p[1] == cy && p[2] == cz && ix->lvl[c] == m) return c;
        }
    }
    return -1;
}

/* snap, brute-force variant: the cell whose half-open box contains q. */
int64_t orc_locate_brute(int64_t n, const int32_t* xyz, const int32_t* lvl, int64_t qx, int64_t qy, int64_t qz) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t w = (int64_t)1 << lvl[i];
        int64_t x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (x <= qx && qx < x + w && y <= qy && qy < y + w && z <= qz && qz < z + w) return i;
    }
    return -1;
}

/* Overlap check.  With ix == NULL: every pair of boxes (O(n^2)).  Otherwise:
   adjacent equal corners in the sorted order, plus, for every cell, a search at
   every level for a cell containing its lower corner (only itself may). */
int orc_check_overlap(const orc_index* ix, int64_t n, const int32_t* xyz, const int32_t* lvl, int64_t* bad) {
    if (!ix) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t wi = (int64_t)1 << lvl[i];
            for (int64_t j = i + 1; j < n; ++j) {
                int64_t wj = (int64_t)1 << lvl[j];
                int disjoint = 0;
                for (int a = 0; a < 3; ++a) {
                    int64_t ai = xyz[3 * i + a], aj = xyz[3 * j + a];
                    if (ai + wi <= aj || aj + wj <= ai) disjoint = 1;
                }
                if (!disjoint) { if (bad) *bad = i; return ORC_EOVERLAP; }
            }
        }
        return ORC_OK;
    }
    for (int64_t k = 1; k < ix->n; ++k) {
        int64_t a = ix->order[k - 1], b = ix->order[k];
        if (sort_cmp(&a, &b, (void*)xyz) == 0) { if (bad) *bad = b; return ORC_EOVERLAP; }
    }
    for (int64_t i = 0; i < n; ++i) {
        int hits = 0;
        for (int m = 0; m <= ix->maxlevel; ++m) {
            int64_t mask = ~(((int64_t)1 << m) - 1);
            int64_t cx = xyz[3 * i] & mask, cy = xyz[3 * i + 1] & mask, cz = xyz[3 * i + 2] & mask;
            int64_t pos = lower_bound_corner(ix, cx, cy, cz);
            if (pos < ix->n) {
                int64_t c = ix->order[pos];
                const int32_t* p = xyz + 3 * c;
                if (p[0] == cx && p[1] == cy && p[2] == cz && lvl[c] == m) ++hits;
            }
        }
        if (hits != 1) { if (bad) *bad = i; return ORC_EOVERLAP; }
    }
    return ORC_OK;
}

static int64_t snap(const orc_index* ix, int64_t n, const int32_t* xyz, const int32_t* lvl,
                    int64_t qx, int64_t qy, int64_t qz) {
    return ix ? orc_locate(ix, qx, qy, qz) : orc_locate_brute(n, xyz, lvl, qx, qy, qz);
}

/* ------------------------------------------------------------------------ */
/* Dual cells (rules 1-3)                                                    */
/* ------------------------------------------------------------------------ */

/* The dual centred on corner `delta` (bit 0 = x, 1 = y, 2 = z) of cell c
   (paper sec. 4.2-4.4).  Its vertex cells are the cells holding the 8
   points P + (e - 1) w around the corner P (slot s = ex + 2 ey + 4 ez).
   Cell c emits the dual when
     rule 1: every vertex exists (no hole around P),
     rule 2: no vertex is finer than c (then a finer dual covers P),
     rule 3: no vertex of c's level comes before c in (z, y, x) order of
             lower corners (that vertex generates the dual instead).
   Returns 1 and fills ids[8] (slot order) if c emits it. */
static int dual_of_cell(const orc_index* ix, int64_t n, const int32_t* xyz, const int32_t* lvl, int64_t c,
                        int delta, int64_t P[3], int64_t ids[8]) {
    const int l = lvl[c];
    const int64_t w = (int64_t)1 << l;
    const int64_t d[3] = {delta & 1, (delta >> 1) & 1, (delta >> 2) & 1};
    for (int a = 0; a < 3; ++a) P[a] = (int64_t)xyz[3 * c + a] + d[a] * w;
    int64_t v[8];
    for (int s = 0; s < 8; ++s) {
        const int64_t e[3] = {s & 1, (s >> 1) & 1, (s >> 2) & 1};
        v[s] = snap(ix, n, xyz, lvl, P[0] + (e[0] - 1) * w, P[1] + (e[1] - 1) * w, P[2] + (e[2] - 1) * w);
    }
    int all_present = 1, none_finer = 1, none_before = 1;
    for (int s = 0; s < 8; ++s) all_present = all_present && v[s] >= 0;
    if (!all_present) return 0; /* rule 1 */
    for (int s = 0; s < 8; ++s) none_finer = none_finer && lvl[v[s]] >= l;
    if (!none_finer) return 0; /* rule 2 */
    for (int s = 0; s < 8; ++s) none_before = none_before && !(lvl[v[s]] == l && cell_before(xyz, v[s], c));
    if (!none_before) return 0; /* rule 3 */
    for (int s = 0; s < 8; ++s) ids[s] = v[s];
    return 1;
}

/* Emitted duals of cells [c0, c1), in (cell, delta) order.  Writes up to cap
   records: pl[k] = (P.x, P.y, P.z, level), ids[k] = 8 cell indices.  Returns
   the total count. */
int64_t orc_dual_cells(const orc_index* ix, int64_t n, const int32_t* xyz, const int32_t* lvl, int64_t c0,
                       int64_t c1, int32_t* pl, int32_t* ids, int64_t cap) {
    int64_t count = 0;
    for (int64_t c = c0; c < c1; ++c) {
        for (int delta = 0; delta < 8; ++delta) {
            int64_t P[3], v[8];
            if (!dual_of_cell(ix, n, xyz, lvl, c, delta, P, v)) continue;
            if (count < cap) {
                if (pl) {
                    pl[4 * count + 0] = (int32_t)P[0];
                    pl[4 * count + 1] = (int32_t)P[1];
                    pl[4 * count + 2] = (int32_t)P[2];
                    pl[4 * count + 3] = lvl[c];
                }
                if (ids)
                    for (int s = 0; s < 8; ++s) ids[8 * count + s] = (int32_t)v[s];
            }
            ++count;
        }
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Marching Cubes, procedural                                                */
/* ------------------------------------------------------------------------ */

/* Hexahedron edges: slot pairs (a, b), a < b, differing in one bit.  Edges
   0-3 run along x (a = 0, 2, 4, 6), 4-7 along y (a = 0, 1, 4, 5), 8-11 along
   z (a = 0, 1, 2, 3). */
static void hex_edges(int ea[12], int eb[12]) {
    int k = 0;
    for (int axis = 0; axis < 3; ++axis)
        for (int s = 0; s < 8; ++s)
            if (!((s >> axis) & 1)) { ea[k] = s; eb[k] = s | (1 << axis); ++k; }
}

static int edge_between(int a, int b) {
    int ea[12], eb[12];
    hex_edges(ea, eb);
    for (int k = 0; k < 12; ++k)
        if ((ea[k] == a && eb[k] == b) || (ea[k] == b && eb[k] == a)) return k;
    return -1;
}

/* Corners of face (axis, side) in counter-clockwise order seen from outside. */
static void face_cycle(int axis, int side, int cyc[4]) {
    int u = (axis + 1) % 3, v = (axis + 2) % 3;
    /* (u,v) = (0,0),(1,0),(1,1),(0,1) turns counter-clockwise about e_u x e_v = +e_axis */
    int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (int i = 0; i < 4; ++i) {
        int s = (side << axis) | (uv[i][0] << u) | (uv[i][1] << v);
        cyc[side ? i : 3 - i] = s;
    }
}

/* Triangles (as hexahedron edge triples) for MC case `cs` (bit s set when the
   value at slot s is >= iso).  Returns the triangle count. */
int orc_polygonize(int cs, int8_t* out /* [16][3] */) {
    int next[12];
    for (int k = 0; k < 12; ++k) next[k] = -1;
    for (int axis = 0; axis < 3; ++axis) {
        for (int side = 0; side < 2; ++side) {
            int cyc[4], pos[4];
            face_cycle(axis, side, cyc);
            for (int i = 0; i < 4; ++i) pos[i] = (cs >> cyc[i]) & 1;
            for (int i = 0; i < 4; ++i) {
                if (!pos[i] || pos[(i + 3) % 4]) continue; /* not the start of a run */
                int j = i;
                while (pos[(j + 1) % 4]) j = (j + 1) % 4;
                int entry = edge_between(cyc[(i + 3) % 4], cyc[i]);
                int exit_ = edge_between(cyc[j], cyc[(j + 1) % 4]);
                if (next[exit_] != -1) return -1; /* cannot happen */
                next[exit_] = entry;
            }
        }
    }
    int seen[12] = {0}, nt = 0;
    for (int e = 0; e < 12; ++e) {
        if (next[e] < 0 || seen[e]) continue;
        int loop[12], k = 0, cur = e;
        while (!seen[cur]) {
            seen[cur] = 1;
            loop[k++] = cur;
            cur = next[cur];
            if (cur < 0) return -1; /* cannot happen */
        }
        for (int i = 1; i + 1 < k; ++i) {
            out[3 * nt + 0] = (int8_t)loop[0];
            out[3 * nt + 1] = (int8_t)loop[i];
            out[3 * nt + 2] = (int8_t)loop[i + 1];
            ++nt;
        }
    }
    return nt;
}

static float cell_centre(const int32_t* xyz, const int32_t* lvl, int64_t c, int axis) {
    double w = (double)((int64_t)1 << lvl[c]);
    return (float)((double)xyz[3 * c + axis] + 0.5 * w);
}

/* The surface vertex on the hexahedron edge between cells ca and cb. */
static void edge_vertex(const int32_t* xyz, const int32_t* lvl, const float* val, float iso, int64_t ca,
                        int64_t cb, float p[3], int64_t* A, int64_t* B) {
    if (val[ca] >= iso) { int64_t t = ca; ca = cb; cb = t; }
    float va = val[ca], vb = val[cb];
    float t = (iso - va) / (vb - va);
    for (int a = 0; a < 3; ++a) {
        float cA = cell_centre(xyz, lvl, ca, a), cB = cell_centre(xyz, lvl, cb, a);
        p[a] = fmaf(t, cB - cA, cA);
    }
    *A = ca;
    *B = cb;
}

/* Triangles of one emitted dual (ids in slot order).  Appends at tris[count]
   (9 floats), tri_cells[count] (3 x (A, B)), tri_dual[count] (dual_no). */
static int64_t mc_dual(const int32_t* xyz, const int32_t* lvl, const float* val, float iso, const int64_t ids[8],
                       int64_t dual_no, float* tris, int32_t* tri_cells, int64_t* tri_dual, int64_t count,
                       int64_t cap) {
    int cs = 0;
    for (int s = 0; s < 8; ++s)
        if (val[ids[s]] >= iso) cs |= 1 << s;
    if (cs == 0 || cs == 255) return count;
    int ea[12], eb[12];
    hex_edges(ea, eb);
    int8_t tri[16 * 3];
    int nt = orc_polygonize(cs, tri);
    for (int t = 0; t < nt; ++t) {
        int64_t k0[3], k1[3];
        for (int v = 0; v < 3; ++v) {
            int64_t a = ids[ea[tri[3 * t + v]]], b = ids[eb[tri[3 * t + v]]];
            k0[v] = a < b ? a : b;
            k1[v] = a < b ? b : a;
        }
        /* keep only triangles with three distinct vertices */
        if ((k0[0] == k0[1] && k1[0] == k1[1]) || (k0[1] == k0[2] && k1[1] == k1[2]) ||
            (k0[0] == k0[2] && k1[0] == k1[2]))
            continue;
        if (count < cap) {
            for (int v = 0; v < 3; ++v) {
                int64_t A, B;
                float p[3];
                edge_vertex(xyz, lvl, val, iso, k0[v], k1[v], p, &A, &B);
                if (tris)
                    for (int a = 0; a < 3; ++a) tris[9 * count + 3 * v + a] = p[a];
                if (tri_cells) {
                    tri_cells[6 * count + 2 * v + 0] = (int32_t)A;
                    tri_cells[6 * count + 2 * v + 1] = (int32_t)B;
                }
            }
            if (tri_dual) tri_dual[count] = dual_no;
        }
        ++count;
    }
    return count;
}

/* Iso-surface of the duals emitted by cells [c0, c1).  Returns the triangle
   count (writes at most cap); *n_duals receives the number of emitted duals
   (tri_dual numbers them in the same order as orc_dual_cells). */
int64_t orc_isosurface(const orc_index* ix, int64_t n, const int32_t* xyz, const int32_t* lvl, const float* val,
                       float iso, int64_t c0, int64_t c1, float* tris, int32_t* tri_cells, int64_t* tri_dual,
                       int64_t cap, int64_t* n_duals) {
    int64_t count = 0, nd = 0;
    for (int64_t c = c0; c < c1; ++c) {
        for (int delta = 0; delta < 8; ++delta) {
            int64_t P[3], v[8];
            if (!dual_of_cell(ix, n, xyz, lvl, c, delta, P, v)) continue;
            count = mc_dual(xyz, lvl, val, iso, v, nd, tris, tri_cells, tri_dual, count, cap);
            ++nd;
        }
    }
    if (n_duals) *n_duals = nd;
    return count;
}

/* Plain Marching Cubes over a regular lattice: vals[(k*ny + j)*nx + i] sits
   at (x0 + i*h, y0 + j*h, z0 + k*h).  Same polygonisation and placement as
   above; lattice point ids stand in for cell ids.  Returns the count. */
int64_t orc_grid_mc(int nx, int ny, int nz, const float* vals, double x0, double y0, double z0, double h,
                    float iso, float* tris, int32_t* tri_pts, int64_t cap) {
    int ea[12], eb[12];
    hex_edges(ea, eb);
    int64_t count = 0;
    for (int k = 0; k + 1 < nz; ++k)
        for (int j = 0; j + 1 < ny; ++j)
            for (int i = 0; i + 1 < nx; ++i) {
                int64_t id[8];
                int cs = 0;
                for (int s = 0; s < 8; ++s) {
                    id[s] = ((int64_t)(k + ((s >> 2) & 1)) * ny + (j + ((s >> 1) & 1))) * nx + (i + (s & 1));
                    if (vals[id[s]] >= iso) cs |= 1 << s;
                }
                if (cs == 0 || cs == 255) continue;
                int8_t tri[16 * 3];
                int nt = orc_polygonize(cs, tri);
                for (int t = 0; t < nt; ++t, ++count) {
                    if (count >= cap) continue;
                    for (int v = 0; v < 3; ++v) {
                        int64_t a = id[ea[tri[3 * t + v]]], b = id[eb[tri[3 * t + v]]];
                        if (vals[a] >= iso) { int64_t tmp = a; a = b; b = tmp; }
                        float va = vals[a], vb = vals[b];
                        float tt = (iso - va) / (vb - va);
                        int64_t pa[3] = {a % nx, (a / nx) % ny, a / ((int64_t)nx * ny)};
                        int64_t pb[3] = {b % nx, (b / nx) % ny, b / ((int64_t)nx * ny)};
                        double o[3] = {x0, y0, z0};
                        for (int ax = 0; ax < 3; ++ax) {
                            float cA = (float)(o[ax] + (double)pa[ax] * h);
                            float cB = (float)(o[ax] + (double)pb[ax] * h);
                            if (tris) tris[9 * count + 3 * v + ax] = fmaf(tt, cB - cA, cA);
                        }
                        if (tri_pts) {
                            tri_pts[6 * count + 2 * v] = (int32_t)a;
                            tri_pts[6 * count + 2 * v + 1] = (int32_t)b;
                        }
                    }
                }
            }
    return count;
}
