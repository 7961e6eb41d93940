// amriso.hip -- HIP implementation of libamriso.so for gfx950 (MI355X).
//
// Dual-mesh and crack-free iso-surface extraction from AMR cells, after
// I. Wald, "A Simple, General, and GPU Friendly Method for Computing Dual
// Mesh and Iso-Surfaces of Adaptive Mesh Refinement (AMR) Data",
// arXiv 2004.08475.  The C ABI is declared in include/amriso.h.
//
// Data layout in HBM
//   input (caller, borrowed): SoA  xyz int32[n][3], level int32[n], value f32[n]
//   index workspace (caller): [records | cell ids | group list | tile states]
//     record (64 B, one per hash slot): val f32[8] | key u64 | pad
//       A record holds the cells of one level that share a 2x2x2 sibling
//       block (a "group"): key = (level, block coordinates), val[c] = value
//       of child c (c = bx + 2 by + 4 bz), NaN where that child is not an
//       actual cell of this level.  One probe thus returns up to 8 cells.
//     cell ids  int32[slots][8]: input index of child c of the slot's group
//     group list int32[]: slots of all occupied records (work list)
//     tile states u64[2][tiles + 1]: decoupled look-back of the extraction
//
// Extraction kernel (paper sec. 4.2-5): one work-group processes 32 groups,
// eight lanes per group.  The lanes first fetch the 27 neighbouring groups
// of their group (same level; absent ones are resolved to the coarser cell
// covering them) into LDS, then evaluate the 27 corners of the group's 2x2x2
// cell block.  A corner's logical dual is emitted when its 8 slots are all
// covered by cells of this level or coarser and the lowest-numbered slot on
// this level belongs to this group -- rules 1-3 of the paper, with the
// "precedes" order of rule 3 read as slot order (= lexicographic (z,y,x)
// order of the lower corners of same-level cells).  Marching Cubes runs on
// each emitted dual from a 256-entry table kept in LDS; degenerate triangles
// are culled by comparing cell references; counts are prefix-summed within
// the work-group and across work-groups by decoupled look-back, so output
// positions are deterministic and no count pass is needed.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "amriso.h"
#include "mc_table.inc"

namespace {

constexpr int kMaxLevel = 20;
constexpr int kCoordLimit = 1 << 23;    // |corner| bound: centres exact in f32
constexpr int kSpanLimit = 1 << 20;     // offset coordinates u < 2^20
constexpr uint64_t kEmpty = ~0ull;
constexpr int kGroupsPerTile = 32;
constexpr int kBlock = 256;             // 32 groups x 8 lanes
constexpr uint32_t kMaxCap = 1u << 28;  // slot * 8 + child fits int32
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

enum : uint32_t { kErrLevel = 1, kErrAlign = 2, kErrValue = 4, kErrCoord = 8 };

struct alignas(64) Record {
    float val[8];
    uint64_t key;
    uint32_t pad[6];
};
static_assert(sizeof(Record) == 64, "record is one 64-byte line");

// Device control block, one per set (library-allocated).
struct Ctrl {
    int32_t lo[3];
    int32_t hi[3];
    int32_t lmin, lmax;
    uint32_t err;
    uint32_t pad0;
    unsigned long long bad;
    unsigned long long level_count[32];
    // index build
    uint32_t n_groups;
    uint32_t overflow;
    uint32_t dup;
    uint32_t overlap;
    unsigned long long bad_build;
};

__device__ __forceinline__ uint64_t group_key(int m, uint32_t gx, uint32_t gy, uint32_t gz) {
    return ((uint64_t)m << 57) | ((uint64_t)gz << 38) | ((uint64_t)gy << 19) | (uint64_t)gx;
}

__device__ __forceinline__ uint32_t slot_of(uint64_t key, int shift) {
    return (uint32_t)((key * kGolden) >> shift);
}

__device__ __forceinline__ float nan_marker() { return __int_as_float(0x7fc00000); }

// Linear probe for `key`; returns the slot or -1.  At most cap steps.
__device__ __forceinline__ int probe(const Record* __restrict__ rec, uint64_t key, int shift, uint32_t mask) {
    uint32_t h = slot_of(key, shift);
    for (uint32_t i = 0; i <= mask; ++i) {
        uint64_t k = rec[h].key;
        if (k == key) return (int)h;
        if (k == kEmpty) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Upload: validation and reductions
// ---------------------------------------------------------------------------

__global__ void k_ctrl_reset(Ctrl* c) {
    int t = threadIdx.x;
    if (t < 3) {
        c->lo[t] = INT32_MAX;
        c->hi[t] = INT32_MIN;
    }
    if (t == 0) {
        c->lmin = INT32_MAX;
        c->lmax = INT32_MIN;
        c->err = 0;
        c->bad = ~0ull;
        c->n_groups = 0;
        c->overflow = 0;
        c->dup = 0;
        c->overlap = 0;
        c->bad_build = ~0ull;
    }
    if (t < 32) c->level_count[t] = 0;
}

__global__ __launch_bounds__(256) void k_upload(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                const float* __restrict__ val, int64_t n, Ctrl* c) {
    __shared__ int s_lo[3], s_hi[3], s_lmin, s_lmax;
    __shared__ unsigned long long s_cnt[kMaxLevel + 1];
    int t = threadIdx.x;
    if (t < 3) {
        s_lo[t] = INT32_MAX;
        s_hi[t] = INT32_MIN;
    }
    if (t == 0) {
        s_lmin = INT32_MAX;
        s_lmax = INT32_MIN;
    }
    if (t <= kMaxLevel) s_cnt[t] = 0;
    __syncthreads();
    int lo0 = INT32_MAX, lo1 = INT32_MAX, lo2 = INT32_MAX, hi0 = INT32_MIN, hi1 = INT32_MIN, hi2 = INT32_MIN;
    int lmin = INT32_MAX, lmax = INT32_MIN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + t; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        int l = lvl[i];
        float v = val[i];
        uint32_t bad = 0;
        if (l < 0 || l > kMaxLevel) {
            bad |= kErrLevel;
        } else {
            int w = 1 << l;
            if ((x | y | z) & (w - 1)) bad |= kErrAlign;
            int64_t mn = x < y ? (x < z ? x : z) : (y < z ? y : z);
            int64_t mx = x > y ? (x > z ? x : z) : (y > z ? y : z);
            if (mn < -(int64_t)kCoordLimit || mx + w > (int64_t)kCoordLimit) bad |= kErrCoord;
        }
        if (!isfinite(v)) bad |= kErrValue;
        if (bad) {
            atomicOr(&c->err, bad);
            atomicMin(&c->bad, (unsigned long long)i);
            continue;
        }
        int w = 1 << l;
        lo0 = min(lo0, x);
        lo1 = min(lo1, y);
        lo2 = min(lo2, z);
        hi0 = max(hi0, x + w);
        hi1 = max(hi1, y + w);
        hi2 = max(hi2, z + w);
        lmin = min(lmin, l);
        lmax = max(lmax, l);
        atomicAdd(&s_cnt[l], 1ull);
    }
    atomicMin(&s_lo[0], lo0);
    atomicMin(&s_lo[1], lo1);
    atomicMin(&s_lo[2], lo2);
    atomicMax(&s_hi[0], hi0);
    atomicMax(&s_hi[1], hi1);
    atomicMax(&s_hi[2], hi2);
    atomicMin(&s_lmin, lmin);
    atomicMax(&s_lmax, lmax);
    __syncthreads();
    if (t < 3) {
        atomicMin(&c->lo[t], s_lo[t]);
        atomicMax(&c->hi[t], s_hi[t]);
    }
    if (t == 0) {
        atomicMin(&c->lmin, s_lmin);
        atomicMax(&c->lmax, s_lmax);
    }
    if (t <= kMaxLevel && s_cnt[t]) atomicAdd(&c->level_count[t], s_cnt[t]);
}

// ---------------------------------------------------------------------------
// Index build
// ---------------------------------------------------------------------------

struct Geo {
    int32_t ox, oy, oz;  // origin: u = x - ox >= 2^(lmax+1)
    int lmax;
    int shift;           // 64 - log2(cap)
    uint32_t mask;       // cap - 1
};

__global__ __launch_bounds__(256) void k_index_init(Record* __restrict__ rec, int32_t* __restrict__ ids, uint32_t cap) {
    float nanv = nan_marker();
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x) {
        Record r;
        for (int c = 0; c < 8; ++c) r.val[c] = nanv;
        r.key = kEmpty;
        for (int c = 0; c < 6; ++c) r.pad[c] = 0;
        rec[i] = r;
        int4* p = reinterpret_cast<int4*>(ids + (size_t)i * 8);
        p[0] = make_int4(-1, -1, -1, -1);
        p[1] = make_int4(-1, -1, -1, -1);
    }
}

__global__ __launch_bounds__(256) void k_index_insert(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                      const float* __restrict__ val, int64_t n, Geo g,
                                                      Record* __restrict__ rec, int32_t* __restrict__ ids,
                                                      int32_t* __restrict__ glist, uint32_t glist_cap, Ctrl* c) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int m = lvl[i];
        uint32_t ux = (uint32_t)(xyz[3 * i] - g.ox), uy = (uint32_t)(xyz[3 * i + 1] - g.oy),
                 uz = (uint32_t)(xyz[3 * i + 2] - g.oz);
        uint64_t key = group_key(m, ux >> (m + 1), uy >> (m + 1), uz >> (m + 1));
        int child = ((ux >> m) & 1) | (((uy >> m) & 1) << 1) | (((uz >> m) & 1) << 2);
        uint32_t h = slot_of(key, g.shift);
        int slot = -1;
        for (uint32_t step = 0; step <= g.mask; ++step) {
            uint64_t k = __hip_atomic_load(&rec[h].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (k == key) {
                slot = (int)h;
                break;
            }
            if (k == kEmpty) {
                uint64_t prev = atomicCAS((unsigned long long*)&rec[h].key, (unsigned long long)kEmpty,
                                          (unsigned long long)key);
                if (prev == kEmpty) {
                    uint32_t pos = atomicAdd(&c->n_groups, 1u);
                    if (pos < glist_cap) glist[pos] = (int32_t)h;
                    else atomicOr(&c->overflow, 1u);
                    slot = (int)h;
                    break;
                }
                if (prev == key) {
                    slot = (int)h;
                    break;
                }
            }
            if (__hip_atomic_load(&c->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            h = (h + 1) & g.mask;
        }
        if (slot < 0) {
            atomicOr(&c->overflow, 1u);
            continue;
        }
        rec[slot].val[child] = val[i];
        int old = atomicExch(&ids[(size_t)slot * 8 + child], (int)i);
        if (old != -1) {
            atomicOr(&c->dup, 1u);
            atomicMin(&c->bad_build, (unsigned long long)i);
        }
    }
}

// Nested cells: a cell of level m' > l containing the lower corner of a
// level-l cell.  (Equal corners on one level were caught as duplicates.)
__global__ __launch_bounds__(256) void k_index_overlap(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                       int64_t n, Geo g, const Record* __restrict__ rec, Ctrl* c) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int l = lvl[i];
        uint32_t ux = (uint32_t)(xyz[3 * i] - g.ox), uy = (uint32_t)(xyz[3 * i + 1] - g.oy),
                 uz = (uint32_t)(xyz[3 * i + 2] - g.oz);
        for (int m = l + 1; m <= g.lmax; ++m) {
            int h = probe(rec, group_key(m, ux >> (m + 1), uy >> (m + 1), uz >> (m + 1)), g.shift, g.mask);
            if (h < 0) continue;
            int child = ((ux >> m) & 1) | (((uy >> m) & 1) << 1) | (((uz >> m) & 1) << 2);
            float v = rec[h].val[child];
            if (v == v) {
                atomicOr(&c->overlap, 1u);
                atomicMin(&c->bad_build, (unsigned long long)i);
            }
            break;  // a present group at level m decides: no coarser cell can contain the corner
        }
    }
}

// ---------------------------------------------------------------------------
// Extraction
// ---------------------------------------------------------------------------

struct ExtractArgs {
    const Record* rec;
    const int32_t* ids;
    const int32_t* glist;
    uint32_t n_groups;
    Geo g;
    float iso;
    // iso-surface outputs
    float* tris;
    int32_t* tri_cells;
    int32_t* tri_dual;
    // dual-cell outputs
    int32_t* corner_level;
    int32_t* verts;
    int64_t cap;
    int64_t* counts;
    unsigned long long* st_t;  // per tile: flag | call parity | triangles
    unsigned long long* st_d;  // per tile: flag | call parity | duals
    struct Sched* sched;
    uint32_t n_tiles;
};

// Look-back state word: flag (2 bits) | parity of the call (1 bit) | value.
// Every call rewrites the state of every tile, so a word left by the
// previous call is recognised by its parity and read as "not yet written";
// the states therefore need no clearing between calls.  Tickets and the
// done-counter grow monotonically; the call number is read at kernel start
// and advanced by the tile that finishes last.
constexpr unsigned long long kFlagShift = 62;
constexpr unsigned long long kParityBit = 1ull << 61;
constexpr unsigned long long kValMask = kParityBit - 1;
constexpr unsigned long long kFlagAgg = 1, kFlagIncl = 2;

struct Sched {
    unsigned long long ticket;  // tiles started, over all calls
    unsigned long long done;    // tiles finished, over all calls
    unsigned long long call;    // calls completed
    unsigned long long pad;
};

__global__ void k_sched_reset(Sched* sc, unsigned long long* st_t, unsigned long long* st_d, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        st_t[i] = 0;
        st_d[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->ticket = 0;
        sc->done = 0;
        sc->call = 0;
        sc->pad = 0;
    }
}

__global__ void k_counts_zero(int64_t* counts) {
    if (threadIdx.x == 0 && counts) {
        counts[0] = 0;
        counts[1] = 0;
    }
}

// hexahedron edge e -> lower slot a (upper slot b = a | (1 << axis))
__device__ __forceinline__ int edge_lo(int e) {
    // edges 0-3 along x: a = 0,2,4,6; 4-7 along y: a = 0,1,4,5; 8-11 along z: a = 0,1,2,3
    constexpr uint64_t kLo = 0x3210541064200ull;  // nibble e = lower slot
    return (int)((kLo >> (4 * e)) & 0xF);
}
__device__ __forceinline__ int edge_hi(int e) { return edge_lo(e) | (1 << (e >> 2)); }

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long x) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

__device__ __forceinline__ unsigned long long ld_acq(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool kDuals>
__global__ __launch_bounds__(kBlock) void k_extract(ExtractArgs a) {
    __shared__ float s_val[kGroupsPerTile][27][8];
    __shared__ int32_t s_ref[kGroupsPerTile][27];
    __shared__ int8_t s_lvl[kGroupsPerTile][27];
    __shared__ unsigned long long s_tab[256];
    __shared__ unsigned long long s_wave[kBlock / 64];
    __shared__ unsigned long long s_pre_t, s_pre_d;
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_call;

    const int t = threadIdx.x;
    const int gi = t >> 3;  // group within the tile
    const int j = t & 7;    // lane within the group
    if (t == 0) {
        unsigned long long call = __hip_atomic_load(&a.sched->call, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long tk = atomicAdd(&a.sched->ticket, 1ull);
        s_call = call;
        s_tile = (uint32_t)(tk - call * a.n_tiles);
    }
    if (!kDuals) s_tab[t] = kMcTable[t];
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t gidx = tile * kGroupsPerTile + gi;
    const bool valid = gidx < a.n_groups;
    const Geo g = a.g;

    int m = 0;
    uint32_t gx = 0, gy = 0, gz = 0;
    int own = 0;
    if (valid) {
        own = a.glist[gidx];
        uint64_t key = a.rec[own].key;
        m = (int)(key >> 57);
        gx = (uint32_t)(key & 0x7FFFF);
        gy = (uint32_t)((key >> 19) & 0x7FFFF);
        gz = (uint32_t)((key >> 38) & 0x7FFFF);
    }

    // ---- phase 1: the 27 neighbouring groups of this group, into LDS ----
    if (valid) {
        for (int dd = j; dd < 27; dd += 8) {
            int dx = dd % 3 - 1, dy = (dd / 3) % 3 - 1, dz = dd / 9 - 1;
            int lv = -1, ref = -1;
            float v8[8];
            int h = own;
            if (dd != 13) h = probe(a.rec, group_key(m, gx + dx, gy + dy, gz + dz), g.shift, g.mask);
            if (h >= 0) {
                const float4* pv = reinterpret_cast<const float4*>(a.rec[h].val);
                float4 p0 = pv[0], p1 = pv[1];
                v8[0] = p0.x; v8[1] = p0.y; v8[2] = p0.z; v8[3] = p0.w;
                v8[4] = p1.x; v8[5] = p1.y; v8[6] = p1.z; v8[7] = p1.w;
                lv = m;
                ref = h;
            } else {
                // no cell of level m in this block: find the coarser cell that
                // covers the whole level-(m+1) block, if any
                uint32_t bx = gx + dx, by = gy + dy, bz = gz + dz;
                for (int L = m + 1; L <= g.lmax; ++L) {
                    int sh = L - m - 1;
                    uint32_t cx = bx >> sh, cy = by >> sh, cz = bz >> sh;
                    int h2 = probe(a.rec, group_key(L, cx >> 1, cy >> 1, cz >> 1), g.shift, g.mask);
                    if (h2 < 0) continue;
                    int child = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
                    float v = a.rec[h2].val[child];
                    if (v == v) {
                        lv = L;
                        ref = h2 * 8 + child;
                        v8[0] = v;
                    }
                    break;
                }
            }
            if (lv == m) {
                for (int c = 0; c < 8; ++c) s_val[gi][dd][c] = v8[c];
            } else if (lv > m) {
                s_val[gi][dd][0] = v8[0];
            }
            s_ref[gi][dd] = ref;
            s_lvl[gi][dd] = (int8_t)lv;
        }
    }
    __syncthreads();

    // ---- phase 2: the 27 corners of the group's 2x2x2 block ----
    const float iso = a.iso;
    uint32_t items[4];  // bit 31 valid | corner k (5 b) << 20 | case << 8 | keep mask (5 b)
    int n_dual = 0, n_tri = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        items[q] = 0;
        int k = j + 8 * q;
        if (!valid || k >= 27) continue;
        int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
        int refs[8];
        float vals[8];
        bool ok = true, owner_seen = false;
        for (int s = 0; s < 8 && ok; ++s) {
            int rx = kx + (s & 1) - 1, ry = ky + ((s >> 1) & 1) - 1, rz = kz + ((s >> 2) & 1) - 1;
            int dd = ((rx + 2) >> 1) + 3 * ((ry + 2) >> 1) + 9 * ((rz + 2) >> 1);
            int lv = s_lvl[gi][dd];
            if (lv < 0) {
                ok = false;  // rule 1 (hole) or rule 2 (finer cells)
                break;
            }
            if (lv == m) {
                int child = (rx & 1) | ((ry & 1) << 1) | ((rz & 1) << 2);
                float v = s_val[gi][dd][child];
                if (v != v) {
                    ok = false;  // not a cell of this level: finer or hole
                    break;
                }
                if (!owner_seen) {
                    owner_seen = true;
                    if (dd != 13) ok = false;  // rule 3: a preceding same-level cell owns it
                }
                vals[s] = v;
                refs[s] = s_ref[gi][dd] * 8 + child;
            } else {
                vals[s] = s_val[gi][dd][0];
                refs[s] = s_ref[gi][dd];
            }
        }
        if (!ok || !owner_seen) continue;
        ++n_dual;
        uint32_t cs = 0, keep = 0;
        if (!kDuals) {
            for (int s = 0; s < 8; ++s) cs |= (vals[s] >= iso ? 1u : 0u) << s;
            unsigned long long e = s_tab[cs];
            int nt = (int)(e >> 60);
            for (int tt = 0; tt < nt; ++tt) {
                int ea = (int)((e >> (12 * tt)) & 0xF), eb = (int)((e >> (12 * tt + 4)) & 0xF),
                    ec = (int)((e >> (12 * tt + 8)) & 0xF);
                int a0 = refs[edge_lo(ea)], a1 = refs[edge_hi(ea)];
                int b0 = refs[edge_lo(eb)], b1 = refs[edge_hi(eb)];
                int c0 = refs[edge_lo(ec)], c1 = refs[edge_hi(ec)];
                bool ab = (a0 == b0 && a1 == b1) || (a0 == b1 && a1 == b0);
                bool bc = (b0 == c0 && b1 == c1) || (b0 == c1 && b1 == c0);
                bool ac = (a0 == c0 && a1 == c1) || (a0 == c1 && a1 == c0);
                if (!(ab || bc || ac)) {
                    keep |= 1u << tt;
                    ++n_tri;
                }
            }
        }
        items[q] = 0x80000000u | ((uint32_t)k << 20) | (cs << 8) | keep;
    }

    // ---- block scan of (triangles, duals) ----
    unsigned long long mine = ((unsigned long long)n_tri << 32) | (unsigned long long)n_dual;
    unsigned long long incl = wave_incl_scan(mine);
    const int wave = t >> 6;
    if ((t & 63) == 63) s_wave[wave] = incl;
    __syncthreads();
    unsigned long long wave_pre = 0, total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) wave_pre += s_wave[w];
        total += s_wave[w];
    }
    unsigned long long excl = wave_pre + incl - mine;

    // ---- decoupled look-back across tiles ----
    if (t == 0) {
        const unsigned long long par = (s_call & 1) ? kParityBit : 0ull;
        unsigned long long agg_t = total >> 32, agg_d = total & 0xFFFFFFFFull;
        unsigned long long pre_t = 0, pre_d = 0;
        if (tile == 0) {
            st_rel(&a.st_d[0], (kFlagIncl << kFlagShift) | par | agg_d);
            st_rel(&a.st_t[0], (kFlagIncl << kFlagShift) | par | agg_t);
        } else {
            st_rel(&a.st_d[tile], (kFlagAgg << kFlagShift) | par | agg_d);
            st_rel(&a.st_t[tile], (kFlagAgg << kFlagShift) | par | agg_t);
            int p = (int)tile - 1;
            while (true) {
                unsigned long long wt = ld_acq(&a.st_t[p]);
                unsigned long long wd = ld_acq(&a.st_d[p]);
                unsigned long long ft = wt >> kFlagShift, fd = wd >> kFlagShift;
                if (ft == 0 || ft != fd || (wt & kParityBit) != par || (wd & kParityBit) != par) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                pre_t += wt & kValMask;
                pre_d += wd & kValMask;
                if (ft == kFlagIncl) break;
                --p;
            }
            st_rel(&a.st_d[tile], (kFlagIncl << kFlagShift) | par | (pre_d + agg_d));
            st_rel(&a.st_t[tile], (kFlagIncl << kFlagShift) | par | (pre_t + agg_t));
        }
        s_pre_t = pre_t;
        s_pre_d = pre_d;
        if (tile == a.n_tiles - 1 && a.counts) {
            a.counts[0] = kDuals ? (int64_t)(pre_d + agg_d) : (int64_t)(pre_t + agg_t);
            a.counts[1] = (int64_t)(pre_d + agg_d);
        }
    }
    __syncthreads();

    // ---- phase 3: write ----
    int64_t out_t = (int64_t)s_pre_t + (int64_t)(excl >> 32);
    int64_t out_d = (int64_t)s_pre_d + (int64_t)(excl & 0xFFFFFFFFull);
    for (int q = 0; q < 4; ++q) {
        uint32_t it = items[q];
        if (!(it & 0x80000000u)) continue;
        int k = (it >> 20) & 31;
        int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
        int refs[8], lvs[8];
        float vals[8];
        for (int s = 0; s < 8; ++s) {
            int rx = kx + (s & 1) - 1, ry = ky + ((s >> 1) & 1) - 1, rz = kz + ((s >> 2) & 1) - 1;
            int dd = ((rx + 2) >> 1) + 3 * ((ry + 2) >> 1) + 9 * ((rz + 2) >> 1);
            int lv = s_lvl[gi][dd];
            if (lv == m) {
                int child = (rx & 1) | ((ry & 1) << 1) | ((rz & 1) << 2);
                vals[s] = s_val[gi][dd][child];
                refs[s] = s_ref[gi][dd] * 8 + child;
            } else {
                vals[s] = s_val[gi][dd][0];
                refs[s] = s_ref[gi][dd];
            }
            lvs[s] = lv;
        }
        if (kDuals) {
            if (out_d < a.cap) {
                if (a.corner_level) {
                    int4 pl;
                    pl.x = (int)(((2 * gx + kx) << m)) + g.ox;
                    pl.y = (int)(((2 * gy + ky) << m)) + g.oy;
                    pl.z = (int)(((2 * gz + kz) << m)) + g.oz;
                    pl.w = m;
                    reinterpret_cast<int4*>(a.corner_level)[out_d] = pl;
                }
                if (a.verts) {
                    int4 v0, v1;
                    v0.x = a.ids[refs[0]]; v0.y = a.ids[refs[1]]; v0.z = a.ids[refs[2]]; v0.w = a.ids[refs[3]];
                    v1.x = a.ids[refs[4]]; v1.y = a.ids[refs[5]]; v1.z = a.ids[refs[6]]; v1.w = a.ids[refs[7]];
                    reinterpret_cast<int4*>(a.verts)[2 * out_d] = v0;
                    reinterpret_cast<int4*>(a.verts)[2 * out_d + 1] = v1;
                }
            }
            ++out_d;
            continue;
        }
        uint32_t cs = (it >> 8) & 0xFF, keep = it & 0x1F;
        unsigned long long e = s_tab[cs];
        int nt = (int)(e >> 60);
        for (int tt = 0; tt < nt; ++tt) {
            if (!((keep >> tt) & 1)) continue;
            if (out_t < a.cap) {
                float p[9];
                int cells[6];
                for (int v = 0; v < 3; ++v) {
                    int ed = (int)((e >> (12 * tt + 4 * v)) & 0xF);
                    int sa = edge_lo(ed), sb = edge_hi(ed);
                    if (vals[sa] >= iso) {
                        int tmp = sa;
                        sa = sb;
                        sb = tmp;
                    }
                    float va = vals[sa], vb = vals[sb];
                    float tp = (iso - va) / (vb - va);
                    int ra[3] = {kx + (sa & 1) - 1, ky + ((sa >> 1) & 1) - 1, kz + ((sa >> 2) & 1) - 1};
                    int rb[3] = {kx + (sb & 1) - 1, ky + ((sb >> 1) & 1) - 1, kz + ((sb >> 2) & 1) - 1};
                    uint32_t gg[3] = {gx, gy, gz};
                    int oo[3] = {g.ox, g.oy, g.oz};
                    for (int ax = 0; ax < 3; ++ax) {
                        // finest-unit offset coordinate of the slot position, floored to the cell's level
                        uint32_t pa = ((2 * gg[ax] + (uint32_t)ra[ax]) << m) & ~((1u << lvs[sa]) - 1u);
                        uint32_t pb = ((2 * gg[ax] + (uint32_t)rb[ax]) << m) & ~((1u << lvs[sb]) - 1u);
                        float ca = (float)((int)pa + oo[ax]) + 0.5f * (float)(1 << lvs[sa]);
                        float cb = (float)((int)pb + oo[ax]) + 0.5f * (float)(1 << lvs[sb]);
                        p[3 * v + ax] = fmaf(tp, cb - ca, ca);
                    }
                    cells[2 * v] = refs[sa];
                    cells[2 * v + 1] = refs[sb];
                }
                if (a.tris) {
                    float* o = a.tris + 9 * out_t;
                    for (int c = 0; c < 9; ++c) o[c] = p[c];
                }
                if (a.tri_cells) {
                    int32_t* o = a.tri_cells + 6 * out_t;
                    for (int c = 0; c < 6; ++c) o[c] = a.ids[cells[c]];
                }
                if (a.tri_dual) a.tri_dual[out_t] = (int32_t)out_d;
            }
            ++out_t;
        }
        ++out_d;
    }

    // ---- the tile that finishes last advances the call number ----
    __syncthreads();
    if (t == 0) {
        unsigned long long d = atomicAdd(&a.sched->done, 1ull) + 1;
        if (d == (s_call + 1) * (unsigned long long)a.n_tiles)
            __hip_atomic_store(&a.sched->call, s_call + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hipfail(hipError_t e, const char* what) {
    return fail(AMR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct amr_set {
    int device = 0;
    Ctrl* ctrl = nullptr;     // device
    Ctrl host_ctrl{};
    // upload
    const int32_t* xyz = nullptr;
    const int32_t* lvl = nullptr;
    const float* val = nullptr;
    int64_t n = 0;
    bool uploaded = false;
    int lmin = 0, lmax = 0;
    int32_t origin[3] = {0, 0, 0};
    uint64_t level_count[kMaxLevel + 1] = {};
    uint64_t group_hint = 0;
    // index
    bool built = false;
    uint32_t cap = 0;
    int shift = 0;
    uint32_t n_groups = 0;
    Record* rec = nullptr;
    int32_t* ids = nullptr;
    int32_t* glist = nullptr;
    unsigned long long* st_t = nullptr;
    unsigned long long* st_d = nullptr;
    Sched* sched = nullptr;
    uint32_t max_tiles = 0;
};

namespace {

uint32_t table_cap(const amr_set* s) {
    uint64_t want = s->group_hint * 2;
    if (want < 1024) want = 1024;
    uint64_t cap = 1;
    while (cap < want) cap <<= 1;
    return cap > kMaxCap ? 0 : (uint32_t)cap;
}

struct Layout {
    size_t rec, ids, glist, st_t, st_d, sched, total;
    uint32_t max_tiles;
};

Layout layout_for(uint32_t cap) {
    Layout L{};
    uint32_t max_groups = cap / 2;
    L.max_tiles = (max_groups + kGroupsPerTile - 1) / kGroupsPerTile + 1;
    size_t off = 0;
    L.rec = off;
    off = align256(off + (size_t)cap * sizeof(Record));
    L.ids = off;
    off = align256(off + (size_t)cap * 8 * sizeof(int32_t));
    L.glist = off;
    off = align256(off + (size_t)max_groups * sizeof(int32_t));
    L.st_t = off;
    off = align256(off + (size_t)L.max_tiles * 8);
    L.st_d = off;
    off = align256(off + (size_t)L.max_tiles * 8);
    L.sched = off;
    off = align256(off + sizeof(Sched));
    L.total = off;
    return L;
}

Geo geo_of(const amr_set* s) {
    Geo g;
    g.ox = s->origin[0];
    g.oy = s->origin[1];
    g.oz = s->origin[2];
    g.lmax = s->lmax;
    int log2cap = 0;
    while ((1u << log2cap) < s->cap) ++log2cap;
    g.shift = 64 - log2cap;
    g.mask = s->cap - 1;
    return g;
}

int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (int)g;
}

int launch_extract(amr_set* s, bool duals, float iso, float* tris, int32_t* tri_cells, int32_t* tri_dual,
                   int32_t* corner_level, int32_t* verts, int64_t cap, int64_t* counts, hipStream_t stream) {
    uint32_t n_tiles = (s->n_groups + kGroupsPerTile - 1) / kGroupsPerTile;
    if (n_tiles == 0) {
        hipLaunchKernelGGL(k_counts_zero, dim3(1), dim3(64), 0, stream, counts);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? AMR_OK : hipfail(e, "extract (empty set)");
    }
    ExtractArgs a;
    a.rec = s->rec;
    a.ids = s->ids;
    a.glist = s->glist;
    a.n_groups = s->n_groups;
    a.g = geo_of(s);
    a.iso = iso;
    a.tris = tris;
    a.tri_cells = tri_cells;
    a.tri_dual = tri_dual;
    a.corner_level = corner_level;
    a.verts = verts;
    a.cap = cap;
    a.counts = counts;
    a.st_t = s->st_t;
    a.st_d = s->st_d;
    a.sched = s->sched;
    a.n_tiles = n_tiles;
    if (duals)
        hipLaunchKernelGGL(k_extract<true>, dim3(n_tiles), dim3(kBlock), 0, stream, a);
    else
        hipLaunchKernelGGL(k_extract<false>, dim3(n_tiles), dim3(kBlock), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AMR_OK : hipfail(e, "extract launch");
}

}  // namespace

extern "C" {

int amr_create(amr_set** out, int hip_device) {
    if (!out) return fail(AMR_EINVAL, "amr_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
        return fail(AMR_EINVAL, "amr_create: no HIP device %d", hip_device);
    DeviceGuard dg(hip_device);
    if (!dg.ok) return fail(AMR_EHIP, "amr_create: cannot select device %d", hip_device);
    amr_set* s = new (std::nothrow) amr_set();
    if (!s) return fail(AMR_ENOMEM, "amr_create: out of host memory");
    s->device = hip_device;
    hipError_t e = hipMalloc((void**)&s->ctrl, sizeof(Ctrl));
    if (e != hipSuccess) {
        delete s;
        return hipfail(e, "amr_create: control block");
    }
    *out = s;
    g_err[0] = 0;
    return AMR_OK;
}

void amr_destroy(amr_set* s) {
    if (!s) return;
    {
        DeviceGuard dg(s->device);
        if (s->ctrl) (void)hipFree(s->ctrl);
    }
    delete s;
}

int amr_upload(amr_set* s, const int32_t* xyz, const int32_t* level, const float* value, int64_t n,
               hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_upload: set is NULL");
    if (n < 0) return fail(AMR_EINVAL, "amr_upload: negative n");
    if (n > 0 && (!xyz || !level || !value)) return fail(AMR_EINVAL, "amr_upload: NULL array");
    if (n >= (int64_t)1 << 31) return fail(AMR_ERANGE, "amr_upload: more than 2^31-1 cells");
    DeviceGuard dg(s->device);
    s->uploaded = false;
    s->built = false;
    s->xyz = xyz;
    s->lvl = level;
    s->val = value;
    s->n = n;
    for (int l = 0; l <= kMaxLevel; ++l) s->level_count[l] = 0;
    s->lmin = s->lmax = 0;
    s->origin[0] = s->origin[1] = s->origin[2] = 0;
    s->group_hint = 0;
    if (n == 0) {
        s->uploaded = true;
        return AMR_OK;
    }
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, stream, s->ctrl);
    hipLaunchKernelGGL(k_upload, dim3(grid_for(n, 256)), dim3(256), 0, stream, xyz, level, value, n, s->ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_upload: launch");
    e = hipMemcpyAsync(&s->host_ctrl, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hipfail(e, "amr_upload: readback");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "amr_upload: synchronize");
    const Ctrl& c = s->host_ctrl;
    if (c.err) {
        const char* why = (c.err & kErrLevel)   ? "level outside [0, 20]"
                          : (c.err & kErrAlign) ? "lower corner not a multiple of 2^level"
                          : (c.err & kErrValue) ? "non-finite value"
                                                : "coordinate outside [-2^23, 2^23]";
        int code = (c.err & (kErrLevel | kErrAlign | kErrValue)) ? AMR_EINVAL : AMR_ERANGE;
        return fail(code, "amr_upload: cell %llu: %s", (unsigned long long)c.bad, why);
    }
    s->lmin = c.lmin;
    s->lmax = c.lmax;
    int64_t blk = (int64_t)1 << (s->lmax + 1);
    for (int a = 0; a < 3; ++a) {
        int64_t lo = c.lo[a], hi = c.hi[a];
        if (hi - lo + ((int64_t)1 << (s->lmax + 3)) > kSpanLimit)
            return fail(AMR_ERANGE, "amr_upload: extent %lld on axis %d too large for level %d (limit 2^20)",
                        (long long)(hi - lo), a, s->lmax);
        int64_t fl = lo >= 0 ? (lo / blk) * blk : -((-lo + blk - 1) / blk) * blk;
        s->origin[a] = (int32_t)(fl - blk);
    }
    uint64_t hint = 0;
    for (int l = 0; l <= kMaxLevel; ++l) {
        s->level_count[l] = c.level_count[l];
        hint += (c.level_count[l] + 7) / 8;
    }
    s->group_hint = hint;
    s->uploaded = true;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_index_bytes(const amr_set* s, size_t* bytes) {
    if (!s || !bytes) return fail(AMR_EINVAL, "amr_index_bytes: NULL argument");
    if (!s->uploaded) return fail(AMR_ESTATE, "amr_index_bytes: call amr_upload first");
    uint32_t cap = table_cap(s);
    if (!cap) return fail(AMR_ERANGE, "amr_index_bytes: more groups than the index supports");
    *bytes = layout_for(cap).total;
    return AMR_OK;
}

int amr_build_index(amr_set* s, void* ws, size_t bytes, hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_build_index: set is NULL");
    if (!s->uploaded) return fail(AMR_ESTATE, "amr_build_index: call amr_upload first");
    s->built = false;
    uint32_t cap = table_cap(s);
    if (!cap) return fail(AMR_ERANGE, "amr_build_index: more groups than the index supports");
    Layout L = layout_for(cap);
    if (!ws || ((uintptr_t)ws & 255)) return fail(AMR_EINVAL, "amr_build_index: workspace NULL or not 256-B aligned");
    if (bytes < L.total)
        return fail(AMR_ENOSPACE, "amr_build_index: workspace of %zu bytes, need %zu", bytes, L.total);
    DeviceGuard dg(s->device);
    char* base = (char*)ws;
    s->cap = cap;
    s->rec = (Record*)(base + L.rec);
    s->ids = (int32_t*)(base + L.ids);
    s->glist = (int32_t*)(base + L.glist);
    s->st_t = (unsigned long long*)(base + L.st_t);
    s->st_d = (unsigned long long*)(base + L.st_d);
    s->sched = (Sched*)(base + L.sched);
    s->max_tiles = L.max_tiles;
    s->n_groups = 0;
    Geo g = geo_of(s);
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, stream, s->ctrl);
    hipLaunchKernelGGL(k_index_init, dim3(grid_for(cap, 256)), dim3(256), 0, stream, s->rec, s->ids, cap);
    hipLaunchKernelGGL(k_sched_reset, dim3(grid_for(L.max_tiles, 256)), dim3(256), 0, stream, s->sched, s->st_t,
                       s->st_d, L.max_tiles);
    if (s->n > 0) {
        hipLaunchKernelGGL(k_index_insert, dim3(grid_for(s->n, 256)), dim3(256), 0, stream, s->xyz, s->lvl, s->val,
                           s->n, g, s->rec, s->ids, s->glist, cap / 2, s->ctrl);
        hipLaunchKernelGGL(k_index_overlap, dim3(grid_for(s->n, 256)), dim3(256), 0, stream, s->xyz, s->lvl, s->n, g,
                           s->rec, s->ctrl);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_build_index: launch");
    e = hipMemcpyAsync(&s->host_ctrl, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hipfail(e, "amr_build_index: readback");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "amr_build_index: synchronize");
    const Ctrl& c = s->host_ctrl;
    if (c.overflow) {
        uint64_t seen = c.n_groups;
        s->group_hint = seen > s->group_hint * 4 ? seen : s->group_hint * 4;
        return fail(AMR_ENOSPACE, "amr_build_index: hash table too small (%u slots); query amr_index_bytes again",
                    cap);
    }
    if (c.dup) return fail(AMR_EOVERLAP, "amr_build_index: duplicate cell (index %llu)", c.bad_build);
    if (c.overlap) return fail(AMR_EOVERLAP, "amr_build_index: cell %llu lies inside a coarser cell", c.bad_build);
    s->n_groups = c.n_groups;
    s->built = true;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_dual_cells(amr_set* s, int32_t* corner_level, int32_t* verts, int64_t cap, int64_t* counts,
                   hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_dual_cells: set is NULL");
    if (!s->built) return fail(AMR_ESTATE, "amr_dual_cells: call amr_build_index first");
    if (cap < 0 || (cap > 0 && !corner_level && !verts)) return fail(AMR_EINVAL, "amr_dual_cells: bad capacity");
    DeviceGuard dg(s->device);
    return launch_extract(s, true, 0.0f, nullptr, nullptr, nullptr, corner_level, verts, cap, counts, stream);
}

int amr_isosurface(amr_set* s, float iso, float* tris, int32_t* tri_cells, int32_t* tri_dual, int64_t cap,
                   int64_t* counts, hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_isosurface: set is NULL");
    if (!s->built) return fail(AMR_ESTATE, "amr_isosurface: call amr_build_index first");
    if (!isfinite(iso)) return fail(AMR_EINVAL, "amr_isosurface: iso is not finite");
    if (cap < 0) return fail(AMR_EINVAL, "amr_isosurface: negative capacity");
    DeviceGuard dg(s->device);
    return launch_extract(s, false, iso, tris, tri_cells, tri_dual, nullptr, nullptr, cap, counts, stream);
}

const char* amr_last_error(void) { return g_err; }

}  // extern "C"
