// amriso.hip -- HIP implementation of libamriso.so for gfx950 (MI355X).
//
// Dual-mesh and crack-free iso-surface extraction from AMR cells, after
// I. Wald, "A Simple, General, and GPU Friendly Method for Computing Dual
// Mesh and Iso-Surfaces of Adaptive Mesh Refinement (AMR) Data",
// arXiv 2004.08475.  The C ABI is declared in include/amriso.h.
//
// Data layout in HBM
//   input (caller, borrowed): SoA  xyz int32[n][3], level int32[n], value f32[n]
//   index workspace (caller): records | cell ids | group list + keys | scan states
//     record (64 B, one per hash slot): val f32[8] | key u64 | homed u32 | pad
//       A record belongs to one 2x2x2 block of level-m logical cells (a
//       "group"): key = (m, block coordinates).  val[c] is the value of
//       child c (c = bx + 2 by + 4 bz) when that child is an actual cell of
//       level m, the NaN "empty" when it is not, or the NaN "refined" when
//       finer cells exist inside it.  One probe thus returns up to 8 cells,
//       and the refined markers end a snap as soon as it meets finer cells.
//       Slots come in regions of 4096, one per 16x16x16 block of groups
//       (Morton order inside), so neighbours share a few cache lines.
//     cell ids  int32[slots][8]: input index of the cell in each child slot,
//       filled in when an output first asks for cell indices
//     group list int32[] + keys u64[]: the records that hold at least one
//       cell, ordered by (home slot, key) -- a function of the cells alone,
//       unlike slot order, which follows the races of the insertion
//     scan states: look-back words of the compaction and of the extraction
//
// Extraction kernel (paper sec. 4.2-5): one work-group processes 32 groups,
// eight lanes per group.  The lanes fetch the level-m cells of the 4x4x4
// block around their group (absent ones resolved to the coarser cell that
// covers them) into LDS, then evaluate the 27 corners of the group's 2x2x2
// cell block.  A corner's logical dual is emitted when its 8 slots are all
// covered by cells of this level or coarser and the lowest-numbered slot on
// this level belongs to this group -- rules 1-3 of the paper, with the
// "precedes" order of rule 3 read as slot order (= lexicographic (z,y,x)
// order of the lower corners of same-level cells).  Marching Cubes runs on
// each emitted dual from a 256-entry table kept in LDS; degenerate triangles
// are culled by comparing cell references.  Small sets run one fused pass
// whose tiles find their output positions by a decoupled look-back; large
// sets run a count pass, a scan of the tile totals and a write pass, so no
// tile waits for another.  Output positions are deterministic either way.
//
// Also here: batched runs of many (set, iso) jobs (a unit of groups loaded
// once per pass for all jobs of its set), the dual mesh as an interpolant
// (a cell-to-dual map and point queries), the paper's own sorted-cells
// index beside the hash (for the comparison), and the weld of fat triangles
// into an indexed face set.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "amriso.h"
#include "mc_table.inc"

namespace {

constexpr int kMaxLevel = 20;
constexpr int kCoordLimit = 1 << 23;    // |corner| bound: centres exact in f32
constexpr int kSpanLimit = 1 << 20;     // offset coordinates u < 2^20
constexpr uint64_t kEmpty = ~0ull;      // key of a free slot
constexpr uint32_t kValEmpty = 0x7fc00000u;    // NaN: no cell of this level here
constexpr uint32_t kValRefined = 0x7fc00001u;  // NaN: finer cells inside
constexpr int kGroupsPerTile = 32;
constexpr int kBlock = 256;             // 32 groups x 8 lanes
constexpr int kTriList = 256;           // triangle entries staged per round
constexpr uint32_t kMaxCap = 1u << 28;  // slot * 8 + child fits int32
constexpr uint32_t kMaxProbe = 1024;    // longer chains mean the table is too full
constexpr int kCompactMaxPerThread = 16;
// Threads per work-group of the compaction: each work-group takes one
// ticket and one look-back step, so fewer, larger tiles (measured: 2^20
// slots 61 us against 66 with 256 threads and 62 with 1024; 2^24 slots
// 0.41 ms against 0.50 and 0.39)
constexpr int kCompactBlock = 512;
constexpr int kReplicas = 64;           // spread of the upload reduction atomics
constexpr uint32_t kFusedMaxTiles = 2048;  // sets up to this many tiles extract in one fused pass
constexpr uint32_t kXcds = 8;              // accelerator complex dies of an MI355X
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

enum : uint32_t { kErrLevel = 1, kErrAlign = 2, kErrValue = 4, kErrCoord = 8 };

struct alignas(64) Record {
    float val[8];
    uint64_t key;
    uint32_t homed;  // group keys homed at this slot that sit elsewhere (counted as they are created)
    uint32_t pad[5];
};
static_assert(sizeof(Record) == 64, "record is one 64-byte line");

// One replica of the upload reduction: work-group b updates replica b % 64,
// so no address receives more than 1/64 of the atomics; the host combines.
struct alignas(256) Partial {
    int32_t lo[3];
    int32_t hi[3];
    int32_t lmin, lmax;
    uint32_t err;
    uint32_t pad0;
    unsigned long long bad;
    unsigned long long level_count[kMaxLevel + 1];
};

// Index geometry: coordinate origin, coarsest level and hash parameters.
struct Geo {
    int32_t ox, oy, oz;  // origin: u = x - ox >= 2^(lmax+1)
    int lmax;
    int shift;           // 64 - log2(cap)
    uint32_t mask;       // cap - 1
};

// Verdict of an upload, reduced on the device from the 64 replicas.
struct UpRes {
    int32_t lo[3], hi[3];
    int32_t lmin, lmax;
    int32_t origin[3];
    int32_t status;  // AMR_OK, AMR_EINVAL or AMR_ERANGE
    uint32_t err;    // error class bits (kErr*), or 16 + axis for an extent error
    uint32_t pad;
    unsigned long long bad;  // lowest offending cell index
    unsigned long long level_count[kMaxLevel + 1];
    unsigned long long record_hint;
};

// Device control block, one per set (library-allocated).  The build's
// verdict (`status`) is decided on the device by a one-lane kernel after the
// ancestor marking; extraction kernels read it, the group count and the
// geometry from here, so nothing of the build has to reach the host before
// the next call is enqueued.
constexpr int32_t kStatusPending = 1;  // a build is enqueued and has not finished

struct Ctrl {
    Partial part[kReplicas];
    uint32_t overflow;
    uint32_t dup;
    uint32_t overlap;
    int32_t status;                // AMR_OK or the build's error code (kStatusPending meanwhile)
    uint32_t pad1[2];
    unsigned long long bad_build;
    unsigned long long n_groups;   // written by the compaction's last tile
    unsigned long long n_records;
    unsigned long long n_leaves;   // cells present in the table
    unsigned long long made[kReplicas * 16];  // marker-only records created (one replica per 128 B)
    UpRes res;                     // upload verdict (k_upload_finish)
    Geo geo;                       // geometry of the index being built (k_build_reset)
};

// Scan bookkeeping inside the workspace.
struct Sched {
    unsigned long long xticket;  // extraction scan tiles started (reset by each count pass)
    unsigned long long fcall;    // fused extraction calls started
    unsigned long long cticket;  // compaction tiles started
    unsigned long long fticket;  // fused extraction tiles started, over all calls
    unsigned long long lticket;  // candidate-list work-groups started, over all calls
    uint32_t rng_ok;             // group value ranges and dual count recorded for this build
    uint32_t pad;
};

__device__ __forceinline__ uint64_t group_key(int m, uint32_t gx, uint32_t gy, uint32_t gz) {
    return ((uint64_t)m << 57) | ((uint64_t)gz << 38) | ((uint64_t)gy << 19) | (uint64_t)gx;
}

// Home slot of a group.  The table is cut into regions of 4096 slots, one
// per block of 16x16x16 groups of one level: the block's key is hashed
// (Fibonacci) to a region and the group's position inside it, as a 12-bit
// Morton code, picks the slot, XORed with 12 more bits of the block hash so
// that sparse patterns still spread over all positions.  XOR with a constant
// keeps every aligned run of 2^k Morton codes together, so 32 consecutive
// slots hold a 4x4x2 block of groups and consecutive runs are neighbours in
// space.  A collision moves on to the same position of the next region
// (probe stride 4096); once every region has been tried at that position
// (the step count a multiple of cap / 4096), the position moves on by one,
// so the probe sequence covers the whole table before it repeats.  (With
// the stride alone a small table has few regions, and a position taken in
// all of them left keys without a slot and lookups cycling through the same
// few slots until the step limit.)
constexpr uint32_t kRegion = 4096;

__device__ __forceinline__ uint32_t spread4(uint32_t v) {
    // bits 0..3 of v to bits 0, 3, 6, 9
    return (v & 1u) | ((v & 2u) << 2) | ((v & 4u) << 4) | ((v & 8u) << 6);
}

__device__ __forceinline__ uint32_t slot_of(uint64_t key, int shift) {
    const uint64_t region = key & ~((15ull << 38) | (15ull << 19) | 15ull);
    const uint32_t local = spread4((uint32_t)key & 15u) | (spread4((uint32_t)(key >> 19) & 15u) << 1) |
                           (spread4((uint32_t)(key >> 38) & 15u) << 2);
    return (uint32_t)((region * kGolden) >> shift) ^ local;
}

// The slot after h, the step-th slot of a probe sequence (step 0 = home).
__device__ __forceinline__ uint32_t next_slot(uint32_t h, uint32_t step, uint32_t mask) {
    uint32_t n = (h + kRegion) & mask;
    if (((step + 1) & (mask >> 12)) == 0) n = (n & ~(kRegion - 1)) | ((n + 1) & (kRegion - 1));
    return n;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T x, Op op) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = op(x, __shfl_xor(x, off, 64));
    return x;
}

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long x) {
    int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

__device__ __forceinline__ unsigned long long ld_relaxed(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Linear probe for `key`; returns the slot or -1 (never more than cap steps).
__device__ __forceinline__ int probe(const Record* __restrict__ rec, uint64_t key, int shift, uint32_t mask) {
    uint32_t h = slot_of(key, shift);
    for (uint32_t i = 0; i <= mask; ++i) {
        uint64_t k = rec[h].key;
        if (k == key) return (int)h;
        if (k == kEmpty) return -1;
        h = next_slot(h, i, mask);
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Decoupled look-back over tiles (called by one whole wave).  A tile's state
// is two words, one per running total, each: flag (2 bits) | parity (1 bit)
// | value; flag 1 = the tile's own aggregate, flag 2 = inclusive prefix.
// Every call rewrites every tile's words, so words left by the previous call
// (other parity) read as "not yet written" and need no clearing.  The wave
// reads 256 predecessors per step; relaxed device-scope accesses suffice
// because the words carry the data themselves.
// ---------------------------------------------------------------------------

constexpr unsigned long long kFlagShift = 62;
constexpr unsigned long long kParityBit = 1ull << 61;
constexpr unsigned long long kValMask = kParityBit - 1;
constexpr unsigned long long kFlagAgg = 1, kFlagIncl = 2;
constexpr int kLookWindows = 4;

__device__ void lookback(unsigned long long* s0, unsigned long long* s1, uint32_t tile, unsigned long long par,
                         unsigned long long a0, unsigned long long a1, unsigned long long& p0,
                         unsigned long long& p1) {
    const int lane = lane_id();
    p0 = 0;
    p1 = 0;
    if (tile == 0) {
        if (lane == 0) {
            st_relaxed(&s1[0], (kFlagIncl << kFlagShift) | par | a1);
            st_relaxed(&s0[0], (kFlagIncl << kFlagShift) | par | a0);
        }
        return;
    }
    if (lane == 0) {
        st_relaxed(&s1[tile], (kFlagAgg << kFlagShift) | par | a1);
        st_relaxed(&s0[tile], (kFlagAgg << kFlagShift) | par | a0);
    }
    auto add = [](unsigned long long x, unsigned long long y) { return x + y; };
    int base = (int)tile - 1;
    while (true) {
        unsigned long long w0[kLookWindows], w1[kLookWindows];
#pragma unroll
        for (int r = 0; r < kLookWindows; ++r) {
            int idx = base - lane - 64 * r;
            w0[r] = 0;
            w1[r] = 0;
            if (idx >= 0) {
                w0[r] = ld_relaxed(&s0[idx]);
                w1[r] = ld_relaxed(&s1[idx]);
            }
        }
        bool found = false, stall = false;
        unsigned long long q0 = 0, q1 = 0;
#pragma unroll
        for (int r = 0; r < kLookWindows; ++r) {
            if (found || stall) continue;
            int idx = base - lane - 64 * r;
            unsigned long long f0 = w0[r] >> kFlagShift, f1 = w1[r] >> kFlagShift;
            bool ready = idx < 0 || (f0 != 0 && f0 == f1 && (w0[r] & kParityBit) == par &&
                                     (w1[r] & kParityBit) == par);
            bool incl = idx >= 0 && ready && f0 == kFlagIncl;
            unsigned long long pm = __ballot(incl);
            unsigned long long nr = __ballot(!ready);
            // lanes up to and including the nearest inclusive prefix count
            unsigned long long need = pm ? (((pm & (~pm + 1)) << 1) - 1) : ~0ull;
            if (nr & need) {
                stall = true;
                continue;
            }
            bool take = idx >= 0 && ((need >> lane) & 1);
            q0 += take ? (w0[r] & kValMask) : 0;
            q1 += take ? (w1[r] & kValMask) : 0;
            if (pm) found = true;
        }
        if (stall) {
            // a predecessor has not published yet: wait, then re-read the stretch
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        p0 += wave_reduce(q0, add);
        p1 += wave_reduce(q1, add);
        if (found) break;
        base -= 64 * kLookWindows;
    }
    if (lane == 0) {
        st_relaxed(&s1[tile], (kFlagIncl << kFlagShift) | par | (p1 + a1));
        st_relaxed(&s0[tile], (kFlagIncl << kFlagShift) | par | (p0 + a0));
    }
}

// ---------------------------------------------------------------------------
// Upload: validation and reductions
// ---------------------------------------------------------------------------

__global__ void k_ctrl_reset(Ctrl* c) {
    for (int r = threadIdx.x; r < kReplicas; r += blockDim.x) {
        Partial& p = c->part[r];
        for (int a = 0; a < 3; ++a) {
            p.lo[a] = INT32_MAX;
            p.hi[a] = INT32_MIN;
        }
        p.lmin = INT32_MAX;
        p.lmax = INT32_MIN;
        p.err = 0;
        p.bad = ~0ull;
        for (int l = 0; l <= kMaxLevel; ++l) p.level_count[l] = 0;
    }
    if (threadIdx.x == 0) {
        c->overflow = 0;
        c->dup = 0;
        c->overlap = 0;
        c->status = kStatusPending;
        c->bad_build = ~0ull;
        c->n_groups = 0;
        c->n_records = 0;
        c->n_leaves = 0;
    }
}

__global__ __launch_bounds__(256) void k_upload(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                const float* __restrict__ val, int64_t n, Ctrl* c) {
    __shared__ int s_lo[3], s_hi[3], s_lmin, s_lmax;
    __shared__ unsigned long long s_cnt[kMaxLevel + 1];
    Partial& P = c->part[blockIdx.x % kReplicas];
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
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = i0 + t;
        int l = -1;
        if (i < n) {
            int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
            l = lvl[i];
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
                atomicOr(&P.err, bad);
                atomicMin(&P.bad, (unsigned long long)i);
                l = -1;
            } else {
                int w = 1 << l;
                lo0 = min(lo0, x);
                lo1 = min(lo1, y);
                lo2 = min(lo2, z);
                hi0 = max(hi0, x + w);
                hi1 = max(hi1, y + w);
                hi2 = max(hi2, z + w);
                lmin = min(lmin, l);
                lmax = max(lmax, l);
            }
        }
        // per-level counts: one ballot per level present in the wave
        unsigned long long bit = l >= 0 ? (1ull << l) : 0ull;
        unsigned long long present =
            wave_reduce(bit, [](unsigned long long a, unsigned long long b) { return a | b; });
        while (present) {
            int L = __ffsll((long long)present) - 1;
            present &= present - 1;
            unsigned long long b = __ballot(l == L);
            if (lane_id() == 0) atomicAdd(&s_cnt[L], (unsigned long long)__popcll(b));
        }
    }
    auto mn = [](int a, int b) { return a < b ? a : b; };
    auto mx = [](int a, int b) { return a > b ? a : b; };
    lo0 = wave_reduce(lo0, mn);
    lo1 = wave_reduce(lo1, mn);
    lo2 = wave_reduce(lo2, mn);
    hi0 = wave_reduce(hi0, mx);
    hi1 = wave_reduce(hi1, mx);
    hi2 = wave_reduce(hi2, mx);
    lmin = wave_reduce(lmin, mn);
    lmax = wave_reduce(lmax, mx);
    if (lane_id() == 0) {
        atomicMin(&s_lo[0], lo0);
        atomicMin(&s_lo[1], lo1);
        atomicMin(&s_lo[2], lo2);
        atomicMax(&s_hi[0], hi0);
        atomicMax(&s_hi[1], hi1);
        atomicMax(&s_hi[2], hi2);
        atomicMin(&s_lmin, lmin);
        atomicMax(&s_lmax, lmax);
    }
    __syncthreads();
    if (t < 3) {
        atomicMin(&P.lo[t], s_lo[t]);
        atomicMax(&P.hi[t], s_hi[t]);
    }
    if (t == 0) {
        atomicMin(&P.lmin, s_lmin);
        atomicMax(&P.lmax, s_lmax);
    }
    if (t <= kMaxLevel && s_cnt[t]) atomicAdd(&P.level_count[t], s_cnt[t]);
}

// One wave: combines the 64 replicas into the upload verdict, and derives
// the index origin (aligned to 2^(lmax+1), one block of margin below the
// cells) and the expected record count from it.
__global__ __launch_bounds__(64) void k_upload_finish(Ctrl* c) {
    const int r = threadIdx.x;
    const Partial& p = c->part[r];
    auto mn = [](int a, int b) { return a < b ? a : b; };
    auto mx = [](int a, int b) { return a > b ? a : b; };
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = wave_reduce(p.lo[a], mn);
        hi[a] = wave_reduce(p.hi[a], mx);
    }
    const int lmin = wave_reduce(p.lmin, mn), lmax = wave_reduce(p.lmax, mx);
    const uint32_t err = wave_reduce(p.err, [](uint32_t a, uint32_t b) { return a | b; });
    const unsigned long long bad =
        wave_reduce(p.bad, [](unsigned long long a, unsigned long long b) { return a < b ? a : b; });
    unsigned long long hint = 0;
    for (int l = 0; l <= kMaxLevel; ++l) {
        // only levels that occur can have cells
        const unsigned long long cnt =
            (l >= lmin && l <= lmax)
                ? wave_reduce(p.level_count[l], [](unsigned long long a, unsigned long long b) { return a + b; })
                : 0ull;
        if (r == 0) c->res.level_count[l] = cnt;
        hint += (cnt + 7) / 8;
    }
    // leave this replica clean for the next upload (every lane has read it)
    {
        Partial& q = c->part[r];
        for (int a = 0; a < 3; ++a) {
            q.lo[a] = INT32_MAX;
            q.hi[a] = INT32_MIN;
        }
        q.lmin = INT32_MAX;
        q.lmax = INT32_MIN;
        q.err = 0;
        q.bad = ~0ull;
        for (int l = 0; l <= kMaxLevel; ++l) q.level_count[l] = 0;
    }
    if (r != 0) return;
    UpRes& u = c->res;
    for (int a = 0; a < 3; ++a) {
        u.lo[a] = lo[a];
        u.hi[a] = hi[a];
        u.origin[a] = 0;
    }
    u.lmin = lmin;
    u.lmax = lmax;
    u.err = err;
    u.bad = bad;
    u.status = AMR_OK;
    // records: one per group of each level, plus refined markers (about one
    // record per 7 groups for octrees)
    u.record_hint = hint + hint / 7 + 64;
    if (err) {
        u.status = (err & (kErrLevel | kErrAlign | kErrValue)) ? AMR_EINVAL : AMR_ERANGE;
        return;
    }
    if (lmax < lmin) {
        // no cells at all (an empty upload): an empty box at the origin
        for (int a = 0; a < 3; ++a) u.lo[a] = u.hi[a] = 0;
        u.lmin = u.lmax = 0;
        return;
    }
    const long long blk = 1ll << (lmax + 1);
    for (int a = 0; a < 3; ++a) {
        if ((long long)hi[a] - lo[a] + (1ll << (lmax + 3)) > kSpanLimit) {
            u.status = AMR_ERANGE;
            u.err = 16u + (uint32_t)a;
            return;
        }
        const long long l0 = lo[a];
        const long long fl = l0 >= 0 ? (l0 / blk) * blk : -((-l0 + blk - 1) / blk) * blk;
        u.origin[a] = (int32_t)(fl - blk);
    }
}

// ---------------------------------------------------------------------------
// Index build
// ---------------------------------------------------------------------------

// Start of a build: empty records, clean scan states, zero build results.
__global__ __launch_bounds__(256) void k_build_reset(Record* __restrict__ rec, uint32_t cap, int shift, Sched* sc,
                                                     unsigned long long* ct0, unsigned long long* ct1, uint32_t nc,
                                                     unsigned long long* fs0, unsigned long long* fs1,
                                                     unsigned long long* ls0, unsigned long long* ls1, uint32_t nl,
                                                     Ctrl* c) {
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x, step = gridDim.x * blockDim.x;
    // the table as 16-byte quarters of records, consecutive lanes on
    // consecutive quarters: values (two quarters of NaN), then key (all ones),
    // homed and padding (zero)
    static_assert(offsetof(Record, key) == 32 && offsetof(Record, homed) == 40, "record quarters");
    uint4* q = reinterpret_cast<uint4*>(rec);
    for (uint32_t i = i0; i < cap * 4u; i += step) {
        const uint32_t part = i & 3u;
        const uint32_t w = part < 2 ? kValEmpty : 0u, kw = part == 2 ? 0xffffffffu : w;
        q[i] = make_uint4(kw, kw, w, w);
    }
    for (uint32_t i = i0; i < nc; i += step) {
        ct0[i] = 0;
        ct1[i] = 0;
    }
    for (uint32_t i = i0; i < kFusedMaxTiles; i += step) {
        fs0[i] = 0;
        fs1[i] = 0;
    }
    for (uint32_t i = i0; i < nl; i += step) {
        ls0[i] = 0;
        ls1[i] = 0;
    }
    if (i0 < (uint32_t)kReplicas) c->made[i0 * 16] = 0;
    if (i0 == 0) {
        sc->xticket = 0;
        sc->fcall = 0;
        sc->cticket = 0;
        sc->fticket = 0;
        sc->lticket = 0;
        sc->rng_ok = 0;
        c->overflow = 0;
        c->dup = 0;
        c->overlap = 0;
        c->status = kStatusPending;
        c->bad_build = ~0ull;
        c->n_groups = 0;
        c->n_records = 0;
        c->n_leaves = 0;
        // the geometry comes from the upload verdict, which the host may not
        // have read yet
        Geo g;
        g.ox = c->res.origin[0];
        g.oy = c->res.origin[1];
        g.oz = c->res.origin[2];
        g.lmax = c->res.lmax;
        g.shift = shift;
        g.mask = cap - 1;
        c->geo = g;
    }
}

// A key never changes once written, so a plain (possibly stale) read can only
// show "free" too often; the compare-and-swap then returns the truth.
__device__ __forceinline__ int find_or_insert(Record* __restrict__ rec, uint64_t key, const Geo& g,
                                              uint32_t* created = nullptr) {
    uint32_t h = slot_of(key, g.shift);
    for (uint32_t step = 0; step < kMaxProbe && step <= g.mask; ++step) {
        uint64_t k = rec[h].key;
        if (k == key) return (int)h;
        if (k == kEmpty) {
            uint64_t prev = atomicCAS((unsigned long long*)&rec[h].key, (unsigned long long)kEmpty,
                                      (unsigned long long)key);
            if (prev == kEmpty && created) ++*created;
            if (prev == kEmpty || prev == key) return (int)h;
        }
        h = next_slot(h, step, g.mask);
    }
    return -1;
}

// The lowest active lane of the wave holding the same key (a lane's own
// index when it holds a key no lower lane holds).  Lanes of one group are
// usually neighbours in a wave, so one of them probes the table for all;
// after 16 distinct keys the rest lead themselves.
__device__ __forceinline__ int same_key_leader(uint64_t key, bool active) {
    const int lane = lane_id();
    int leader = lane;
    unsigned long long todo = __ballot(active);
    for (int it = 0; it < 16 && todo; ++it) {
        const int l = __ffsll((long long)todo) - 1;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(key >> 32), l);
        const bool same = active && key == (((uint64_t)hi << 32) | lo);
        if (same) leader = l;
        todo &= ~__ballot(same);
    }
    return leader;
}

// Every cell stores its value in its group record (a plain store: a
// duplicate cell overwrites its twin and shows up later as a missing leaf in
// the count of the compaction).  The cell that creates a group's record
// away from the key's home slot counts the key there (a key at home is
// counted by the compaction), which orders the group list.
// Input indices are filled in later, and only when an output asks for them
// (k_index_ids).
__global__ __launch_bounds__(256) void k_index_insert(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                      const float* __restrict__ val, int64_t n,
                                                      Record* __restrict__ rec, Ctrl* c) {
    if (c->res.status != AMR_OK) return;  // invalid cells: nothing to index
    const Geo g = c->geo;
    const int lane = lane_id();
    // whole waves step together (the leader election needs every lane)
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = b + threadIdx.x;
        const bool live = i < n;
        int m = 0, child = 0;
        uint64_t key = 0;
        if (live) {
            m = lvl[i];
            const uint32_t ux = (uint32_t)(xyz[3 * i] - g.ox), uy = (uint32_t)(xyz[3 * i + 1] - g.oy),
                           uz = (uint32_t)(xyz[3 * i + 2] - g.oz);
            key = group_key(m, ux >> (m + 1), uy >> (m + 1), uz >> (m + 1));
            child = ((ux >> m) & 1) | (((uy >> m) & 1) << 1) | (((uz >> m) & 1) << 2);
        }
        const int leader = same_key_leader(key, live);
        int slot = -1;
        if (live && leader == lane) {
            uint32_t created = 0;
            slot = find_or_insert(rec, key, g, &created);
            if (created) {
                const uint32_t hs = slot_of(key, g.shift);
                if ((uint32_t)slot != hs) atomicAdd(&rec[hs].homed, 1u);  // a key at home counts itself
            }
        }
        slot = __shfl(slot, leader, 64);
        if (!live) continue;
        if (slot < 0) {
            atomicOr(&c->overflow, 1u);
            continue;
        }
        rec[slot].val[child] = val[i];
    }
}

// The input index of every cell, beside its value (slot * 8 + child).
__global__ __launch_bounds__(256) void k_index_ids(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                   int64_t n, const Ctrl* c, const Record* __restrict__ rec,
                                                   int32_t* __restrict__ ids) {
    if (c->res.status != AMR_OK) return;  // invalid cells: nothing was indexed
    const Geo g = c->geo;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int m = lvl[i];
        uint32_t ux = (uint32_t)(xyz[3 * i] - g.ox), uy = (uint32_t)(xyz[3 * i + 1] - g.oy),
                 uz = (uint32_t)(xyz[3 * i + 2] - g.oz);
        int slot = probe(rec, group_key(m, ux >> (m + 1), uy >> (m + 1), uz >> (m + 1)), g.shift, g.mask);
        if (slot < 0) continue;
        int child = ((ux >> m) & 1) | (((uy >> m) & 1) << 1) | (((uz >> m) & 1) << 2);
        ids[(size_t)slot * 8 + child] = (int32_t)i;
    }
}

// Every group holding a cell marks its ancestors as refined, level by
// level, until it meets a mark set by another group.  All leaves are stored
// before this pass, so a mark that lands on a leaf is a coarser cell
// containing finer ones.  The pass runs over the compacted group list (the
// compaction's count is on the device), and counts the marker-only records
// it creates, one atomic per work-group into one of 64 replicas.
__global__ __launch_bounds__(256) void k_index_mark(Record* __restrict__ rec,
                                                    const unsigned long long* __restrict__ gkey, Ctrl* c) {
    __shared__ uint32_t s_made;
    if (c->res.status != AMR_OK) return;
    const Geo g = c->geo;
    const uint32_t ng = (uint32_t)c->n_groups;
    if (threadIdx.x == 0) s_made = 0;
    __syncthreads();
    uint32_t made = 0;
    const int lane = lane_id();
    // whole waves step together, level by level (the leader election needs
    // every lane); sibling groups sit side by side in the list and share
    // the record one level up, which one of them probes for all
    for (uint32_t b = blockIdx.x * blockDim.x; b < ng; b += gridDim.x * blockDim.x) {
        const uint32_t i = b + threadIdx.x;
        uint64_t key = 0;
        if (i < ng) key = gkey[i];
        const int m = (int)(key >> 57);
        bool going = i < ng && m < g.lmax;
        const uint32_t gx = (uint32_t)(key & 0x7FFFF), gy = (uint32_t)((key >> 19) & 0x7FFFF),
                       gz = (uint32_t)((key >> 38) & 0x7FFFF);
        int L = m + 1;
        while (__ballot(going)) {
            // the level-L cell holding this group's block, and its group
            const int sh = L - m - 1;
            const uint32_t cx = gx >> sh, cy = gy >> sh, cz = gz >> sh;
            const uint64_t pkey = going ? group_key(L, cx >> 1, cy >> 1, cz >> 1) : 0;
            const int leader = same_key_leader(pkey, going);
            int s2 = -1;
            if (going && leader == lane) s2 = find_or_insert(rec, pkey, g, &made);
            s2 = __shfl(s2, leader, 64);
            if (!going) continue;
            if (s2 < 0) {
                atomicOr(&c->overflow, 1u);
                going = false;
                continue;
            }
            const int c2 = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
            unsigned int* slot_val = reinterpret_cast<unsigned int*>(&rec[s2].val[c2]);
            // a mark already seen needs no atomic (a stale read only costs one)
            uint32_t prev = *slot_val;
            if (prev == kValEmpty) {
                // the first level up is this group's own block: finer groups
                // inside it may mark it too, but only with the same value
                if (L == m + 1) *slot_val = kValRefined;
                else prev = atomicCAS(slot_val, kValEmpty, kValRefined);
            }
            if (prev == kValEmpty) {  // marked here: carry on upwards
                ++L;
                going = L <= g.lmax;
                continue;
            }
            if (prev != kValRefined) {  // a coarser cell contains this group
                atomicOr(&c->overlap, 1u);
                atomicMin(&c->bad_build, (unsigned long long)s2 * 8 + c2);  // its slot * 8 + child
            }
            going = false;
        }
    }
    made = (uint32_t)wave_reduce((unsigned long long)made,
                                 [](unsigned long long x, unsigned long long y) { return x + y; });
    if (lane_id() == 0 && made) atomicAdd(&s_made, made);
    __syncthreads();
    if (threadIdx.x == 0 && s_made) atomicAdd(&c->made[(blockIdx.x % kReplicas) * 16], (unsigned long long)s_made);
}

// The build's verdict, decided on the device by one lane after the marking:
// the upload's error, a table too full (a failed insertion, more than 3/4
// of the slots in use, or more groups than the `max_groups` the extraction
// grids are sized for), a coarser cell containing finer ones, or fewer
// leaves than cells (a duplicate overwrote its twin).  A kernel of its own:
// a last-work-group test inside the marking pass costs one device-scope
// atomic per work-group on one address, serialised across the XCDs (1.8 ms
// for the 16384 work-groups of a 50M-cell set).
__global__ void k_index_verdict(int64_t n, uint32_t cap, uint32_t max_groups, Ctrl* c) {
    if (threadIdx.x != 0) return;
    int32_t st = c->res.status;
    if (st == AMR_OK) {
        unsigned long long recs = c->n_records;  // records at compaction time: the groups
        for (int r = 0; r < kReplicas; ++r) recs += c->made[r * 16];
        if (c->overflow || recs * 4 > (unsigned long long)cap * 3 || c->n_groups > max_groups)
            st = AMR_ENOSPACE;
        else if (c->overlap || c->n_leaves != (unsigned long long)n)
            st = AMR_EOVERLAP;
    }
    c->status = st;
}

// Error path only: the lowest input index whose entry was overwritten by a
// duplicate of the same cell.
__global__ __launch_bounds__(256) void k_index_find_dup(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                        int64_t n, const Record* __restrict__ rec,
                                                        const int32_t* __restrict__ ids, Ctrl* c) {
    const Geo g = c->geo;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int m = lvl[i];
        uint32_t ux = (uint32_t)(xyz[3 * i] - g.ox), uy = (uint32_t)(xyz[3 * i + 1] - g.oy),
                 uz = (uint32_t)(xyz[3 * i + 2] - g.oz);
        int slot = probe(rec, group_key(m, ux >> (m + 1), uy >> (m + 1), uz >> (m + 1)), g.shift, g.mask);
        if (slot < 0) continue;
        int child = ((ux >> m) & 1) | (((uy >> m) & 1) << 1) | (((uz >> m) & 1) << 2);
        if (ids[(size_t)slot * 8 + child] != (int32_t)i) atomicMin(&c->bad_build, (unsigned long long)i);
    }
}

// Group list: the slots and keys of all records holding at least one cell,
// ordered by (home slot, key).  That order is a function of the set of
// cells alone: which of two colliding keys won a slot is not, so neither is
// plain slot order.  Every key homed at slot h lies on h's probe sequence
// (the sequence depends on the slot only), and h's record counts those that
// sit elsewhere (the one at h, if homed there, is seen here), so a block
// scan plus look-back over the counts of tiles of slots gives each
// home its first list position; a home with one key that sits at home (the
// common case) writes it at once, others walk their probe sequence and write
// their keys in ascending order.  Also counts all occupied records (groups
// plus marker-only records) and their leaves.  At this point of a build
// every record is a group's.
__global__ __launch_bounds__(kCompactBlock) void k_index_compact(const Record* __restrict__ rec, uint32_t cap,
                                                          int32_t* __restrict__ glist,
                                                          unsigned long long* __restrict__ gkey, unsigned long long* s0,
                                                          unsigned long long* s1, Sched* sc, uint32_t n_tiles,
                                                          int per, Ctrl* c) {
    __shared__ uint32_t s_rcount[kCompactMaxPerThread][kCompactBlock / 64];
    __shared__ unsigned long long s_wave[kCompactBlock / 64];
    __shared__ unsigned long long s_pre0;
    __shared__ uint32_t s_tile;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    if (t == 0) s_tile = (uint32_t)atomicAdd(&sc->cticket, 1ull);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int shift = c->geo.shift;
    // thread t looks at slots base + r*512 + t, r < per (coalesced); row r
    // precedes row r+1 in slot order
    const uint32_t base = tile * (uint32_t)(kCompactBlock * per);
    uint32_t homed[kCompactMaxPerThread], excl[kCompactMaxPerThread];
#pragma unroll
    for (int r = 0; r < kCompactMaxPerThread; ++r) homed[r] = 0;
    unsigned long long n_rec = 0;
    // rows in batches of four, each record's first three quarters loaded
    // whatever its key (one line either way), so that a batch's loads are
    // all in flight together
#pragma unroll
    for (int r0 = 0; r0 < kCompactMaxPerThread; r0 += 4) {
        if (r0 >= per) break;
        uint4 q0[4], q1[4], q2[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t s = base + (r0 + j) * kCompactBlock + t;
            const bool in = r0 + j < per && s < cap;
            const uint4* pq = reinterpret_cast<const uint4*>(rec + (in ? s : 0u));
            q0[j] = pq[0];
            q1[j] = pq[1];
            q2[j] = pq[2];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + j;
            const uint32_t s = base + r * kCompactBlock + t;
            if (r >= per || s >= cap) continue;
            const uint64_t key = ((uint64_t)q2[j].y << 32) | q2[j].x;
            homed[r] = q2[j].z + (key != kEmpty && slot_of(key, shift) == s ? 1u : 0u);
            if (key == kEmpty) continue;
            const float a[8] = {__uint_as_float(q0[j].x), __uint_as_float(q0[j].y), __uint_as_float(q0[j].z),
                                __uint_as_float(q0[j].w), __uint_as_float(q1[j].x), __uint_as_float(q1[j].y),
                                __uint_as_float(q1[j].z), __uint_as_float(q1[j].w)};
            uint32_t leaves = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) leaves += a[c] == a[c] ? 1u : 0u;
            // records in the low 29 bits, leaves above (cap <= 2^28 keeps them apart)
            n_rec += 1ull + ((unsigned long long)leaves << 29);
        }
    }
    // per row, each lane's keys before its own within the wave (a ballot
    // when no slot of the row is home to two or more keys, else a scan)
#pragma unroll
    for (int r = 0; r < kCompactMaxPerThread; ++r) {
        if (r >= per) break;
        const uint32_t x = homed[r];
        const unsigned long long any = __ballot(x != 0), multi = __ballot(x > 1);
        uint32_t tot;
        if (multi == 0) {
            excl[r] = (uint32_t)__popcll(any & below);
            tot = (uint32_t)__popcll(any);
        } else {
            const unsigned long long incl = wave_incl_scan((unsigned long long)x);
            excl[r] = (uint32_t)incl - x;
            tot = (uint32_t)__shfl(incl, 63, 64);
        }
        if (lane == 0) s_rcount[r][wave] = tot;
    }
    unsigned long long recs = wave_reduce((unsigned long long)n_rec,
                                          [](unsigned long long x, unsigned long long y) { return x + y; });
    if (lane == 0) s_wave[wave] = recs;
    __syncthreads();
    uint32_t total_g = 0;
    unsigned long long total_r = 0;
    for (int r = 0; r < per; ++r)
        for (int w = 0; w < kCompactBlock / 64; ++w) total_g += s_rcount[r][w];
    for (int w = 0; w < kCompactBlock / 64; ++w) total_r += s_wave[w];
    if (wave == 0) {
        unsigned long long p0, p1;
        lookback(s0, s1, tile, 0ull, total_g, total_r, p0, p1);
        if (lane == 0) {
            s_pre0 = p0;
            if (tile == n_tiles - 1) {
                c->n_groups = p0 + total_g;
                c->n_records = (p1 + total_r) & ((1ull << 29) - 1);
                c->n_leaves = (p1 + total_r) >> 29;
            }
        }
    }
    __syncthreads();
    uint32_t row = (uint32_t)s_pre0;
#pragma unroll
    for (int r = 0; r < kCompactMaxPerThread; ++r) {
        if (r >= per) break;
        uint32_t before = 0, in_row = 0;
        for (int w = 0; w < kCompactBlock / 64; ++w) {
            if (w < wave) before += s_rcount[r][w];
            in_row += s_rcount[r][w];
        }
        const uint32_t n_here = homed[r];
        if (n_here) {
            const uint32_t h = base + r * kCompactBlock + t;
            const uint32_t pos = row + before + excl[r];
            const uint64_t k0 = rec[h].key;
            if (n_here == 1 && slot_of(k0, shift) == h) {
                glist[pos] = (int32_t)h;
                gkey[pos] = k0;  // beside the slot, so extraction needs no dependent load
            } else {
                // the keys homed here, smallest first: one walk of the probe
                // sequence per key, each taking the least key above the last
                uint64_t last = 0;
                for (uint32_t q = 0; q < n_here; ++q) {
                    uint64_t best = kEmpty;
                    uint32_t best_slot = h, seen = 0, x = h;
                    for (uint32_t step = 0; step < kMaxProbe && seen < n_here; ++step) {
                        const uint64_t k = rec[x].key;
                        if (k == kEmpty) break;
                        if (slot_of(k, shift) == h) {
                            ++seen;
                            if ((q == 0 || k > last) && k < best) {
                                best = k;
                                best_slot = x;
                            }
                        }
                        x = next_slot(x, step, cap - 1);
                    }
                    if (best == kEmpty) {  // cannot happen while the counts hold
                        atomicOr(&c->overflow, 1u);
                        break;
                    }
                    glist[pos + q] = (int32_t)best_slot;
                    gkey[pos + q] = best;
                    last = best;
                }
            }
        }
        row += in_row;
    }
}

// ---------------------------------------------------------------------------
// Extraction
// ---------------------------------------------------------------------------

struct ExtractArgs {
    const Record* rec;
    const int32_t* ids;
    const int32_t* glist;
    const unsigned long long* gkey;
    const Ctrl* ctrl;  // build verdict, group count and geometry (written by the build's kernels)
    float iso;
    // iso-surface outputs
    float* tris;
    int32_t* tri_cells;
    int64_t* tri_dual;
    // dual-cell outputs
    int32_t* corner_level;
    int32_t* verts;
    float* dvals;
    int64_t cap;
    int64_t* counts;
    unsigned long long* tot;    // per tile: triangles << 32 | duals (count pass)
    unsigned long long* gcnt;   // per group: triangles << 32 | duals (count pass)
    unsigned long long* pre_t;  // per tile: exclusive prefix of triangles (scan)
    unsigned long long* pre_d;  // per tile: exclusive prefix of duals (scan)
    unsigned long long* sc0;    // per scan tile: look-back states
    unsigned long long* sc1;
    Sched* sched;
    uint32_t n_scan_tiles;  // work-groups of the scan launch (their look-back states)
    // value range of each group's 4x4x4 neighbourhood (min, max over its
    // cells), recorded by the second extraction after a build and then used
    // to skip groups in iso-surface passes; the set's dual count goes with
    // it, and sched->rng_ok says both are there (the host only asks for
    // culling; without recorded ranges the kernels run full passes)
    float2* rng;
    unsigned long long* dual_total;
    int rng_mode;
    int list_from_cull;  // the list passes run over culled candidates (dual count: the recorded one)
    // group list of a list count / write pass (k_group_list); with lcnt the
    // list's triangle counts come from there (no list count pass), and
    // list_duals holds the set's dual count
    const uint32_t* clist;
    const unsigned long long* n_list;
    const uint32_t* lcnt;
    const unsigned long long* list_duals;
};

enum : int { kRngNone = 0, kRngRecord = 1, kRngCull = 2 };

// Hexahedron edge e -> lower slot (upper slot = lower | (1 << axis)).  Edges
// 0-3 run along x, 4-7 along y, 8-11 along z; the i-th edge of an axis starts
// at the slot whose bits are i with a 0 inserted at that axis:
// x: 0,2,4,6   y: 0,1,4,5   z: 0,1,2,3
__host__ __device__ constexpr int edge_lo(int e) {
    return (((e & 3) >> (e >> 2)) << ((e >> 2) + 1)) | ((e & 3) & ((1 << (e >> 2)) - 1));
}
__host__ __device__ constexpr int edge_hi(int e) { return edge_lo(e) | (1 << (e >> 2)); }

// The 27 corners of a group's 2x2x2 block, k = kx + 3 ky + 9 kz with
// kx, ky, kz in {0, 1, 2}, in the order the eight lanes of a group take them:
// first the 8 corners whose slot 0 lies inside the group (kx, ky, kz >= 1:
// the ones the group usually owns), then the other 19 in increasing order,
// which a dense neighbourhood settles after one look at slot 0.  That keeps
// whole waves on the same side of that early exit.
struct CornerOrder {
    unsigned long long lo = 0, hi = 0;  // 5 bits per corner, 12 + 7 corners
    constexpr CornerOrder() {
        int r = 0;
        for (int k = 0; k < 27; ++k) {
            const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
            if (kx >= 1 && ky >= 1 && kz >= 1) continue;
            if (r < 12) lo |= (unsigned long long)k << (5 * r);
            else hi |= (unsigned long long)k << (5 * (r - 12));
            ++r;
        }
    }
};
constexpr CornerOrder kCornerOrder{};

__device__ __forceinline__ int corner_of(int idx) {
    if (idx < 8) return 13 + (idx & 1) + 3 * ((idx >> 1) & 1) + 9 * (idx >> 2);
    const int r = idx - 8;
    return r < 12 ? (int)((kCornerOrder.lo >> (5 * r)) & 31) : (int)((kCornerOrder.hi >> (5 * (r - 12))) & 31);
}

// Degenerate duals: a cell may sit at several slots.  A triangle is kept when
// its three vertices join three different (unordered) cell pairs.  Each slot
// gets the lowest slot holding the same cell as its class (3 bits per slot);
// a vertex is the unordered class pair of its edge.
__device__ __forceinline__ uint32_t slot_classes(const int (&refs)[8]) {
    uint32_t cls = 0;
#pragma unroll
    for (int s1 = 1; s1 < 8; ++s1) {
        int c = s1;
#pragma unroll
        for (int s0 = s1 - 1; s0 >= 0; --s0)
            if (refs[s0] == refs[s1]) c = s0;
        cls |= (uint32_t)c << (3 * s1);
    }
    return cls;
}

// Keep mask of the nt triangles in e (three 4-bit edges per 12 bits).
__device__ __forceinline__ uint32_t keep_by_classes(uint32_t cls, unsigned long long e, int nt) {
    uint32_t keep = 0;
    for (int tt = 0; tt < nt; ++tt) {
        uint32_t pr[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const int ed = (int)((e >> (12 * tt + 4 * v)) & 0xF);
            const uint32_t a = (cls >> (3 * edge_lo(ed))) & 7u, b = (cls >> (3 * edge_hi(ed))) & 7u;
            pr[v] = a < b ? (a << 3) | b : (b << 3) | a;
        }
        if (pr[0] != pr[1] && pr[1] != pr[2] && pr[0] != pr[2]) keep |= 1u << tt;
    }
    return keep;
}


// Phase 1 of a tile for one group (called by its eight lanes, j = 0..7):
// the level-m cells of the 4x4x4 block around the group (offsets -1..2
// from its lower corner, x fastest) into the group's LDS rows: value, cell
// reference (slot * 8 + child), level of the cell that covers the position
// (-1: none).  kWalk home slots of coarser levels are read at once when a
// neighbour block holds no level-m record.
template <int kWalk>
__device__ __forceinline__ void load_neighbourhood(const Record* __restrict__ rec, const Geo& g, const int j,
                                                   const int m, const uint32_t gx, const uint32_t gy,
                                                   const uint32_t gz, const int own, float* sv, int32_t* sr,
                                                   int8_t* sl) {
    // lane j owns neighbours j, j+8, j+16 (and j+24 for j < 3); the home
    // slots of all of them are loaded before any is examined
    uint64_t want[4], got[4];
    uint32_t home[4];
    float4 va[4], vb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int dd = j + 8 * q;
        if (dd >= 27) continue;
        int dx = dd % 3 - 1, dy = (dd / 3) % 3 - 1, dz = dd / 9 - 1;
        want[q] = group_key(m, gx + dx, gy + dy, gz + dz);
        home[q] = dd == 13 ? (uint32_t)own : slot_of(want[q], g.shift);
        const Record* r = rec + home[q];
        va[q] = reinterpret_cast<const float4*>(r->val)[0];
        vb[q] = reinterpret_cast<const float4*>(r->val)[1];
        got[q] = r->key;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int dd = j + 8 * q;
        if (dd >= 27) continue;
        int lv = -1, ref = -1;
        uint32_t h = home[q];
        uint64_t k = got[q];
        float4 xa = va[q], xb = vb[q];
        if (k != want[q] && k != kEmpty) {
            for (uint32_t step = 0; k != want[q] && k != kEmpty && step <= g.mask; ++step) {
                h = next_slot(h, step, g.mask);
                k = rec[h].key;
            }
            if (k == want[q]) {
                xa = reinterpret_cast<const float4*>(rec[h].val)[0];
                xb = reinterpret_cast<const float4*>(rec[h].val)[1];
            }
        }
        float cv = 0.f;
        const bool hit = k == want[q];
        if (hit) {
            lv = m;
        } else {
            // The block holds neither cells of level m nor finer cells (either
            // would have left a record): it lies inside a coarser cell or in a
            // hole.  The first record found going up decides; kWalk levels
            // are read per memory round trip.
            int dx = dd % 3 - 1, dy = (dd / 3) % 3 - 1, dz = dd / 9 - 1;
            uint32_t bx = gx + dx, by = gy + dy, bz = gz + dz;
            // Each level's home slot is read with the one child value the
            // block would need there (same line), so a record found at its
            // home slot costs no further round trip.
            int found_l = -1, found_h = -1, found_c = 0;
            float found_v = 0.f;
            for (int L0 = m + 1; L0 <= g.lmax && found_l < 0; L0 += kWalk) {
                uint64_t wk[kWalk], kk[kWalk];
                uint32_t hh[kWalk];
                int ch[kWalk];
                float vv[kWalk];
#pragma unroll
                for (int u = 0; u < kWalk; ++u) {
                    const int L = L0 + u, sh = L - m - 1;
                    wk[u] = group_key(L, bx >> (sh + 1), by >> (sh + 1), bz >> (sh + 1));
                    hh[u] = slot_of(wk[u], g.shift);
                    ch[u] = ((bx >> sh) & 1) | (((by >> sh) & 1) << 1) | (((bz >> sh) & 1) << 2);
                    kk[u] = kEmpty;
                    vv[u] = 0.f;
                    if (L <= g.lmax) {
                        kk[u] = rec[hh[u]].key;
                        vv[u] = rec[hh[u]].val[ch[u]];
                    }
                }
#pragma unroll
                for (int u = 0; u < kWalk; ++u) {
                    if (found_l >= 0 || L0 + u > g.lmax) continue;
                    uint32_t h2 = hh[u];
                    uint64_t k2 = kk[u];
                    float v2 = vv[u];
                    if (k2 != wk[u] && k2 != kEmpty) {
                        for (uint32_t step = 0; k2 != wk[u] && k2 != kEmpty && step <= g.mask; ++step) {
                            h2 = next_slot(h2, step, g.mask);
                            k2 = rec[h2].key;
                        }
                        if (k2 == wk[u]) v2 = rec[h2].val[ch[u]];
                    }
                    if (k2 == wk[u]) {
                        found_l = L0 + u;
                        found_h = (int)h2;
                        found_c = ch[u];
                        found_v = v2;
                    }
                }
            }
            // the lowest level with a record decides (a NaN there: finer
            // cells or none at all, either way no cell covers this block)
            if (found_l >= 0 && found_v == found_v) {
                lv = found_l;
                ref = found_h * 8 + found_c;
                cv = found_v;
            }
        }
        // the cells of this neighbour that lie in the 4x4x4 block
        const float v8[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
        const int dx = dd % 3 - 1, dy = (dd / 3) % 3 - 1, dz = dd / 9 - 1;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int chx = c & 1, chy = (c >> 1) & 1, chz = c >> 2;
            const bool need = (dx == 0 || (dx < 0) == (chx == 1)) && (dy == 0 || (dy < 0) == (chy == 1)) &&
                              (dz == 0 || (dz < 0) == (chz == 1));
            if (!need) continue;
            const int p = (2 * dx + chx + 1) + 4 * (2 * dy + chy + 1) + 16 * (2 * dz + chz + 1);
            sv[p] = hit ? v8[c] : cv;
            sr[p] = hit ? (int)h * 8 + c : ref;
            sl[p] = (int8_t)lv;
        }
    }
}

// Phase 2 of a tile for lane j of one group: the corners j, j+8, j+16 (and
// j+24) of the group's 27 (order: corner_of).  A corner's dual is emitted
// when its 8 slots hold cells of level m or coarser (rules 1 and 2) and the
// lowest same-level slot lies in this group (rule 3); for iso-surfaces its
// Marching Cubes case and the mask of kept triangles follow.  items[q]:
// bit 31 emitted | corner << 20 | case << 8 | keep mask.
template <bool kDuals>
__device__ __forceinline__ void corner_items(const int j, const int m, const float iso, const float* sv,
                                             const int32_t* sr, const int8_t* sl,
                                             const unsigned long long* s_tab, const bool work,
                                             uint32_t (&items)[4], int& n_dual, int& n_tri) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        items[q] = 0;
        const int idx = j + 8 * q;
        if (!work || idx >= 27) continue;
        const int k = corner_of(idx);
        const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
        const int p0 = kx + 4 * ky + 16 * kz;  // slot 0's cell; slot s adds ex + 4 ey + 16 ez
        // Slot 0 decides most corners: a level-m cell there outside this
        // group is the lowest same-level slot, so the dual belongs to another
        // group (or is rejected by rule 2 when that cell is refined)
        if ((kx == 0 || ky == 0 || kz == 0) && sl[p0] == m) continue;
        int refs[8];
        float vals[8];
        bool ok = true;
        uint32_t same = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int p = p0 + (s & 1) + 4 * ((s >> 1) & 1) + 16 * (s >> 2);
            const int lv = sl[p];
            const float v = sv[p];
            refs[s] = sr[p];
            vals[s] = v;
            // rule 1 (hole) and rule 2 (finer cells) both show as lv < 0 or a NaN
            ok = ok && lv >= 0 && v == v;
            same |= (lv == m ? 1u : 0u) << s;
        }
        // the slots inside this group (cell positions 1..2 on every axis):
        // on an axis where the corner sits at 0 only e = 1, at 2 only e = 0
        const uint32_t mine = (kx == 0 ? 0xAAu : kx == 1 ? 0xFFu : 0x55u) &
                              (ky == 0 ? 0xCCu : ky == 1 ? 0xFFu : 0x33u) &
                              (kz == 0 ? 0xF0u : kz == 1 ? 0xFFu : 0x0Fu);
        // rule 3: the lowest same-level slot must be a cell of this group
        if (!ok || !(same & (0u - same) & mine)) continue;
        ++n_dual;
        uint32_t cs = 0, keep = 0;
        if (!kDuals) {
#pragma unroll
            for (int s = 0; s < 8; ++s) cs |= (vals[s] >= iso ? 1u : 0u) << s;
            unsigned long long e = s_tab[cs];
            int nt = (int)(e >> 60);
            if (nt) {
                keep = (1u << nt) - 1u;
                // eight level-m slots are eight different cells: nothing to drop;
                // otherwise drop triangles whose vertices repeat a cell pair
                if (same != 0xFFu) keep = keep_by_classes(slot_classes(refs), e, nt);
                n_tri += __popc(keep);
            }
        }
        items[q] = 0x80000000u | ((uint32_t)k << 20) | (cs << 8) | keep;
    }
}

// Phase 3 of a tile, triangles: every kept triangle gets an entry (owner
// lane, item, triangle) in an LDS list, in output order, and the block's
// lanes take entries round-robin; long tiles go through the list in chunks.
// Called by the whole work-group (kB lanes, eight per group) after the
// block scan: my_first = the lane's first triangle within the tile,
// dual_first its first emitted dual, pre_t / pre_d the tile's first output
// positions.  Triangles at positions >= cap are not written.
template <int kB>
__device__ __forceinline__ void write_triangles(const int t, const Geo& g, const float iso, const int gi, const int j,
                                                const int m,
                                                const uint32_t gx, const uint32_t gy, const uint32_t gz,
                                                const uint32_t (&items)[4], const uint32_t tile_tris,
                                                const uint32_t my_first, const uint32_t dual_first,
                                                const int64_t pre_t, const int64_t pre_d, const int64_t cap,
                                                float* tris, int32_t* tri_cells, int64_t* tri_dual,
                                                const int32_t* ids, const float (*s_v)[64],
                                                const int32_t (*s_r)[64], const int8_t (*s_l)[64],
                                                const unsigned long long* s_tab, uint32_t (*s_items)[4],
                                                uint32_t* s_dual, uint32_t* s_list, int* s_gm,
                                                uint32_t (*s_gx)[3]) {
    if (j == 0) {
        s_gm[gi] = m;
        s_gx[gi][0] = gx;
        s_gx[gi][1] = gy;
        s_gx[gi][2] = gz;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s_items[t][q] = items[q];
    s_dual[t] = dual_first;
    for (uint32_t c0 = 0; c0 < tile_tris; c0 += kTriList) {
        __syncthreads();
        // publish my triangles that fall into [c0, c0 + kTriList)
        uint32_t idx = my_first;
        for (int q = 0; q < 4; ++q) {
            uint32_t it = items[q];
            uint32_t keep = it & 0x1F;
            for (int tt = 0; tt < 5; ++tt) {
                if (!((keep >> tt) & 1)) continue;
                if (idx >= c0 && idx < c0 + kTriList) s_list[idx - c0] = ((uint32_t)t << 8) | (q << 4) | tt;
                ++idx;
            }
        }
        __syncthreads();
        uint32_t n_here = tile_tris - c0 < (uint32_t)kTriList ? tile_tris - c0 : (uint32_t)kTriList;
        for (uint32_t w = t; w < n_here; w += kB) {
            uint32_t en = s_list[w];
            int owner = (int)(en >> 8), q = (int)((en >> 4) & 3), tt = (int)(en & 15);
            int og = owner >> 3;
            uint32_t it = s_items[owner][q];
            int k = (it >> 20) & 31;
            int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
            int om = s_gm[og];
            uint32_t gg[3] = {s_gx[og][0], s_gx[og][1], s_gx[og][2]};
            unsigned long long e = s_tab[(it >> 8) & 0xFF];
            int64_t o_t = pre_t + c0 + w;
            if (o_t >= cap) continue;
            float p[9];
            int cells[6];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                int ed = (int)((e >> (12 * tt + 4 * v)) & 0xF);
                float ev[2];
                int el[2], er[2], epos[2][3];
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    int sl = side ? edge_hi(ed) : edge_lo(ed);
                    const int p = (kx + (sl & 1)) + 4 * (ky + ((sl >> 1) & 1)) + 16 * (kz + (sl >> 2));
                    ev[side] = s_v[og][p];
                    er[side] = s_r[og][p];
                    el[side] = s_l[og][p];
                    epos[side][0] = kx + (sl & 1) - 1;
                    epos[side][1] = ky + ((sl >> 1) & 1) - 1;
                    epos[side][2] = kz + ((sl >> 2) & 1) - 1;
                }
                // A = the end below iso, B = the end at or above it
                const bool swap = ev[0] >= iso;
                const float va = swap ? ev[1] : ev[0], vb = swap ? ev[0] : ev[1];
                const int la = swap ? el[1] : el[0], lb = swap ? el[0] : el[1];
                float tp = (iso - va) / (vb - va);
                const int oo[3] = {g.ox, g.oy, g.oz};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    int ra = swap ? epos[1][ax] : epos[0][ax], rb = swap ? epos[0][ax] : epos[1][ax];
                    // finest-unit offset coordinate of the slot position, floored to the cell's level
                    uint32_t pa = ((2 * gg[ax] + (uint32_t)ra) << om) & ~((1u << la) - 1u);
                    uint32_t pb = ((2 * gg[ax] + (uint32_t)rb) << om) & ~((1u << lb) - 1u);
                    float ca = (float)((int)pa + oo[ax]) + 0.5f * (float)(1 << la);
                    float cb = (float)((int)pb + oo[ax]) + 0.5f * (float)(1 << lb);
                    p[3 * v + ax] = fmaf(tp, cb - ca, ca);
                }
                cells[2 * v] = swap ? er[1] : er[0];
                cells[2 * v + 1] = swap ? er[0] : er[1];
            }
            if (tris) {
                float* o = tris + 9 * o_t;
#pragma unroll
                for (int c = 0; c < 9; ++c) o[c] = p[c];
            }
            if (tri_cells) {
                int32_t* o = tri_cells + 6 * o_t;
#pragma unroll
                for (int c = 0; c < 6; ++c) o[c] = ids[cells[c]];
            }
            if (tri_dual) {
                // the owner lane's emitted duals before item q
                uint32_t rank = 0;
                for (int q2 = 0; q2 < q; ++q2) rank += s_items[owner][q2] >> 31;
                tri_dual[o_t] = pre_d + s_dual[owner] + rank;
            }
        }
    }
}

// Extraction of a large set runs as three launches: a count pass (phases
// 1-2, per-tile totals), a scan of the tile totals, and a write pass that
// repeats phases 1-2 for the tiles that have output below the capacity and
// writes it at the scanned positions; no tile waits for another in the heavy
// passes.  A small set (few tiles, where a global ticket per tile is cheap)
// runs one fused pass: tiles take tickets in start order and find their
// output position by a decoupled look-back over earlier tickets.
enum : int { kPassCount = 0, kPassWrite = 1, kPassFused = 2 };

// One tile of 32 groups: all of them (group index = tile * 32 + i, n_groups
// in all, n_tiles tiles) or, with kList, 32 entries of the candidate list of
// an iso-value (n_list long).  `call` is the fused pass's call number and
// `rng_mode` the effective range mode (culling only when ranges are
// recorded).  Every return is taken by the whole work-group.
template <bool kDuals, int kPass, bool kList>
__device__ __forceinline__ void extract_tile(const ExtractArgs& a, const Geo& g, const uint32_t n_groups,
                                             const uint32_t n_tiles, const uint32_t tile, const uint32_t n_list,
                                             const unsigned long long call, const int rng_mode) {
    // the 4x4x4 cells of level m around each group (offsets -1..2 from its
    // lower corner, x fastest): value, cell reference, level of the cell that
    // covers the position (-1: none)
    __shared__ float s_v[kGroupsPerTile][64];
    __shared__ int32_t s_r[kGroupsPerTile][64];
    __shared__ int8_t s_l[kGroupsPerTile][64];
    __shared__ unsigned long long s_tab[256];
    __shared__ unsigned long long s_wave[kBlock / 64];
    __shared__ unsigned long long s_pre_t, s_pre_d;
    __shared__ uint32_t s_items[kBlock][4];
    __shared__ uint32_t s_dual[kBlock];
    __shared__ uint32_t s_list[kTriList];
    __shared__ int s_gm[kGroupsPerTile];
    __shared__ uint32_t s_gx[kGroupsPerTile][3];

    const int t = threadIdx.x;
    const int gi = t >> 3;  // group within the tile
    const int j = t & 7;    // lane within the group
    if (kPass == kPassWrite) {
        // nothing of this tile lands below the capacity: done
        const unsigned long long tt = a.tot[tile];
        const unsigned long long mine_n = kDuals ? (tt & 0xFFFFFFFFull) : (tt >> 32);
        const unsigned long long mine_pre = kDuals ? a.pre_d[tile] : a.pre_t[tile];
        if (mine_n == 0 || (int64_t)mine_pre >= a.cap) return;
        if (t == 0) {
            s_pre_t = a.pre_t[tile];
            s_pre_d = a.pre_d[tile];
        }
    }
    if (!kDuals) s_tab[t] = kMcTable[t];
    __syncthreads();
    uint32_t gidx;
    bool valid;
    if (kList) {
        const uint32_t li = tile * kGroupsPerTile + gi;
        valid = li < n_list;
        gidx = valid ? a.clist[li] : 0u;
    } else {
        gidx = tile * kGroupsPerTile + gi;
        valid = gidx < n_groups;
    }

    // In the write pass a group with nothing to write this time needs no
    // neighbourhood: it only brings its dual count (from the count pass) to
    // the scan, through its first lane.
    bool work = valid;
    uint32_t carried_duals = 0;
    if (kPass == kPassWrite && valid) {
        const unsigned long long gc = a.gcnt[gidx];
        if ((kDuals ? (gc & 0xFFFFFFFFull) : (gc >> 32)) == 0) {
            work = false;
            carried_duals = j == 0 ? (uint32_t)(gc & 0xFFFFFFFFull) : 0u;
        }
    }
    // A group whose neighbourhood values all lie on one side of iso has only
    // Marching Cubes cases 0 and 255 at its corners: no triangles.  (Its
    // duals are not counted here; the set's total was recorded.)  The count
    // and write passes get such groups filtered out beforehand (kList).
    const bool cull = !kDuals && kPass == kPassFused && rng_mode == kRngCull;
    if (cull && valid) {
        const float2 r = a.rng[gidx];
        work = r.x < a.iso && r.y >= a.iso;
    }

    int m = 0;
    uint32_t gx = 0, gy = 0, gz = 0;
    int own = 0;
    if (work) {
        own = a.glist[gidx];
        uint64_t key = a.gkey[gidx];
        m = (int)(key >> 57);
        gx = (uint32_t)(key & 0x7FFFF);
        gy = (uint32_t)((key >> 19) & 0x7FFFF);
        gz = (uint32_t)((key >> 38) & 0x7FFFF);
    }

    // ---- phase 1: the 27 neighbouring groups of this group, into LDS ----
    // (in the fused pass -- small sets, one wave of tiles: latency bound --
    // the home slots of four coarser levels are read at once; the
    // throughput passes walk one level at a time, which keeps their register
    // count, and occupancy, down)
    if (work) load_neighbourhood<kPass == kPassFused ? 4 : 1>(a.rec, g, j, m, gx, gy, gz, own, s_v[gi], s_r[gi], s_l[gi]);
    __syncthreads();
    if (kPass != kPassWrite && rng_mode == kRngRecord) {
        // the range of the cells in the neighbourhood (holes and the markers
        // of refined or empty slots excluded); lane j takes 8 of the 64
        float lo = INFINITY, hi = -INFINITY;
        if (work) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float v = s_v[gi][8 * j + c];
                if (s_l[gi][8 * j + c] >= 0 && v == v) {
                    lo = fminf(lo, v);
                    hi = fmaxf(hi, v);
                }
            }
        }
        lo = fminf(lo, __shfl_xor(lo, 1, 64));
        hi = fmaxf(hi, __shfl_xor(hi, 1, 64));
        lo = fminf(lo, __shfl_xor(lo, 2, 64));
        hi = fmaxf(hi, __shfl_xor(hi, 2, 64));
        lo = fminf(lo, __shfl_xor(lo, 4, 64));
        hi = fmaxf(hi, __shfl_xor(hi, 4, 64));
        if (valid && j == 0) a.rng[gidx] = make_float2(lo, hi);
    }

    // ---- phase 2: the 27 corners of the group's 2x2x2 block ----
    uint32_t items[4];  // bit 31 valid | corner k (5 b) << 20 | case << 8 | keep mask (5 b)
    int n_dual = 0, n_tri = 0;
    corner_items<kDuals>(j, m, a.iso, s_v[gi], s_r[gi], s_l[gi], s_tab, work, items, n_dual, n_tri);

    n_dual += (int)carried_duals;
    if (kPass == kPassCount) {
        // the group's totals, for the write pass to skip groups without output
        unsigned long long gsum = ((unsigned long long)n_tri << 32) | (unsigned long long)n_dual;
        gsum += __shfl_xor(gsum, 1, 64);
        gsum += __shfl_xor(gsum, 2, 64);
        gsum += __shfl_xor(gsum, 4, 64);
        if (valid && j == 0) a.gcnt[gidx] = gsum;
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

    if (kPass == kPassCount) {
        if (t == 0) a.tot[tile] = total;
        return;
    }
    if (kPass == kPassFused) {
        if (wave == 0) {
            unsigned long long pre_t, pre_d;
            const unsigned long long agg_t = total >> 32, agg_d = total & 0xFFFFFFFFull;
            // states of the previous call carry the other parity
            const unsigned long long par = (call & 1) ? kParityBit : 0ull;
            lookback(a.sc0, a.sc1, tile, par, agg_t, agg_d, pre_t, pre_d);
            if (lane_id() == 0) {
                s_pre_t = pre_t;
                s_pre_d = pre_d;
                if (tile == n_tiles - 1) {
                    const unsigned long long nd = cull ? *a.dual_total : pre_d + agg_d;
                    if (rng_mode == kRngRecord) {
                        *a.dual_total = nd;
                        a.sched->rng_ok = 1;
                    }
                    if (a.counts) {
                        a.counts[0] = kDuals ? (int64_t)nd : (int64_t)(pre_t + agg_t);
                        a.counts[1] = (int64_t)nd;
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- phase 3: write ----
    if (kDuals) {
        int64_t out_d = (int64_t)s_pre_d + (int64_t)(excl & 0xFFFFFFFFull);
        for (int q = 0; q < 4; ++q) {
            uint32_t it = items[q];
            if (!(it & 0x80000000u)) continue;
            int k = (it >> 20) & 31;
            int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
            if (out_d < a.cap) {
                if (a.corner_level) {
                    int4 pl;
                    pl.x = (int)((2 * gx + kx) << m) + g.ox;
                    pl.y = (int)((2 * gy + ky) << m) + g.oy;
                    pl.z = (int)((2 * gz + kz) << m) + g.oz;
                    pl.w = m;
                    reinterpret_cast<int4*>(a.corner_level)[out_d] = pl;
                }
                if (a.verts) {
                    int id[8];
#pragma unroll
                    for (int s = 0; s < 8; ++s)
                        id[s] = a.ids[s_r[gi][(kx + (s & 1)) + 4 * (ky + ((s >> 1) & 1)) + 16 * (kz + (s >> 2))]];
                    reinterpret_cast<int4*>(a.verts)[2 * out_d] = make_int4(id[0], id[1], id[2], id[3]);
                    reinterpret_cast<int4*>(a.verts)[2 * out_d + 1] = make_int4(id[4], id[5], id[6], id[7]);
                }
                if (a.dvals) {
                    float v[8];
#pragma unroll
                    for (int s = 0; s < 8; ++s)
                        v[s] = s_v[gi][(kx + (s & 1)) + 4 * (ky + ((s >> 1) & 1)) + 16 * (kz + (s >> 2))];
                    reinterpret_cast<float4*>(a.dvals)[2 * out_d] = make_float4(v[0], v[1], v[2], v[3]);
                    reinterpret_cast<float4*>(a.dvals)[2 * out_d + 1] = make_float4(v[4], v[5], v[6], v[7]);
                }
            }
            ++out_d;
        }
        return;
    }
    write_triangles<kBlock>(t, g, a.iso, gi, j, m, gx, gy, gz, items, (uint32_t)(total >> 32), (uint32_t)(excl >> 32),
                            (uint32_t)(excl & 0xFFFFFFFFull), (int64_t)s_pre_t, (int64_t)s_pre_d, a.cap, a.tris,
                            a.tri_cells, a.tri_dual, a.ids, s_v, s_r, s_l, s_tab, s_items, s_dual, s_list, s_gm,
                            s_gx);
}

// What every extraction kernel reads first: the build's verdict, the group
// count and the geometry, written on the device by the build (a failed build
// extracts nothing), and the range mode the ranges on hand allow.
struct TileSetup {
    Geo g;
    uint32_t n_groups, n_tiles;
    bool ok;
    int rng_mode;
};

// Every lane reads the same words; readfirstlane tells the compiler so, which
// keeps them (and all that is derived from them) in scalar registers.
__device__ __forceinline__ int32_t uniform_i32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ __forceinline__ TileSetup tile_setup(const ExtractArgs& a) {
    TileSetup u;
    const Geo g = a.ctrl->geo;
    u.g.ox = uniform_i32(g.ox);
    u.g.oy = uniform_i32(g.oy);
    u.g.oz = uniform_i32(g.oz);
    u.g.lmax = uniform_i32(g.lmax);
    u.g.shift = uniform_i32(g.shift);
    u.g.mask = uniform_u32(g.mask);
    u.ok = uniform_i32(a.ctrl->status) == AMR_OK;
    u.n_groups = u.ok ? uniform_u32((uint32_t)a.ctrl->n_groups) : 0u;
    u.n_tiles = (u.n_groups + kGroupsPerTile - 1) / kGroupsPerTile;
    u.rng_mode = (a.rng_mode == kRngCull && uniform_u32(a.sched->rng_ok) == 0) ? kRngNone : a.rng_mode;
    return u;
}

// Counts of a call that has no tiles: zeros, or -1 after a failed build.
__device__ __forceinline__ void write_empty_counts(const ExtractArgs& a, const TileSetup& u) {
    if (a.counts) {
        a.counts[0] = u.ok ? 0 : -1;
        a.counts[1] = u.ok ? 0 : -1;
    }
    if (u.ok && u.rng_mode == kRngRecord) {
        *a.dual_total = 0;
        a.sched->rng_ok = 1;
    }
}

// The group count is known on the device only.  The host sizes the grids for
// a bound it chose at the build (the build fails if the groups exceed it), so
// every tile has a work-group and work-groups past the last tile leave.
//  - fused pass: tiles are handed out as tickets in start order (a tile's
//    look-back then only waits on tiles that running work-groups hold); each
//    call takes exactly gridDim.x tickets, which numbers the calls and gives
//    the look-back states their parity;
//  - count and write passes: work-groups go round-robin to the 8 XCDs, so
//    XCD x is given the contiguous run of tiles [x*T, (x+1)*T) in order and
//    its L2 sees neighbouring tiles one after another.
template <bool kDuals, int kPass>
__global__ __launch_bounds__(kBlock) void k_extract(ExtractArgs a) {
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_call;
    TileSetup u = tile_setup(a);
    if (kPass == kPassFused) {
        // the host picks this pass only when the bound fits the look-back
        // states of kFusedMaxTiles tiles
        if (u.n_tiles > gridDim.x || u.n_tiles > kFusedMaxTiles) {
            u.ok = false;
            u.n_groups = u.n_tiles = 0;
        }
        if (threadIdx.x == 0) {
            // The call number is read before the ticket: the ticket's address
            // depends on the value read (call >> 63 is always 0), so the read
            // completes first.  By the time the last ticket of this call is
            // taken every work-group of the call has read the number, and its
            // holder may advance it at once for the next call.
            const unsigned long long call = ld_relaxed(&a.sched->fcall);
            const unsigned long long tk = atomicAdd(&a.sched->fticket + (call >> 63), 1ull);
            const unsigned long long tl = tk - call * gridDim.x;
            s_call = call;
            s_tile = tl < gridDim.x ? (uint32_t)tl : 0xFFFFFFFFu;
            if (tl == gridDim.x - 1)
                __hip_atomic_store(&a.sched->fcall, call + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (tl == 0 && u.n_tiles == 0) write_empty_counts(a, u);
        }
        __syncthreads();
        const uint32_t tile = uniform_u32(s_tile);
        if (tile >= u.n_tiles) return;  // past the last tile (or calls overlapping, which they must not)
        extract_tile<kDuals, kPass, false>(a, u.g, u.n_groups, u.n_tiles, tile, 0u, s_call, u.rng_mode);
        return;
    }
    if (kPass == kPassCount) {
        // the scan that follows starts from clean states
        for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n_scan_tiles; i += gridDim.x * kBlock) {
            a.sc0[i] = 0;
            a.sc1[i] = 0;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) a.sched->xticket = 0;
    }
    const uint32_t per_xcd = (u.n_tiles + kXcds - 1) / kXcds;
    const uint32_t k = blockIdx.x / kXcds;
    const uint32_t tile = (blockIdx.x % kXcds) * per_xcd + k;
    if (k < per_xcd && tile < u.n_tiles)
        extract_tile<kDuals, kPass, false>(a, u.g, u.n_groups, u.n_tiles, tile, 0u, 0ull, u.rng_mode);
}

// Lists of groups in group order, for passes that need only some of them:
//  - with `rng`: the candidates of one iso-value, groups whose neighbourhood
//    range straddles iso (all others have only Marching Cubes cases 0 and
//    255);
//  - without: the groups a count pass found triangles in (`gcnt`), with each
//    entry's triangle count beside it (`lcnt`) and the dual count of all
//    groups summed on the way (`n_duals`).
// The compaction is stable, so passes over a list emit the triangles in the
// order passes over all groups would.  Work-groups take tickets in start
// order; each call takes exactly n_wgs of them, so the ticket also gives the
// call's parity for the look-back states.  The last work-group writes the
// list's length.
constexpr int kListPer = 16;  // groups per thread

__global__ __launch_bounds__(kBlock) void k_group_list(const float2* __restrict__ rng,
                                                       const unsigned long long* __restrict__ gcnt,
                                                       const Ctrl* ctrl, float iso, uint32_t n_wgs,
                                                       uint32_t* __restrict__ clist, uint32_t* __restrict__ lcnt,
                                                       unsigned long long* n_list, unsigned long long* n_duals,
                                                       unsigned long long* ls0, unsigned long long* ls1, Sched* sc) {
    __shared__ uint32_t s_row[kListPer][kBlock / 64];
    __shared__ unsigned long long s_dual[kBlock / 64];
    __shared__ unsigned long long s_tk, s_pre;
    const int t = threadIdx.x, wave = t >> 6, lane = lane_id();
    // groups of a good build; without recorded ranges every group is a candidate
    const uint32_t n_groups = ctrl->status == AMR_OK ? (uint32_t)ctrl->n_groups : 0u;
    const bool ranged = rng != nullptr && sc->rng_ok != 0;
    if (t == 0) s_tk = atomicAdd(&sc->lticket, 1ull);
    __syncthreads();
    const unsigned long long tk = s_tk;
    const uint32_t wg = (uint32_t)(tk % n_wgs);
    const unsigned long long par = ((tk / n_wgs) & 1) ? kParityBit : 0ull;
    const uint64_t base = (uint64_t)wg * (kBlock * kListPer);
    const unsigned long long below = (1ull << lane) - 1ull;
    uint32_t keep = 0, rank[kListPer], tris[kListPer];
    unsigned long long duals = 0;
#pragma unroll
    for (int r = 0; r < kListPer; ++r) {
        const uint64_t i = base + (uint64_t)r * kBlock + t;
        bool c = false;
        tris[r] = 0;
        if (i < n_groups) {
            if (ranged) {
                const float2 g = rng[i];
                c = g.x < iso && g.y >= iso;
            } else if (rng) {
                c = true;
            } else {
                const unsigned long long gc = gcnt[i];
                tris[r] = (uint32_t)(gc >> 32);
                duals += gc & 0xFFFFFFFFull;
                c = tris[r] != 0;
            }
        }
        const unsigned long long b = __ballot(c);
        rank[r] = (uint32_t)__popcll(b & below);
        keep |= (c ? 1u : 0u) << r;
        if (lane == 0) s_row[r][wave] = (uint32_t)__popcll(b);
    }
    duals = wave_reduce(duals, [](unsigned long long x, unsigned long long y) { return x + y; });
    if (lane == 0) s_dual[wave] = duals;
    __syncthreads();
    if (wave == 0) {
        uint32_t total = 0;
        for (int r = 0; r < kListPer; ++r)
            for (int q = 0; q < kBlock / 64; ++q) total += s_row[r][q];
        unsigned long long dsum = 0;
        for (int q = 0; q < kBlock / 64; ++q) dsum += s_dual[q];
        unsigned long long p0, p1;
        lookback(ls0, ls1, wg, par, total, dsum, p0, p1);
        if (lane == 0) {
            s_pre = p0;
            if (wg == n_wgs - 1) {
                *n_list = p0 + total;
                if (n_duals) *n_duals = p1 + dsum;
            }
        }
    }
    __syncthreads();
    unsigned long long carry = s_pre;
    for (int r = 0; r < kListPer; ++r) {
        uint32_t wave_pre = 0, row = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            if (q < wave) wave_pre += s_row[r][q];
            row += s_row[r][q];
        }
        if ((keep >> r) & 1) {
            const unsigned long long at = carry + wave_pre + rank[r];
            clist[at] = (uint32_t)(base + (uint64_t)r * kBlock + t);
            if (lcnt) lcnt[at] = tris[r];
        }
        carry += row;
    }
}

// Count and write passes over a group list.  The list's length is known
// only on the device: the grid covers every group, and work-groups past the
// list's last tile leave at once.  As in the passes over all groups, XCD x
// (work-groups go round-robin to the 8 XCDs) gets a contiguous run of the
// list's tiles, so its L2 sees neighbouring groups one after another.
template <int kPass>
__global__ __launch_bounds__(kBlock) void k_extract_list(ExtractArgs a) {
    const TileSetup u = tile_setup(a);
    const uint32_t n = (uint32_t)*a.n_list;
    const uint32_t n_tiles = (n + kGroupsPerTile - 1) / kGroupsPerTile;
    const uint32_t per_xcd = (n_tiles + kXcds - 1) / kXcds;
    if (kPass == kPassCount) {
        // the scan that follows starts from clean states
        for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n_scan_tiles; i += gridDim.x * kBlock) {
            a.sc0[i] = 0;
            a.sc1[i] = 0;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) a.sched->xticket = 0;
    }
    const uint32_t k = blockIdx.x / kXcds;
    const uint32_t tile = (blockIdx.x % kXcds) * per_xcd + k;
    if (k < per_xcd && tile < n_tiles)
        extract_tile<false, kPass, true>(a, u.g, u.n_groups, n_tiles, tile, n, 0ull, u.rng_mode);
}

// ---------------------------------------------------------------------------
// Count passes with one lane per group.  extract_tile gives a group eight
// lanes, which take different neighbours and corners, so where a
// neighbour's children land in the 4x4x4 block and which positions a
// corner reads are run-time values in every lane.  Counting needs less:
// every lane holds one group and walks the same 27 neighbours and 27
// corners in the same order, so all positions are compile-time constants,
// and the block is kept as one byte per position in 16 registers: bit 7 a
// cell of level m or coarser covers the position, bit 6 its value is >=
// iso, bits 0-4 its level above m.  Two slots hold the same cell exactly
// when that level is the same, above m, and their level-m positions fall
// into one cell of it (the references extract_tile compares).  The counts
// equal extract_tile's group for group.
// ---------------------------------------------------------------------------

constexpr uint32_t kPosValid = 0x80u, kPosAbove = 0x40u, kPosLevel = 0x1Fu;
constexpr uint32_t kLaneCountMinGroups = 1u << 21;  // group bound from which full count passes use k_count
constexpr int kCountBatch = 3;  // neighbours whose home slots are read at once (3 of 1, 2, 9 and 27 measured fastest)

template <int p>
__device__ __forceinline__ uint32_t pos_byte(const uint32_t (&pos)[16]) {
    return (pos[p >> 2] >> (8 * (p & 3))) & 0xFFu;
}

// Neighbours d0 .. d0 + kN - 1 (dd = dx+1 + 3 (dy+1) + 9 (dz+1)) of the
// group: the home slots of all of them are read at once, then each one's
// record at level m or, when its block holds no level-m record, the coarser
// cell covering it; the children that lie in the 4x4x4 block go into `pos`.
template <int d0, int kN>
__device__ __forceinline__ void count_neighbours(const Record* __restrict__ rec, const Geo& g, const int m,
                                                 uint32_t gx, uint32_t gy, uint32_t gz, const int own,
                                                 const float iso, uint32_t (&pos)[16], float& lo, float& hi) {
    // computed here, not for all 27 neighbours up front (which would hold
    // them all in registers)
    asm volatile("" : "+v"(gx), "+v"(gy), "+v"(gz));
    uint64_t want[kN], key[kN];
    uint32_t h[kN];
    float4 va[kN], vb[kN];
#pragma unroll
    for (int i = 0; i < kN; ++i) {
        const int dd = d0 + i;
        const int dx = dd % 3 - 1, dy = (dd / 3) % 3 - 1, dz = dd / 9 - 1;
        want[i] = group_key(m, gx + dx, gy + dy, gz + dz);
        h[i] = dd == 13 ? (uint32_t)own : slot_of(want[i], g.shift);
    }
#pragma unroll
    for (int i = 0; i < kN; ++i) {
        va[i] = reinterpret_cast<const float4*>(rec[h[i]].val)[0];
        vb[i] = reinterpret_cast<const float4*>(rec[h[i]].val)[1];
        key[i] = rec[h[i]].key;
    }
#pragma unroll
    for (int i = 0; i < kN; ++i) {
        const int dd = d0 + i;
        const int dx = dd % 3 - 1, dy = (dd / 3) % 3 - 1, dz = dd / 9 - 1;
        const uint32_t bx = gx + dx, by = gy + dy, bz = gz + dz;
        uint64_t k = key[i];
        uint32_t hh = h[i];
        float4 xa = va[i], xb = vb[i];
        if (k != want[i] && k != kEmpty) {
            for (uint32_t step = 0; k != want[i] && k != kEmpty && step <= g.mask; ++step) {
                hh = next_slot(hh, step, g.mask);
                k = rec[hh].key;
            }
            if (k == want[i]) {
                xa = reinterpret_cast<const float4*>(rec[hh].val)[0];
                xb = reinterpret_cast<const float4*>(rec[hh].val)[1];
            }
        }
        const bool hit = k == want[i];
        float cv = 0.f;
        uint32_t cbyte = 0;  // the covering cell's byte when the block holds no level-m record
        if (!hit) {
            // the first record found going up decides (a NaN there: finer
            // cells or none at all, either way no cell covers the block)
            for (int L = m + 1; L <= g.lmax; ++L) {
                const int sh = L - m - 1;
                const uint64_t wk = group_key(L, bx >> (sh + 1), by >> (sh + 1), bz >> (sh + 1));
                const int ch = ((bx >> sh) & 1) | (((by >> sh) & 1) << 1) | (((bz >> sh) & 1) << 2);
                uint32_t h2 = slot_of(wk, g.shift);
                uint64_t k2 = rec[h2].key;
                for (uint32_t step = 0; k2 != wk && k2 != kEmpty && step <= g.mask; ++step) {
                    h2 = next_slot(h2, step, g.mask);
                    k2 = rec[h2].key;
                }
                if (k2 == wk) {
                    cv = rec[h2].val[ch];
                    if (cv == cv) cbyte = kPosValid | (cv >= iso ? kPosAbove : 0u) | (uint32_t)(L - m);
                    break;
                }
            }
            if (cbyte) {
                lo = fminf(lo, cv);
                hi = fmaxf(hi, cv);
            }
        }
        const float v8[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int chx = c & 1, chy = (c >> 1) & 1, chz = c >> 2;
            const bool need = (dx == 0 || (dx < 0) == (chx == 1)) && (dy == 0 || (dy < 0) == (chy == 1)) &&
                              (dz == 0 || (dz < 0) == (chz == 1));
            if (!need) continue;
            const int p = (2 * dx + chx + 1) + 4 * (2 * dy + chy + 1) + 16 * (2 * dz + chz + 1);
            const float v = v8[c];
            uint32_t byte = cbyte;
            if (hit) {
                byte = v == v ? kPosValid | (v >= iso ? kPosAbove : 0u) : 0u;
                if (v == v) {
                    lo = fminf(lo, v);
                    hi = fmaxf(hi, v);
                }
            }
            pos[p >> 2] |= byte << (8 * (p & 3));
        }
    }
    if constexpr (d0 + kN < 27)
        count_neighbours<d0 + kN, (27 - d0 - kN < kN ? 27 - d0 - kN : kN)>(rec, g, m, gx, gy, gz, own, iso, pos,
                                                                          lo, hi);
}

// Corner k (kx, ky, kz in 0..2) of the group's 2x2x2 block: its dual is
// emitted when its 8 slots are covered by cells of level m or coarser and
// the lowest same-level slot lies in the group (rules 1-3); then its
// Marching Cubes case and kept triangles.
template <bool kDuals, int k>
__device__ __forceinline__ void count_corner(const uint32_t (&pos)[16], const int m, const uint32_t gx,
                                             const uint32_t gy, const uint32_t gz,
                                             const unsigned long long* s_tab, int& n_dual, int& n_tri) {
    constexpr int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    constexpr int p0 = kx + 4 * ky + 16 * kz;
    uint32_t b[8];
    b[0] = pos_byte<p0>(pos);
    b[1] = pos_byte<p0 + 1>(pos);
    b[2] = pos_byte<p0 + 4>(pos);
    b[3] = pos_byte<p0 + 5>(pos);
    b[4] = pos_byte<p0 + 16>(pos);
    b[5] = pos_byte<p0 + 17>(pos);
    b[6] = pos_byte<p0 + 20>(pos);
    b[7] = pos_byte<p0 + 21>(pos);
    // a level-m cell at slot 0 outside this group is the lowest same-level
    // slot (the dual is another group's), or slot 0 is not covered
    if constexpr (kx == 0 || ky == 0 || kz == 0)
        if ((b[0] & kPosLevel) == 0) return;
    uint32_t all = kPosValid, same = 0, cs = 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        all &= b[s];
        same |= ((b[s] & kPosLevel) == 0 ? 1u : 0u) << s;
        cs |= ((b[s] >> 6) & 1u) << s;
    }
    constexpr uint32_t mine = (kx == 0 ? 0xAAu : kx == 1 ? 0xFFu : 0x55u) &
                              (ky == 0 ? 0xCCu : ky == 1 ? 0xFFu : 0x33u) &
                              (kz == 0 ? 0xF0u : kz == 1 ? 0xFFu : 0x0Fu);
    if (!all || !(same & (0u - same) & mine)) return;
    ++n_dual;
    if (kDuals) return;
    const unsigned long long e = s_tab[cs];
    const int nt = (int)(e >> 60);
    if (!nt) return;
    uint32_t keep = (1u << nt) - 1u;
    if (same != 0xFFu) {
        // slot classes: the lowest slot holding the same cell
        const uint32_t A[3] = {2 * gx + kx - 1, 2 * gy + ky - 1, 2 * gz + kz - 1};
        uint32_t cls = 0;
#pragma unroll
        for (int s1 = 1; s1 < 8; ++s1) {
            int c = s1;
            const uint32_t d1 = b[s1] & kPosLevel;
#pragma unroll
            for (int s0 = s1 - 1; s0 >= 0; --s0) {
                const uint32_t d0 = b[s0] & kPosLevel;
                bool eq = d0 == d1 && d1 != 0;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax)
                    if (((s0 ^ s1) >> ax) & 1) eq = eq && (((A[ax] + 1) & ((1u << d1) - 1u)) != 0);
                if (eq) c = s0;
            }
            cls |= (uint32_t)c << (3 * s1);
        }
        keep = keep_by_classes(cls, e, nt);
    }
    n_tri += __popc(keep);
}

template <bool kDuals, int k>
__device__ __forceinline__ void count_corners(const uint32_t (&pos)[16], const int m, const uint32_t gx,
                                              const uint32_t gy, const uint32_t gz,
                                              const unsigned long long* s_tab, int& n_dual, int& n_tri) {
    count_corner<kDuals, k>(pos, m, gx, gy, gz, s_tab, n_dual, n_tri);
    if constexpr (k + 1 < 27) count_corners<kDuals, k + 1>(pos, m, gx, gy, gz, s_tab, n_dual, n_tri);
}

// One launch: 256 groups per work-group, XCD x taking a contiguous run of
// work-groups; per group its totals (gcnt), per tile of 32 its totals
// (tot), with recording on the groups' value ranges.  Used for full count
// passes over large sets: there it beats the eight-lanes-per-group pass
// (1.48 against 1.87 ms on a 50.8M-cell set), while on sets of a few
// hundred thousand groups, where one lane per group leaves too few waves to
// hide the probes' latency, it loses (0.29 against 0.19 ms at 2M cells).
template <bool kDuals>
__global__ __launch_bounds__(256) void k_count(ExtractArgs a) {
    __shared__ unsigned long long s_tab[256];
    const TileSetup u = tile_setup(a);
    const int t = threadIdx.x;
    if (!kDuals) s_tab[t] = kMcTable[t];
    // the scan that follows starts from clean states
    for (uint32_t i = blockIdx.x * 256 + t; i < a.n_scan_tiles; i += gridDim.x * 256) {
        a.sc0[i] = 0;
        a.sc1[i] = 0;
    }
    if (blockIdx.x == 0 && t == 0) a.sched->xticket = 0;
    const uint32_t n_items = u.n_groups;
    const uint32_t n_tiles = (n_items + kGroupsPerTile - 1) / kGroupsPerTile;
    const uint32_t n_units = (n_items + 255) / 256;
    const uint32_t per_xcd = (n_units + kXcds - 1) / kXcds;
    const uint32_t kk = blockIdx.x / kXcds;
    const uint32_t unit = (blockIdx.x % kXcds) * per_xcd + kk;
    __syncthreads();
    if (kk >= per_xcd || unit >= n_units) return;
    const uint32_t li = unit * 256 + t;
    const bool valid = li < n_items;
    const bool record = u.rng_mode == kRngRecord;
    uint32_t gidx = 0;
    int m = 0, own = 0;
    uint32_t gx = 0, gy = 0, gz = 0;
    int n_dual = 0, n_tri = 0;
    if (valid) {
        gidx = li;
        own = a.glist[gidx];
        const uint64_t key = a.gkey[gidx];
        m = (int)(key >> 57);
        gx = (uint32_t)(key & 0x7FFFF);
        gy = (uint32_t)((key >> 19) & 0x7FFFF);
        gz = (uint32_t)((key >> 38) & 0x7FFFF);
        uint32_t pos[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) pos[i] = 0;
        float lo = INFINITY, hi = -INFINITY;
        count_neighbours<0, kCountBatch>(a.rec, u.g, m, gx, gy, gz, own, a.iso, pos, lo, hi);
        if (record) a.rng[gidx] = make_float2(lo, hi);
        count_corners<kDuals, 0>(pos, m, gx, gy, gz, s_tab, n_dual, n_tri);
        a.gcnt[gidx] = ((unsigned long long)n_tri << 32) | (unsigned long long)n_dual;
    }
    // per tile of 32 items: half a wave
    unsigned long long sum = ((unsigned long long)n_tri << 32) | (unsigned long long)n_dual;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    const uint32_t tile = (unit * 256 + t) / kGroupsPerTile;
    if ((t & 31) == 0 && tile < n_tiles) a.tot[tile] = sum;
}

// Exclusive scan of the per-tile (triangles, duals) totals of a count pass:
// 1024 tiles per work-group, decoupled look-back across work-groups (tickets
// keep the look-back waiting only on work-groups that already run).  The
// last work-group writes the grand totals.  (Measured: 4 rows per thread
// beat 8 and 16, by 5 us of the 2M-cell octree's 0.26 ms iso call against
// 16; the scan is a chain of dependent round trips, which more, smaller
// work-groups shorten.)
constexpr int kScanPer = 4;

__global__ __launch_bounds__(kBlock) void k_tile_scan(ExtractArgs a, int duals) {
    __shared__ unsigned long long s_row[kScanPer][kBlock / 64];
    __shared__ unsigned long long s_p0, s_p1;
    __shared__ uint32_t s_st;
    const int t = threadIdx.x, wave = t >> 6, lane = lane_id();
    // tile counts are known on the device only
    const TileSetup u = tile_setup(a);
    const uint32_t n_tiles = a.n_list ? (uint32_t)((*a.n_list + kGroupsPerTile - 1) / kGroupsPerTile) : u.n_tiles;
    if (t == 0) s_st = (uint32_t)atomicAdd(&a.sched->xticket, 1ull);
    __syncthreads();
    const uint32_t st = s_st;
    const uint64_t base = (uint64_t)st * (kBlock * kScanPer);
    // row r covers tiles base + r*256 + [0, 256); values are packed
    // triangles << 32 | duals, and no half carries inside one work-group
    // (at most 1024 tiles of at most 4320 triangles each)
    unsigned long long v[kScanPer], incl[kScanPer];
    const uint32_t n_entries = a.lcnt ? (uint32_t)*a.n_list : 0u;
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) {
        uint64_t i = base + (uint64_t)r * kBlock + t;
        if (a.lcnt) {
            // a list tile's triangles: the counts of its 32 entries
            unsigned long long tt = 0;
            if (i < n_tiles) {
                // 16-byte loads (the buffer has a tile of slack past its end)
#pragma unroll
                for (int k = 0; k < kGroupsPerTile; k += 4) {
                    const uint64_t e = i * kGroupsPerTile + k;
                    const uint4 c4 = *reinterpret_cast<const uint4*>(a.lcnt + e);
                    tt += (e < n_entries ? c4.x : 0u) + (e + 1 < n_entries ? c4.y : 0u) +
                          (e + 2 < n_entries ? c4.z : 0u) + (e + 3 < n_entries ? c4.w : 0u);
                }
                a.tot[i] = tt << 32;
            }
            v[r] = tt << 32;
        } else {
            v[r] = i < n_tiles ? a.tot[i] : 0ull;
        }
        incl[r] = wave_incl_scan(v[r]);
        if (lane == 63) s_row[r][wave] = incl[r];
    }
    __syncthreads();
    unsigned long long total = 0;
    for (int r = 0; r < kScanPer; ++r)
        for (int q = 0; q < kBlock / 64; ++q) total += s_row[r][q];
    if (wave == 0) {
        unsigned long long p0, p1;
        lookback(a.sc0, a.sc1, st, 0ull, total >> 32, total & 0xFFFFFFFFull, p0, p1);
        if (lane == 0) {
            s_p0 = p0;
            s_p1 = p1;
            if (st == a.n_scan_tiles - 1) {
                // a pass over a list of candidates counts only their duals: the
                // set's recorded total stands in (without recorded ranges the
                // list held every group, and the count is complete)
                const bool stand_in = a.list_duals && (!a.list_from_cull || u.rng_mode == kRngCull);
                const unsigned long long nd = stand_in ? *a.list_duals : p1 + (total & 0xFFFFFFFFull);
                if (u.ok && u.rng_mode == kRngRecord) {
                    *a.dual_total = nd;
                    a.sched->rng_ok = 1;
                }
                if (a.counts) {
                    a.counts[0] = u.ok ? (int64_t)(duals ? nd : p0 + (total >> 32)) : -1;
                    a.counts[1] = u.ok ? (int64_t)nd : -1;
                }
            }
        }
    }
    __syncthreads();
    const unsigned long long p0 = s_p0, p1 = s_p1;
    unsigned long long carry = 0;
    for (int r = 0; r < kScanPer; ++r) {
        unsigned long long wave_pre = 0, row = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            if (q < wave) wave_pre += s_row[r][q];
            row += s_row[r][q];
        }
        uint64_t i = base + (uint64_t)r * kBlock + t;
        if (i < n_tiles) {
            unsigned long long ex = carry + wave_pre + incl[r] - v[r];
            a.pre_t[i] = p0 + (ex >> 32);
            a.pre_d[i] = p1 + (ex & 0xFFFFFFFFull);
        }
        carry += row;
    }
}

// ---------------------------------------------------------------------------
// Batched iso-surfaces: many (set, iso) jobs in one enqueue.  The dual cells
// do not depend on the field (sec. 4), so a work-group loads the
// neighbourhoods of a unit of groups into LDS once and runs Marching Cubes
// (sec. 5) for every job of the unit's set against them.  Four launches: a
// one-work-group preparation orders the jobs and lays out the per-(job,
// unit) counts; a counting launch (one work-group per unit) counts each
// job's triangles per unit; a scan launch (one work-group per job) turns
// them into output positions; a writing launch loads the units that have
// output again and writes.  A group whose neighbourhood value range
// straddles no job's iso is skipped before its neighbourhood is read when
// the set has recorded ranges (see range culling above), else after.  Every
// job's triangles come out in the order, and with the bits, of
// amr_isosurface on its set.
// ---------------------------------------------------------------------------

constexpr int kMaxJobs = 256;
constexpr int kMaxSets = 256;
constexpr int kMaxUnit = 1024;  // groups per unit, at most

// One set of a batch, as the kernels read it (device table).
struct BatchSet {
    const Record* rec;
    const int32_t* glist;
    const unsigned long long* gkey;
    const Ctrl* ctrl;            // verdict, group count, geometry
    const float2* rng;           // recorded neighbourhood ranges, when *rng_ok
    const uint32_t* rng_ok;
    uint32_t bound;              // groups the set can hold (its extraction grid)
    uint32_t pad;
};

// A valid job, by its rank among the valid jobs (by set, then iso, then index).
struct BatchRank {
    float iso;
    int32_t job;
    int64_t jbase;  // its first per-unit count
};

// The batch's job layout, written by the preparation launch.
struct BatchTab {
    int32_t first[kMaxSets + 1];  // first rank of each set
    int64_t tbase[kMaxSets + 1];  // first global unit of each set
    int64_t jbase[kMaxJobs];      // per job index: first per-unit count (-1: invalid job)
    int64_t jn[kMaxJobs];         // per job index: units of its set
    BatchRank rank[kMaxJobs];
};

struct BatchArgs {
    const BatchSet* sets;
    int n_sets;
    const amr_iso_job* jobs;
    int n_jobs;
    int unit;        // groups per unit (a power of two, 64 .. kMaxUnit)
    int unit_shift;
    float* tris;
    int64_t* counts;
    BatchTab* tab;
    uint32_t* tcnt;  // per (job, unit of its set): triangles
    uint32_t* tpre;  // the same, exclusive prefix over the job's units
};

// exclusive block scan of x (blockDim.x <= 512); returns the prefix, *total = sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_w, uint32_t* total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    unsigned long long incl = wave_incl_scan((unsigned long long)x);
    if (lane == 63) s_w[wave] = (uint32_t)incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) pre += s_w[w];
        tot += s_w[w];
    }
    __syncthreads();
    *total = tot;
    return pre + (uint32_t)incl - x;
}

// A batched launch works through units of consecutive groups of one set.
// A unit's candidates -- the groups whose neighbourhood value range (lo, hi]
// contains some job's iso -- are compacted in LDS in group order, then taken
// kG at a time (a chunk, eight lanes per group), so that sparse candidates
// still fill the work-groups.  The set's isos are sorted ascending; a group
// has triangles only for the isos with lo < iso <= hi, the sorted positions
// [ia, ib).  Without recorded ranges every group is a candidate and its
// range comes from the loaded neighbourhood.
constexpr int kPairWin = 256;  // (group, job) pairs of a chunk listed at a time

template <int kG>
struct BatchTile {
    float v[kG][64];
    int32_t r[kG][64];
    int8_t l[kG][64];
    int16_t ia[kG], ib[kG];
    int gm[kG];            // each chunk group's level and block coordinates
    uint32_t gxyz[kG][3];
    int fa, fb;
    uint16_t cl[kMaxUnit];  // the unit's candidates (group index within the unit)
    uint32_t wc[4];
    // the chunk's (group, job) pairs, job-major, groups in order within a job
    uint32_t pm[kMaxJobs];      // per job (from fa): the chunk groups that straddle it
    uint16_t pb[kMaxJobs + 1];  // per job: its first pair
    uint16_t pair[kPairWin];    // group | job << 5
    // per octet (eight lanes, one pair) of a writing round
    int pg[kG];
    uint32_t pfirst[kG];
    float piso[kG];
    int64_t pbase[kG], pcap[kG];
};

// first sorted position whose iso exceeds x
__device__ __forceinline__ int iso_upper(const float* iso_sorted, int n_iso, float x) {
    int a = 0, b = n_iso;
    while (a < b) {
        const int c = (a + b) >> 1;
        if (iso_sorted[c] > x) b = c;
        else a = c + 1;
    }
    return a;
}

// The candidates of unit `st` (groups st * unit ..) into T.cl; returns their count.
template <int kG>
__device__ __forceinline__ int batch_candidates(const BatchSet& S, uint32_t ng, int64_t st, int unit, bool ranged,
                                                const float* iso_sorted, int n_iso, BatchTile<kG>& T) {
    constexpr int kB = kG * 8;
    const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    int base = 0;
    for (int r0 = 0; r0 < unit; r0 += kB) {
        const int li = r0 + t;
        const int64_t gidx = st * unit + li;
        bool cand = li < unit && gidx < (int64_t)ng;
        if (cand && ranged) {
            const float2 rg = S.rng[gidx];
            cand = iso_upper(iso_sorted, n_iso, rg.x) < iso_upper(iso_sorted, n_iso, rg.y);
        }
        const unsigned long long bal = __ballot(cand);
        if (lane == 0) T.wc[wave] = (uint32_t)__popcll(bal);
        __syncthreads();
        int before = base, total = 0;
        for (int w = 0; w < kB / 64; ++w) {
            if (w < wave) before += T.wc[w];
            total += T.wc[w];
        }
        if (cand) T.cl[before + __popcll(bal & below)] = (uint16_t)li;
        base += total;
        __syncthreads();
    }
    return base;
}

// Chunk c0 of a unit's candidates: their neighbourhoods into LDS, each
// group's [ia, ib) and the union over the chunk (T.fa, T.fb).
template <int kG>
__device__ __forceinline__ void batch_load_chunk(const BatchSet& S, const Geo& g, int64_t st, int unit, int c0,
                                                 int n_c, bool ranged, int gi, int j, const float* iso_sorted,
                                                 int n_iso, BatchTile<kG>& T) {
    const int k = c0 + gi;
    const bool work = k < n_c;
    if (threadIdx.x == 0) {
        T.fa = n_iso;
        T.fb = 0;
    }
    int m = 0;
    uint32_t gx = 0, gy = 0, gz = 0;
    int64_t gidx = 0;
    if (work) {
        gidx = st * unit + T.cl[k];
        const int own = S.glist[gidx];
        const uint64_t key = S.gkey[gidx];
        m = (int)(key >> 57);
        gx = (uint32_t)(key & 0x7FFFF);
        gy = (uint32_t)((key >> 19) & 0x7FFFF);
        gz = (uint32_t)((key >> 38) & 0x7FFFF);
        load_neighbourhood<1>(S.rec, g, j, m, gx, gy, gz, own, T.v[gi], T.r[gi], T.l[gi]);
    }
    if (j == 0) {
        T.gm[gi] = m;
        T.gxyz[gi][0] = gx;
        T.gxyz[gi][1] = gy;
        T.gxyz[gi][2] = gz;
    }
    __syncthreads();
    int ia = 0, ib = 0;
    if (ranged) {
        if (work) {
            const float2 rg = S.rng[gidx];
            ia = iso_upper(iso_sorted, n_iso, rg.x);
            ib = iso_upper(iso_sorted, n_iso, rg.y);
        }
    } else {
        // the range of the cells in the neighbourhood (holes and the markers
        // of refined or empty slots excluded); lane j takes 8 of the 64
        float lo = INFINITY, hi = -INFINITY;
        if (work) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float v = T.v[gi][8 * j + c];
                if (T.l[gi][8 * j + c] >= 0 && v == v) {
                    lo = fminf(lo, v);
                    hi = fmaxf(hi, v);
                }
            }
        }
        lo = fminf(lo, __shfl_xor(lo, 1, 64));
        hi = fmaxf(hi, __shfl_xor(hi, 1, 64));
        lo = fminf(lo, __shfl_xor(lo, 2, 64));
        hi = fmaxf(hi, __shfl_xor(hi, 2, 64));
        lo = fminf(lo, __shfl_xor(lo, 4, 64));
        hi = fmaxf(hi, __shfl_xor(hi, 4, 64));
        if (work) {
            ia = iso_upper(iso_sorted, n_iso, lo);
            ib = iso_upper(iso_sorted, n_iso, hi);
        }
    }
    if (!work) ia = ib = 0;
    if (j == 0) {
        T.ia[gi] = (int16_t)ia;
        T.ib[gi] = (int16_t)ib;
        if (ia < ib) {
            atomicMin(&T.fa, ia);
            atomicMax(&T.fb, ib);
        }
    }
    __syncthreads();
}

// The chunk's (group, job) pairs: per job the groups straddling it (T.pm)
// and, by an exclusive scan over the jobs [fa, fb), each job's first pair
// (T.pb).  Returns the number of pairs.
template <int kG>
__device__ __forceinline__ int batch_pairs(BatchTile<kG>& T, int gi, int j, uint32_t* s_w) {
    constexpr int kB = kG * 8;
    const int t = threadIdx.x;
    const int fa = uniform_i32(T.fa), fb = uniform_i32(T.fb), nf = fb > fa ? fb - fa : 0;
    for (int f = t; f < nf; f += kB) T.pm[f] = 0;
    __syncthreads();
    if (j == 0 && T.ia[gi] < T.ib[gi])
        for (int f = T.ia[gi]; f < T.ib[gi]; ++f) atomicOr(&T.pm[f - fa], 1u << gi);
    __syncthreads();
    uint32_t carry = 0;
    for (int f0 = 0; f0 < nf; f0 += kB) {
        const int f = f0 + t;
        const uint32_t c = f < nf ? (uint32_t)__popc(T.pm[f]) : 0u;
        uint32_t tot;
        const uint32_t pre = block_excl_scan(c, s_w, &tot);
        if (f < nf) T.pb[f] = (uint16_t)(carry + pre);
        carry += tot;
    }
    if (t == 0) T.pb[nf] = (uint16_t)carry;
    __syncthreads();
    return (int)carry;
}

// Pairs [p0, p0 + kPairWin) into T.pair.
template <int kG>
__device__ __forceinline__ void batch_pair_window(BatchTile<kG>& T, int gi, int j, int p0) {
    const int fa = T.fa, ib = T.ib[gi];
    for (int f = T.ia[gi] + j; f < ib; f += 8) {
        const int at = T.pb[f - fa] + __popc(T.pm[f - fa] & ((1u << gi) - 1u)) - p0;
        if (at >= 0 && at < kPairWin) T.pair[at] = (uint16_t)(gi | ((f - fa) << 5));
    }
    __syncthreads();
}

// Triangles of one writing round of a batched launch: as write_triangles,
// with each octet holding its own pair (group T.pg, iso T.piso), the output
// position of the round's triangle 0 were it of the octet's job (T.pbase),
// and the end of that job's capacity (T.pcap).
template <int kG>
__device__ __forceinline__ void write_pair_triangles(const int t, const Geo& g, const uint32_t (&items)[4],
                                                     const uint32_t round_tris, const uint32_t my_first,
                                                     BatchTile<kG>& T, float* tris,
                                                     const unsigned long long* s_tab, uint32_t (*s_items)[4],
                                                     uint32_t* s_list) {
    constexpr int kB = kG * 8;
#pragma unroll
    for (int q = 0; q < 4; ++q) s_items[t][q] = items[q];
    for (uint32_t c0 = 0; c0 < round_tris; c0 += kTriList) {
        __syncthreads();
        uint32_t idx = my_first;
        for (int q = 0; q < 4; ++q) {
            const uint32_t keep = items[q] & 0x1F;
            for (int tt = 0; tt < 5; ++tt) {
                if (!((keep >> tt) & 1)) continue;
                if (idx >= c0 && idx < c0 + kTriList) s_list[idx - c0] = ((uint32_t)t << 8) | (q << 4) | tt;
                ++idx;
            }
        }
        __syncthreads();
        const uint32_t n_here = round_tris - c0 < (uint32_t)kTriList ? round_tris - c0 : (uint32_t)kTriList;
        for (uint32_t w = t; w < n_here; w += kB) {
            const uint32_t en = s_list[w];
            const int owner = (int)(en >> 8), q = (int)((en >> 4) & 3), tt = (int)(en & 15);
            const int oc = owner >> 3, og = T.pg[oc];
            const float iso = T.piso[oc];
            const int64_t o_t = T.pbase[oc] + (int64_t)(c0 + w);
            if (o_t >= T.pcap[oc]) continue;
            const uint32_t it = s_items[owner][q];
            const int k = (it >> 20) & 31;
            const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
            const int om = T.gm[og];
            const uint32_t gg[3] = {T.gxyz[og][0], T.gxyz[og][1], T.gxyz[og][2]};
            const unsigned long long e = s_tab[(it >> 8) & 0xFF];
            float p[9];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const int ed = (int)((e >> (12 * tt + 4 * v)) & 0xF);
                float ev[2];
                int el[2], epos[2][3];
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int sl = side ? edge_hi(ed) : edge_lo(ed);
                    const int pp = (kx + (sl & 1)) + 4 * (ky + ((sl >> 1) & 1)) + 16 * (kz + (sl >> 2));
                    ev[side] = T.v[og][pp];
                    el[side] = T.l[og][pp];
                    epos[side][0] = kx + (sl & 1) - 1;
                    epos[side][1] = ky + ((sl >> 1) & 1) - 1;
                    epos[side][2] = kz + ((sl >> 2) & 1) - 1;
                }
                // A = the end below iso, B = the end at or above it
                const bool swap = ev[0] >= iso;
                const float va = swap ? ev[1] : ev[0], vb = swap ? ev[0] : ev[1];
                const int la = swap ? el[1] : el[0], lb = swap ? el[0] : el[1];
                const float tp = (iso - va) / (vb - va);
                const int oo[3] = {g.ox, g.oy, g.oz};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const int ra = swap ? epos[1][ax] : epos[0][ax], rb = swap ? epos[0][ax] : epos[1][ax];
                    const uint32_t pa = ((2 * gg[ax] + (uint32_t)ra) << om) & ~((1u << la) - 1u);
                    const uint32_t pb = ((2 * gg[ax] + (uint32_t)rb) << om) & ~((1u << lb) - 1u);
                    const float ca = (float)((int)pa + oo[ax]) + 0.5f * (float)(1 << la);
                    const float cb = (float)((int)pb + oo[ax]) + 0.5f * (float)(1 << lb);
                    p[3 * v + ax] = fmaf(tp, cb - ca, ca);
                }
            }
            if (tris) {
                float* o = tris + 9 * o_t;
#pragma unroll
                for (int c = 0; c < 9; ++c) o[c] = p[c];
            }
        }
    }
}

// Values every lane of a work-group holds alike, kept in scalar registers.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    return reinterpret_cast<T*>(uniform_i64((int64_t)reinterpret_cast<uintptr_t>(p)));
}

__device__ __forceinline__ BatchSet uniform_set(const BatchSet& s) {
    BatchSet u;
    u.rec = uniform_ptr(s.rec);
    u.glist = uniform_ptr(s.glist);
    u.gkey = uniform_ptr(s.gkey);
    u.ctrl = uniform_ptr(s.ctrl);
    u.rng = uniform_ptr(s.rng);
    u.rng_ok = uniform_ptr(s.rng_ok);
    u.bound = uniform_u32(s.bound);
    u.pad = 0;
    return u;
}

// Preparation (one work-group of 256): every valid job's rank among the
// valid jobs (by set, then iso, then job index), each set's first rank and
// first global unit, each job's first per-unit count.  A job naming no set
// of the batch, with a non-finite iso, or on a set whose build failed, takes
// part in nothing and counts -1.
__global__ __launch_bounds__(256) void k_batch_prep(BatchArgs a) {
    __shared__ amr_iso_job s_job[kMaxJobs];
    __shared__ int s_ok[kMaxJobs];
    __shared__ int64_t s_units[kMaxSets];
    __shared__ int s_rank[kMaxJobs];
    const int t = threadIdx.x;
    BatchTab* tab = a.tab;
    for (int i = t; i < a.n_sets; i += blockDim.x) {
        const BatchSet& S = a.sets[i];
        const Ctrl* c = S.ctrl;
        int64_t ng = c->status == AMR_OK ? (int64_t)c->n_groups : -1;
        if (ng > (int64_t)S.bound) ng = S.bound;  // cannot happen for a set built once; bounds the layout
        s_units[i] = ng < 0 ? -1 : (ng + a.unit - 1) >> a.unit_shift;
    }
    for (int i = t; i < a.n_jobs; i += blockDim.x) s_job[i] = a.jobs[i];
    __syncthreads();
    for (int i = t; i < a.n_jobs; i += blockDim.x) {
        const int si = s_job[i].set;
        s_ok[i] = si >= 0 && si < a.n_sets && isfinite(s_job[i].iso) && s_units[si] >= 0;
    }
    __syncthreads();
    for (int i = t; i < a.n_jobs; i += blockDim.x) {
        s_rank[i] = -1;
        if (!s_ok[i]) continue;
        const int si = s_job[i].set;
        const float vi = s_job[i].iso;
        int rank = 0;
        for (int k = 0; k < a.n_jobs; ++k) {
            if (!s_ok[k]) continue;
            const int sk = s_job[k].set;
            const float vk = s_job[k].iso;
            rank += sk < si || (sk == si && (vk < vi || (vk == vi && k < i)));
        }
        s_rank[i] = rank;
    }
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int si = 0; si < a.n_sets; ++si) {
            tab->tbase[si] = acc;
            acc += s_units[si] > 0 ? s_units[si] : 0;
        }
        tab->tbase[a.n_sets] = acc;
        int64_t jb = 0;
        for (int i = 0; i < a.n_jobs; ++i) {
            const int64_t n = s_ok[i] ? s_units[s_job[i].set] : 0;
            tab->jbase[i] = s_ok[i] ? jb : -1;
            tab->jn[i] = n;
            jb += n;
        }
    }
    // each set's first rank: the valid jobs on sets before it
    for (int si = t; si <= a.n_sets; si += blockDim.x) {
        int n = 0;
        for (int k = 0; k < a.n_jobs; ++k) n += s_ok[k] && s_job[k].set < si;
        tab->first[si] = n;
    }
    __syncthreads();
    for (int i = t; i < a.n_jobs; i += blockDim.x) {
        if (s_rank[i] < 0) continue;
        BatchRank r;
        r.iso = s_job[i].iso;
        r.job = i;
        r.jbase = tab->jbase[i];
        tab->rank[s_rank[i]] = r;
    }
}

__device__ __forceinline__ Geo batch_geo(const BatchSet& S) {
    Geo g = S.ctrl->geo;
    g.ox = uniform_i32(g.ox);
    g.oy = uniform_i32(g.oy);
    g.oz = uniform_i32(g.oz);
    g.lmax = uniform_i32(g.lmax);
    g.shift = uniform_i32(g.shift);
    g.mask = uniform_u32(g.mask);
    return g;
}

// the set's groups (never more than its bound, as the layout assumes)
__device__ __forceinline__ uint32_t batch_groups(const BatchSet& S) {
    const uint32_t ng = uniform_u32(S.ctrl->n_groups);
    return ng < S.bound ? ng : S.bound;
}

// The unit of global unit index `tile`: its set, the unit within the set,
// the set's ranks [f0, f1) (isos into s_iso); false past the last unit.
__device__ __forceinline__ bool batch_unit(const BatchArgs& a, int64_t tile, int* s_si, float* s_iso, int& si,
                                           int64_t& lt, int& f0, int& f1) {
    const BatchTab* tab = a.tab;
    const int t = threadIdx.x;
    if (t == 0) *s_si = -1;
    __syncthreads();
    for (int i = t; i < a.n_sets; i += blockDim.x)
        if (tab->tbase[i] <= tile && tile < tab->tbase[i + 1]) *s_si = i;
    __syncthreads();
    si = uniform_i32(*s_si);
    if (si < 0) return false;
    lt = uniform_i64(tile - tab->tbase[si]);
    f0 = uniform_i32(tab->first[si]);
    f1 = uniform_i32(tab->first[si + 1]);
    for (int f = t; f < f1 - f0; f += blockDim.x) s_iso[f] = tab->rank[f0 + f].iso;
    __syncthreads();
    return true;
}

// Counting: one work-group per unit; each job of the unit's set gets its
// triangle count in the unit.
template <int kG>
__global__ __launch_bounds__(kG * 8) void k_batch_count(BatchArgs a) {
    __shared__ BatchTile<kG> T;
    __shared__ unsigned long long s_tab[256];
    __shared__ float s_iso[kMaxJobs];     // the set's isos, ascending
    __shared__ uint32_t s_acc[kMaxJobs];  // per rank of the set: triangles in the unit
    __shared__ uint32_t s_w[8];
    __shared__ int s_si;
    const int t = threadIdx.x;
    for (int i = t; i < 256; i += kG * 8) s_tab[i] = kMcTable[i];
    int si, f0, f1;
    int64_t lt;
    if (!batch_unit(a, blockIdx.x, &s_si, s_iso, si, lt, f0, f1)) return;
    const int n_f = f1 - f0;
    if (n_f == 0) return;
    for (int f = t; f < n_f; f += kG * 8) s_acc[f] = 0;
    const BatchSet S = uniform_set(a.sets[si]);
    const Geo g = batch_geo(S);
    const bool ranged = uniform_u32(*S.rng_ok) != 0;
    const int n_c = uniform_i32(batch_candidates<kG>(S, batch_groups(S), lt, a.unit, ranged, s_iso, n_f, T));
    for (int c0 = 0; c0 < n_c; c0 += kG) {
        // the lane's place, opaque to the compiler in every iteration: what
        // derives from it is recomputed instead of held in registers across
        // the loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int gi = tid >> 3, j = tid & 7;
        batch_load_chunk<kG>(S, g, lt, a.unit, c0, n_c, ranged, gi, j, s_iso, n_f, T);
        const int n_p = uniform_i32(batch_pairs<kG>(T, gi, j, s_w));
        const int fa = uniform_i32(T.fa);
        for (int p0 = 0; p0 < n_p; p0 += kPairWin) {
            batch_pair_window<kG>(T, gi, j, p0);
            const int pe = n_p - p0 < kPairWin ? n_p - p0 : kPairWin;
            for (int r0 = 0; r0 < pe; r0 += kG) {
                int tid2 = threadIdx.x;
                asm volatile("" : "+v"(tid2));
                const int gi = tid2 >> 3, j = tid2 & 7;
                const bool on = r0 + gi < pe;
                const uint32_t pr = on ? T.pair[r0 + gi] : 0u;
                const int pgi = (int)(pr & 31), f = fa + (int)(pr >> 5);
                uint32_t items[4];
                int n_dual = 0, n_tri = 0;
                corner_items<false>(j, T.gm[pgi], s_iso[f], T.v[pgi], T.r[pgi], T.l[pgi], s_tab, on, items, n_dual,
                                    n_tri);
                n_tri += __shfl_xor(n_tri, 1, 64);
                n_tri += __shfl_xor(n_tri, 2, 64);
                n_tri += __shfl_xor(n_tri, 4, 64);
                if (on && j == 0 && n_tri) atomicAdd(&s_acc[f], (uint32_t)n_tri);
            }
            __syncthreads();  // T.pair is rewritten by the next window
        }
        __syncthreads();  // the chunk's LDS is reused by the next chunk
    }
    for (int f = t; f < n_f; f += kG * 8) a.tcnt[a.tab->rank[f0 + f].jbase + lt] = s_acc[f];
}

// Scan: one work-group (256) per job over the job's per-unit counts (eight
// consecutive per lane); the job's total into counts (-1: invalid job).
__global__ __launch_bounds__(256) void k_batch_scan(BatchArgs a) {
    __shared__ uint32_t s_w[8];
    const int jb = blockIdx.x, t = threadIdx.x;
    const int64_t base = a.tab->jbase[jb];
    if (base < 0) {
        if (t == 0) a.counts[jb] = -1;
        return;
    }
    const int64_t n = a.tab->jn[jb];
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += 256 * 8) {
        const int64_t i0 = c0 + (int64_t)t * 8;
        uint32_t x[8], sum = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            x[k] = i0 + k < n ? a.tcnt[base + i0 + k] : 0u;
            sum += x[k];
        }
        uint32_t tot;
        uint32_t run = (uint32_t)carry + block_excl_scan(sum, s_w, &tot);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (i0 + k < n) a.tpre[base + i0 + k] = run;
            run += x[k];
        }
        carry += tot;
    }
    if (t == 0) a.counts[jb] = (int64_t)carry;
}

// Writing: one work-group per unit that has output below some job's
// capacity; each job's triangles of the unit go to its output from the
// unit's scanned position on, in the plain path's order.
template <int kG>
__global__ __launch_bounds__(kG * 8) void k_batch_write(BatchArgs a) {
    constexpr int kB = kG * 8;
    __shared__ BatchTile<kG> T;
    __shared__ unsigned long long s_tab[256];
    __shared__ float s_iso[kMaxJobs];     // the set's isos, ascending
    __shared__ uint32_t s_acc[kMaxJobs];  // per rank: the job's next output position (from its out_offset)
    __shared__ uint32_t s_items[kB][4];
    __shared__ uint32_t s_list[kTriList];
    __shared__ uint32_t s_w[8];
    __shared__ int s_si;
    __shared__ uint32_t s_any;
    const int t = threadIdx.x;
    for (int i = t; i < 256; i += kB) s_tab[i] = kMcTable[i];
    int si, f0, f1;
    int64_t lt;
    if (!batch_unit(a, blockIdx.x, &s_si, s_iso, si, lt, f0, f1)) return;
    const int n_f = f1 - f0;
    if (n_f == 0) return;
    if (t == 0) s_any = 0;
    __syncthreads();
    for (int f = t; f < n_f; f += kB) {
        const BatchRank r = a.tab->rank[f0 + f];
        const int64_t e = r.jbase + lt;
        s_acc[f] = a.tpre[e];
        if (a.tcnt[e] && (int64_t)a.tpre[e] < a.jobs[r.job].out_cap) s_any = 1;
    }
    __syncthreads();
    if (uniform_u32(s_any) == 0) return;
    const BatchSet S = uniform_set(a.sets[si]);
    const Geo g = batch_geo(S);
    const bool ranged = uniform_u32(*S.rng_ok) != 0;
    const int n_c = uniform_i32(batch_candidates<kG>(S, batch_groups(S), lt, a.unit, ranged, s_iso, n_f, T));
    for (int c0 = 0; c0 < n_c; c0 += kG) {
        // the lane's place, opaque to the compiler in every iteration: what
        // derives from it is recomputed instead of held in registers across
        // the loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int gi = tid >> 3, j = tid & 7;
        batch_load_chunk<kG>(S, g, lt, a.unit, c0, n_c, ranged, gi, j, s_iso, n_f, T);
        const int n_p = uniform_i32(batch_pairs<kG>(T, gi, j, s_w));
        const int fa = uniform_i32(T.fa);
        for (int p0 = 0; p0 < n_p; p0 += kPairWin) {
            batch_pair_window<kG>(T, gi, j, p0);
            const int pe = n_p - p0 < kPairWin ? n_p - p0 : kPairWin;
            for (int r0 = 0; r0 < pe; r0 += kG) {
                int tid2 = threadIdx.x;
                asm volatile("" : "+v"(tid2));
                const int gi = tid2 >> 3, j = tid2 & 7;
                const bool on = r0 + gi < pe;
                const uint32_t pr = on ? T.pair[r0 + gi] : 0u;
                const int pgi = (int)(pr & 31), f = fa + (int)(pr >> 5);
                const float iso = s_iso[f];
                uint32_t items[4];
                int n_dual = 0, n_tri = 0;
                corner_items<false>(j, T.gm[pgi], iso, T.v[pgi], T.r[pgi], T.l[pgi], s_tab, on, items, n_dual,
                                    n_tri);
                uint32_t tot;
                const uint32_t first = block_excl_scan((uint32_t)n_tri, s_w, &tot);
                int osum = n_tri;
                osum += __shfl_xor(osum, 1, 64);
                osum += __shfl_xor(osum, 2, 64);
                osum += __shfl_xor(osum, 4, 64);
                if (j == 0) {
                    T.pg[gi] = pgi;
                    T.piso[gi] = iso;
                    T.pfirst[gi] = first;
                }
                __syncthreads();
                // an octet's round triangle 0, were it of the octet's job: the
                // job's next position in the unit less the round position of
                // the job's first triangle in the round (the job's pairs are
                // consecutive, from octet k on)
                if (on && j == 0) {
                    const int k = T.pb[f - fa] > p0 + r0 ? T.pb[f - fa] - p0 - r0 : 0;
                    const amr_iso_job& jo = a.jobs[a.tab->rank[f0 + f].job];
                    T.pbase[gi] = jo.out_offset + (int64_t)s_acc[f] - (int64_t)T.pfirst[k];
                    T.pcap[gi] = jo.out_offset + jo.out_cap;
                }
                __syncthreads();
                if (on && j == 0 && osum) atomicAdd(&s_acc[f], (uint32_t)osum);
                if (uniform_u32(tot)) write_pair_triangles<kG>(t, g, items, tot, first, T, a.tris, s_tab, s_items, s_list);
                __syncthreads();  // s_items, s_list and the octet data are reused by the next round
            }
            __syncthreads();  // T.pair is rewritten by the next window
        }
        __syncthreads();  // the chunk's LDS is reused by the next chunk
    }
}

// ---------------------------------------------------------------------------
// Indexed face set: weld the corners of fat triangles by their edge's cell
// pair.  A hash table maps each key to the lowest corner index carrying it;
// a scan over corners numbers those first corners in corner order.
// ---------------------------------------------------------------------------

constexpr int kWeldTile = 4096;  // corners per scan tile (256 threads x 16)

struct WeldWs {
    unsigned long long* key;   // [cap]
    unsigned int* first;       // [cap] lowest corner with this key
    unsigned int* vid;         // [cap] vertex index of the key
    unsigned int* cslot;       // [3 n_tris] slot of each corner
    unsigned long long* s0;    // scan states
    unsigned long long* s1;
    Sched* sched;
    uint32_t cap;
    int shift;
};

__global__ void k_weld_init(WeldWs w, uint32_t n_tiles) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < w.cap; i += gridDim.x * blockDim.x) {
        w.key[i] = kEmpty;
        w.first[i] = 0xFFFFFFFFu;
    }
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n_tiles; i += gridDim.x * blockDim.x) {
        w.s0[i] = 0;
        w.s1[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) w.sched->cticket = 0;
}

__global__ void k_weld_empty(int64_t* n_verts) {
    if (threadIdx.x == 0) *n_verts = 0;
}

__global__ __launch_bounds__(256) void k_weld_insert(const int32_t* __restrict__ cells, int64_t n_corners, WeldWs w) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_corners;
         i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long key = ((unsigned long long)(uint32_t)cells[2 * i] << 32) | (uint32_t)cells[2 * i + 1];
        uint32_t mask = w.cap - 1, h = (uint32_t)((key * kGolden) >> w.shift);
        for (uint32_t step = 0; step <= mask; ++step) {
            unsigned long long k = w.key[h];
            if (k == kEmpty) {
                unsigned long long prev = atomicCAS(&w.key[h], kEmpty, key);
                if (prev == kEmpty) k = key;
                else k = prev;
            }
            if (k == key) {
                atomicMin(&w.first[h], (unsigned int)i);
                w.cslot[i] = h;
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_weld_scan(const float* __restrict__ tris, int64_t n_corners, WeldWs w,
                                                      uint32_t n_tiles, float* __restrict__ verts, int64_t cap_v,
                                                      int64_t* n_verts) {
    __shared__ uint32_t s_rc[16][kBlock / 64];
    __shared__ unsigned long long s_pre;
    __shared__ uint32_t s_tile;
    const int t = threadIdx.x, wave = t >> 6, lane = lane_id();
    if (t == 0) s_tile = (uint32_t)atomicAdd(&w.sched->cticket, 1ull);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * kWeldTile;
    uint32_t bits = 0;
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
        int64_t i = base + r * kBlock + t;
        if (i < n_corners && w.first[w.cslot[i]] == (unsigned int)i) bits |= 1u << r;
    }
    for (int r = 0; r < 16; ++r) {
        unsigned long long b = __ballot((bits >> r) & 1);
        if (lane == 0) s_rc[r][wave] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    uint32_t total = 0;
    for (int r = 0; r < 16; ++r)
        for (int q = 0; q < kBlock / 64; ++q) total += s_rc[r][q];
    if (wave == 0) {
        unsigned long long p0, p1;
        lookback(w.s0, w.s1, tile, 0ull, total, 0ull, p0, p1);
        if (lane == 0) {
            s_pre = p0;
            if (tile == n_tiles - 1) *n_verts = (int64_t)(p0 + total);
        }
    }
    __syncthreads();
    uint64_t pos = s_pre;
    for (int r = 0; r < 16; ++r) {
        unsigned long long b = __ballot((bits >> r) & 1);
        uint32_t before = 0;
        for (int q = 0; q < wave; ++q) before += s_rc[r][q];
        if ((bits >> r) & 1) {
            int64_t i = base + r * kBlock + t;
            uint64_t v = pos + before + (uint64_t)__popcll(b & ((1ull << lane) - 1));
            w.vid[w.cslot[i]] = (unsigned int)v;
            if ((int64_t)v < cap_v) {
                verts[3 * v] = tris[3 * i];
                verts[3 * v + 1] = tris[3 * i + 1];
                verts[3 * v + 2] = tris[3 * i + 2];
            }
        }
        for (int q = 0; q < kBlock / 64; ++q) pos += s_rc[r][q];
    }
}

__global__ __launch_bounds__(256) void k_weld_index(int64_t n_corners, WeldWs w, int32_t* __restrict__ idx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_corners;
         i += (int64_t)gridDim.x * blockDim.x)
        idx[i] = (int32_t)w.vid[w.cslot[i]];
}

// ---------------------------------------------------------------------------
// The paper's cell-location scheme, for comparison with the hash (sec. 3.2):
// the cells sorted by (level, Morton code of their level-l coordinates),
// and a point located by a binary search per level, a hit counting only
// when its level matches.  Built by a least-significant-digit radix sort
// (8-bit digits, stable).  amr_locate answers point queries from either
// index, and amr_snap_count runs the snap queries of every cell (the 27
// points lo + o * 2^l, o in {-1, 0, 1}^3, whose cells are the vertices of
// the cell's 8 corner duals) through either, which is what the two are
// timed on.
// ---------------------------------------------------------------------------

constexpr int kSortPer = 16;                 // keys per thread in the sort passes
constexpr int kSortTile = 256 * kSortPer;    // keys per work-group

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    // bits 0..20 of v to bits 0, 3, 6, ...
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// sort key of the level-l cell with offset coordinates (ux, uy, uz)
__device__ __forceinline__ uint64_t cell_sort_key(int l, int lmin, int bits, uint32_t ux, uint32_t uy, uint32_t uz) {
    return ((uint64_t)(l - lmin) << (3 * bits)) | spread3(ux >> l) | (spread3(uy >> l) << 1) | (spread3(uz >> l) << 2);
}

__global__ __launch_bounds__(256) void k_sort_keys(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                   int64_t n, int32_t ox, int32_t oy, int32_t oz, int lmin, int bits,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int l = lvl[i];
        keys[i] = cell_sort_key(l, lmin, bits, (uint32_t)(xyz[3 * i] - ox), (uint32_t)(xyz[3 * i + 1] - oy),
                                (uint32_t)(xyz[3 * i + 2] - oz));
        vals[i] = (uint32_t)i;
    }
}

// digit histogram of each tile of kSortTile keys, digit-major: hist[d * n_tiles + tile]
__global__ __launch_bounds__(256) void k_sort_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                   uint32_t n_tiles, uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[256];
    const int t = threadIdx.x;
    s_h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortPer; ++r) {
        const int64_t i = base + r * 256 + t;
        if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(size_t)t * n_tiles + blockIdx.x] = s_h[t];
}

// Stable scatter: the keys of a tile in rounds of 256, each key at
// off[digit][tile] + the keys of that digit before it in the tile.  Within
// a wave the lanes holding the same digit are found with 8 ballots (one per
// digit bit).
__global__ __launch_bounds__(256) void k_sort_scatter(const uint64_t* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin, int64_t n, int shift,
                                                      uint32_t n_tiles, const int64_t* __restrict__ off,
                                                      uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
    __shared__ uint32_t s_cnt[4][256];
    __shared__ int64_t s_base[256];
    const int t = threadIdx.x, wave = t >> 6, lane = lane_id();
    s_base[t] = off[(size_t)t * n_tiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortPer; ++r) {
        for (int w = 0; w < 4; ++w) s_cnt[w][t] = 0;
        __syncthreads();
        const int64_t i = base + r * 256 + t;
        const bool live = i < n;
        uint64_t k = 0;
        uint32_t v = 0, d = 0;
        if (live) {
            k = kin[i];
            v = vin[i];
            d = (uint32_t)(k >> shift) & 0xFFu;
        }
        unsigned long long peers = __ballot(live);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long bal = __ballot(live && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (live && rank == 0) s_cnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (live) {
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += s_cnt[w][d];
            const int64_t pos = s_base[d] + before + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        s_base[t] += s_cnt[0][t] + s_cnt[1][t] + s_cnt[2][t] + s_cnt[3][t];
        __syncthreads();
    }
}

// The sorted index as the kernels read it.
struct SortedIndex {
    const uint64_t* keys;    // sorted
    const uint32_t* cells;   // input index of the cell of each key
    int64_t lo[kMaxLevel + 2];  // keys of level l: [lo[l], lo[l + 1])
    int lmin, lmax, bits;
    int32_t ox, oy, oz;
};

__device__ __forceinline__ int64_t sorted_locate(const SortedIndex& si, int64_t ux, int64_t uy, int64_t uz) {
    if (ux < 0 || uy < 0 || uz < 0 || ux >= ((int64_t)1 << si.bits) || uy >= ((int64_t)1 << si.bits) ||
        uz >= ((int64_t)1 << si.bits))
        return -1;
    for (int L = si.lmin; L <= si.lmax; ++L) {
        int64_t a = si.lo[L], b = si.lo[L + 1];
        const int64_t end = b;
        if (a == b) continue;
        const uint64_t key = cell_sort_key(L, si.lmin, si.bits, (uint32_t)ux, (uint32_t)uy, (uint32_t)uz);
        while (a < b) {
            const int64_t c = (a + b) >> 1;
            if (si.keys[c] < key) a = c + 1;
            else b = c;
        }
        if (a < end && si.keys[a] == key) return si.cells[a];
    }
    return -1;
}

// The hash: from the coarsest level down, the record of the block holding
// the position says "a cell" (done), "refined" (finer cells inside: go
// down) or nothing (no cell covers the position).
__device__ __forceinline__ int64_t hash_locate(const Record* __restrict__ rec, const int32_t* __restrict__ ids,
                                               const Geo& g, int64_t ux, int64_t uy, int64_t uz) {
    if (ux < 0 || uy < 0 || uz < 0 || ux >= kSpanLimit || uy >= kSpanLimit || uz >= kSpanLimit) return -1;
    for (int L = g.lmax; L >= 0; --L) {
        const int slot = probe(rec, group_key(L, (uint32_t)ux >> (L + 1), (uint32_t)uy >> (L + 1),
                                              (uint32_t)uz >> (L + 1)),
                               g.shift, g.mask);
        if (slot < 0) return -1;
        const int c = (int)(((ux >> L) & 1) | (((uy >> L) & 1) << 1) | (((uz >> L) & 1) << 2));
        const uint32_t bits = __float_as_uint(rec[slot].val[c]);
        if (bits == kValRefined) continue;
        if (bits == kValEmpty) return -1;
        return ids[(size_t)slot * 8 + c];
    }
    return -1;
}

template <bool kSorted>
__global__ __launch_bounds__(256) void k_locate(const Record* __restrict__ rec, const int32_t* __restrict__ ids,
                                                const Ctrl* ctrl, SortedIndex si, const int32_t* __restrict__ pts,
                                                int64_t n, int32_t* __restrict__ cells) {
    const bool ok = kSorted || ctrl->status == AMR_OK;
    const Geo g = ctrl->geo;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = -1;
        if (ok) {
            if (kSorted)
                c = sorted_locate(si, (int64_t)pts[3 * i] - si.ox, (int64_t)pts[3 * i + 1] - si.oy,
                                  (int64_t)pts[3 * i + 2] - si.oz);
            else
                c = hash_locate(rec, ids, g, (int64_t)pts[3 * i] - g.ox, (int64_t)pts[3 * i + 1] - g.oy,
                                (int64_t)pts[3 * i + 2] - g.oz);
        }
        cells[i] = (int32_t)c;
    }
}

// The snap queries of every cell: the 27 points lo + o * 2^l, o in
// {-1, 0, 1}^3, each located; out[0] += points found, out[1] += the sum of
// (cell index + 1) over them (a checksum both indexes must agree on).
template <bool kSorted>
__global__ __launch_bounds__(256) void k_snap(const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                              int64_t n, const Record* __restrict__ rec,
                                              const int32_t* __restrict__ ids, const Ctrl* ctrl, SortedIndex si,
                                              unsigned long long* out) {
    const bool ok = kSorted || ctrl->status == AMR_OK;
    const Geo g = ctrl->geo;
    const int32_t ox = kSorted ? si.ox : g.ox, oy = kSorted ? si.oy : g.oy, oz = kSorted ? si.oz : g.oz;
    unsigned long long found = 0, sum = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ok && i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int l = lvl[i];
        const int64_t w = (int64_t)1 << l;
        const int64_t x = (int64_t)xyz[3 * i] - ox, y = (int64_t)xyz[3 * i + 1] - oy, z = (int64_t)xyz[3 * i + 2] - oz;
        for (int o = 0; o < 27; ++o) {
            const int64_t qx = x + (o % 3 - 1) * w, qy = y + ((o / 3) % 3 - 1) * w, qz = z + (o / 9 - 1) * w;
            const int64_t c = kSorted ? sorted_locate(si, qx, qy, qz) : hash_locate(rec, ids, g, qx, qy, qz);
            if (c >= 0) {
                ++found;
                sum += (unsigned long long)c + 1ull;
            }
        }
    }
    __shared__ unsigned long long s_f[4], s_s[4];
    auto add = [](unsigned long long p, unsigned long long q) { return p + q; };
    found = wave_reduce(found, add);
    sum = wave_reduce(sum, add);
    if (lane_id() == 0) {
        s_f[threadIdx.x >> 6] = found;
        s_s[threadIdx.x >> 6] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        found = s_f[0] + s_f[1] + s_f[2] + s_f[3];
        sum = s_s[0] + s_s[1] + s_s[2] + s_s[3];
        if (found) {
            atomicAdd(&out[0], found);
            atomicAdd(&out[1], sum);
        }
    }
}

__global__ void k_zero2(unsigned long long* out) {
    if (threadIdx.x < 2) out[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Dual-mesh interpolant.  The paper names the dual mesh as an interpolant
// of the cell values (sec. 5, after Moran et al.) and leaves its use for
// volume rendering to future work (sec. 7); it defines no interpolant.
// Reading taken: a dual is the trilinear hexahedron over the centres of its
// 8 vertex cells (slot s = ex + 2 ey + 4 ez at parameter (ex, ey, ez)) and
// carries the trilinear interpolant of their values; a point takes the
// value of the dual whose map reaches it, and where several do (shared
// faces, and the duals that overlap when their cells span three or more
// levels) the one with the smallest (level, P.z, P.y, P.x) wins.  The map
// sends each corner of the unit cube to its slot's cell centre exactly, so
// a dual reaches the centres of its vertex cells (with that cell's value);
// Newton alone would leave those points to rounding where a degenerate
// dual's map is singular.
// Candidates for a point are the duals that have the point's cell as a
// vertex: a map from every cell to its duals (CSR: offsets per cell, dual
// indices) is built once per dual list.  The inverse map is Newton's method
// from the centre in float64, 40 steps, each clamped to [-1/2, 3/2]; a dual
// reaches the point when every Jacobian on the way was regular
// (|det| > 1e-14), the final residual is below 1e-9 and the parameter lies
// in [-1e-9, 1 + 1e-9] on every axis.
// ---------------------------------------------------------------------------

constexpr int kSmpPer = 16;  // cells per thread in the offset scan (4096 per work-group)
constexpr int kSmpNewton = 40;
constexpr double kSmpEps = 1e-9;
constexpr int kSmpBatch = 8;  // candidate duals whose boxes a query loads at once
constexpr double kSmpDet = 1e-14;

// the dual's distinct vertex cells: slot s counts unless an earlier slot
// holds the same cell (degenerate duals repeat cells); ids outside [0, n)
// are skipped
__device__ __forceinline__ uint32_t smp_distinct(const int32_t (&v)[8], int64_t n) {
    uint32_t keep = 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        bool first = v[s] >= 0 && (int64_t)v[s] < n;
#pragma unroll
        for (int r = 0; r < s; ++r) first = first && v[r] != v[s];
        keep |= (first ? 1u : 0u) << s;
    }
    return keep;
}

__device__ __forceinline__ void smp_load_verts(const int32_t* __restrict__ verts, int64_t d, int32_t (&v)[8]) {
    const int4 a = reinterpret_cast<const int4*>(verts)[2 * d], b = reinterpret_cast<const int4*>(verts)[2 * d + 1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__global__ __launch_bounds__(256) void k_smp_clear(uint32_t* __restrict__ cur, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        cur[i] = 0;
}

// duals per cell, and every dual's bounding box (the box of its vertex
// cells' centres, exact in float32; a dual with a vertex outside [0, n) gets
// an empty box)
__global__ __launch_bounds__(256) void k_smp_count(const int32_t* __restrict__ verts, int64_t m, int64_t n,
                                                   const int32_t* __restrict__ xyz, const int32_t* __restrict__ lvl,
                                                   uint32_t* __restrict__ cur, float4* __restrict__ box) {
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < m; d += (int64_t)gridDim.x * blockDim.x) {
        int32_t v[8];
        smp_load_verts(verts, d, v);
        const uint32_t keep = smp_distinct(v, n);
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        bool good = true;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            if ((keep >> s) & 1) atomicAdd(&cur[v[s]], 1u);
            good = good && v[s] >= 0 && (int64_t)v[s] < n;
            const int64_t c = good ? v[s] : 0;
            const float h = 0.5f * (float)(1 << lvl[c]);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float x = (float)xyz[3 * c + ax] + h;
                lo[ax] = fminf(lo[ax], x);
                hi[ax] = fmaxf(hi[ax], x);
            }
        }
        if (!good) {
            lo[0] = lo[1] = lo[2] = INFINITY;
            hi[0] = hi[1] = hi[2] = -INFINITY;
        }
        box[2 * d] = make_float4(lo[0], lo[1], lo[2], 0.f);
        box[2 * d + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
    }
}

// sum of each work-group's 4096 counts
__global__ __launch_bounds__(256) void k_smp_block_sums(const uint32_t* __restrict__ cur, int64_t n,
                                                        int64_t* __restrict__ bsum) {
    __shared__ unsigned long long s_w[4];
    const int64_t base = (int64_t)blockIdx.x * (256 * kSmpPer);
    unsigned long long x = 0;
    for (int r = 0; r < kSmpPer; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) x += cur[i];
    }
    x = wave_reduce(x, [](unsigned long long p, unsigned long long q) { return p + q; });
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = (int64_t)(s_w[0] + s_w[1] + s_w[2] + s_w[3]);
}

// exclusive scan of the nb work-group sums in place (one work-group);
// bsum[nb] receives the total
__global__ __launch_bounds__(256) void k_smp_scan_sums(int64_t* __restrict__ bsum, int64_t nb) {
    __shared__ unsigned long long s_w[4];
    unsigned long long carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += 256) {
        const int64_t i = c0 + threadIdx.x;
        const unsigned long long x = i < nb ? (unsigned long long)bsum[i] : 0ull;
        const unsigned long long incl = wave_incl_scan(x);
        if (lane_id() == 63) s_w[threadIdx.x >> 6] = incl;
        __syncthreads();
        unsigned long long pre = 0, tot = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < (int)(threadIdx.x >> 6)) pre += s_w[w];
            tot += s_w[w];
        }
        if (i < nb) bsum[i] = (int64_t)(carry + pre + incl - x);
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[nb] = (int64_t)carry;
}

// offsets of every cell's list; the counters restart at zero as fill cursors
__global__ __launch_bounds__(256) void k_smp_offsets(uint32_t* __restrict__ cur, int64_t n,
                                                     const int64_t* __restrict__ bsum, int64_t nb,
                                                     int64_t* __restrict__ off) {
    __shared__ unsigned long long s_w[kSmpPer][4];
    const int t = threadIdx.x, wave = t >> 6, lane = lane_id();
    const int64_t base = (int64_t)blockIdx.x * (256 * kSmpPer);
    unsigned long long v[kSmpPer], incl[kSmpPer];
#pragma unroll
    for (int r = 0; r < kSmpPer; ++r) {
        const int64_t i = base + r * 256 + t;
        v[r] = i < n ? cur[i] : 0u;
        incl[r] = wave_incl_scan(v[r]);
        if (lane == 63) s_w[r][wave] = incl[r];
    }
    __syncthreads();
    unsigned long long carry = (unsigned long long)bsum[blockIdx.x];
    for (int r = 0; r < kSmpPer; ++r) {
        unsigned long long pre = 0, row = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wave) pre += s_w[r][w];
            row += s_w[r][w];
        }
        const int64_t i = base + r * 256 + t;
        if (i < n) {
            off[i] = (int64_t)(carry + pre + incl[r] - v[r]);
            cur[i] = 0;
        }
        carry += row;
    }
    if (blockIdx.x == 0 && t == 0) off[n] = bsum[nb];
}

// every dual into the lists of its distinct vertex cells
__global__ __launch_bounds__(256) void k_smp_fill(const int32_t* __restrict__ verts, int64_t m, int64_t n,
                                                  const int64_t* __restrict__ off, uint32_t* __restrict__ cur,
                                                  uint32_t* __restrict__ ent) {
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < m; d += (int64_t)gridDim.x * blockDim.x) {
        int32_t v[8];
        smp_load_verts(verts, d, v);
        const uint32_t keep = smp_distinct(v, n);
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if ((keep >> s) & 1) ent[off[v[s]] + atomicAdd(&cur[v[s]], 1u)] = (uint32_t)d;
    }
}

struct SampleArgs {
    const Record* rec;
    const int32_t* ids;
    const Ctrl* ctrl;
    const int32_t* xyz;
    const int32_t* lvl;
    const float* val;
    int64_t n;
    const int32_t* corner_level;
    const int32_t* verts;
    const int64_t* off;
    const uint32_t* ent;
    const float4* box;
    const float* pts;
    int64_t n_pts;
    float* out;
    int64_t* dual;
};

// (level, z, y, x) of a dual, compared lexicographically
__device__ __forceinline__ bool smp_key_less(const int4& a, const int4& b) {
    if (a.w != b.w) return a.w < b.w;
    if (a.z != b.z) return a.z < b.z;
    if (a.y != b.y) return a.y < b.y;
    return a.x < b.x;
}

// The cell containing the finest-level position (ix, iy, iz), or -1.
__device__ __forceinline__ int64_t smp_locate(const SampleArgs& a, const Geo& g, int64_t ix, int64_t iy,
                                              int64_t iz) {
    return hash_locate(a.rec, a.ids, g, ix - g.ox, iy - g.oy, iz - g.oz);
}

__device__ __forceinline__ double smp_det3(const double (&J)[3][3]) {
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Does the trilinear map of the hexahedron V reach p?  On success u is the
// parameter of p.
__device__ bool smp_invert(const double (&V)[8][3], const double (&p)[3], double (&u)[3]) {
    u[0] = u[1] = u[2] = 0.5;
    for (int it = 0; it < kSmpNewton; ++it) {
        double x[3] = {0.0, 0.0, 0.0}, J[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const double fx = (s & 1) ? u[0] : 1.0 - u[0], fy = (s & 2) ? u[1] : 1.0 - u[1],
                         fz = (s & 4) ? u[2] : 1.0 - u[2];
            const double dx = (s & 1) ? 1.0 : -1.0, dy = (s & 2) ? 1.0 : -1.0, dz = (s & 4) ? 1.0 : -1.0;
            const double w = fx * fy * fz, d0 = dx * fy * fz, d1 = fx * dy * fz, d2 = fx * fy * dz;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                x[ax] += w * V[s][ax];
                J[ax][0] += d0 * V[s][ax];
                J[ax][1] += d1 * V[s][ax];
                J[ax][2] += d2 * V[s][ax];
            }
        }
        const double det = smp_det3(J);
        if (!(fabs(det) > kSmpDet)) return false;  // a singular step: this dual does not take the point
        const double r[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
        // Cramer's rule: step_b = det(J with column b replaced by r) / det
        double st[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double M[3][3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
#pragma unroll
                for (int c = 0; c < 3; ++c) M[ax][c] = c == b ? r[ax] : J[ax][c];
            st[b] = smp_det3(M) / det;
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) u[b] = fmin(fmax(u[b] + st[b], -0.5), 1.5);
        // converged: the remaining steps would only move u by rounding
        if (fmax(fabs(st[0]), fmax(fabs(st[1]), fabs(st[2]))) < 1e-15) break;
    }
    double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const double w = ((s & 1) ? u[0] : 1.0 - u[0]) * ((s & 2) ? u[1] : 1.0 - u[1]) * ((s & 4) ? u[2] : 1.0 - u[2]);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) x[ax] += w * V[s][ax];
    }
    double res = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) res = fmax(res, fabs(x[ax] - p[ax]));
    if (!(res < kSmpEps)) return false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
        if (!(u[ax] >= -kSmpEps && u[ax] <= 1.0 + kSmpEps)) return false;
    return true;
}

// One thread per point.
__global__ __launch_bounds__(256) void k_smp_query(SampleArgs a) {
    const bool ok = a.ctrl->status == AMR_OK;
    const Geo g = a.ctrl->geo;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.n_pts;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double p[3] = {(double)a.pts[3 * q], (double)a.pts[3 * q + 1], (double)a.pts[3 * q + 2]};
        float value = __uint_as_float(0x7fc00000u);
        int64_t best = -1;
        int64_t c = -1;
        // finest-level position of the point (floor), inside the coordinate limits
        if (ok && fabs(p[0]) < (double)kCoordLimit && fabs(p[1]) < (double)kCoordLimit &&
            fabs(p[2]) < (double)kCoordLimit)
            c = smp_locate(a, g, (int64_t)floor(p[0]), (int64_t)floor(p[1]), (int64_t)floor(p[2]));
        if (c >= 0) {
            int4 bkey = make_int4(0, 0, 0, 0x7fffffff);
            const int64_t e1 = a.off[c + 1];
            // candidates kSmpBatch at a time: their indices, then their boxes,
            // each batch's loads in flight together (cells beside much finer
            // ones have thousands of candidates, and one candidate at a time
            // paid two dependent loads for each); then the few whose box
            // holds the point, in list order
            for (int64_t e0 = a.off[c]; e0 < e1; e0 += kSmpBatch) {
                int64_t dd[kSmpBatch];
#pragma unroll
                for (int u = 0; u < kSmpBatch; ++u) dd[u] = e0 + u < e1 ? (int64_t)a.ent[e0 + u] : -1;
                uint32_t hits = 0;
#pragma unroll
                for (int u = 0; u < kSmpBatch; ++u) {
                    if (dd[u] < 0) continue;
                    const float4 b0 = a.box[2 * dd[u]], b1 = a.box[2 * dd[u] + 1];
                    if (p[0] >= (double)b0.x - kSmpEps && p[0] <= (double)b1.x + kSmpEps &&
                        p[1] >= (double)b0.y - kSmpEps && p[1] <= (double)b1.y + kSmpEps &&
                        p[2] >= (double)b0.z - kSmpEps && p[2] <= (double)b1.z + kSmpEps)
                        hits |= 1u << u;
                }
                for (; hits; hits &= hits - 1) {
                    const int hu = __ffs(hits) - 1;
                    int64_t d = dd[0];
    #pragma unroll
                    for (int u = 1; u < kSmpBatch; ++u)
                        if (hu == u) d = dd[u];
                    const int4 key = reinterpret_cast<const int4*>(a.corner_level)[d];
                    if (best >= 0 && !smp_key_less(key, bkey)) continue;
                    // the dual's cells
                    int32_t v[8];
                    smp_load_verts(a.verts, d, v);
                    double V[8][3];
                    bool good = true;
    #pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const int64_t id = v[s];
                        good = good && id >= 0 && id < a.n;
                        const int64_t ci = good ? id : 0;
                        const double h = 0.5 * (double)(1 << a.lvl[ci]);
    #pragma unroll
                        for (int ax = 0; ax < 3; ++ax) V[s][ax] = (double)a.xyz[3 * ci + ax] + h;
                    }
                    if (!good) continue;
                    // the map sends each cube corner to its slot's cell centre
                    // exactly: a vertex cell centred at p settles it (first slot)
                    int at = -1;
    #pragma unroll
                    for (int s = 7; s >= 0; --s)
                        if (V[s][0] == p[0] && V[s][1] == p[1] && V[s][2] == p[2]) at = s;
                    if (at >= 0) {
                        best = d;
                        bkey = key;
                        value = a.val[v[at]];
                        continue;
                    }
                    double u[3];
                    if (!smp_invert(V, p, u)) continue;
                    double f = 0.0;
    #pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const double ux = fmin(fmax(u[0], 0.0), 1.0), uy = fmin(fmax(u[1], 0.0), 1.0),
                                     uz = fmin(fmax(u[2], 0.0), 1.0);
                        const double w = ((s & 1) ? ux : 1.0 - ux) * ((s & 2) ? uy : 1.0 - uy) * ((s & 4) ? uz : 1.0 - uz);
                        f += w * (double)a.val[v[s]];
                    }
                    best = d;
                    bkey = key;
                    value = (float)f;
                }
            }
        }
        a.out[q] = value;
        if (a.dual) a.dual[q] = best;
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
    Ctrl* ctrl = nullptr;  // device
    Ctrl* host_ctrl = nullptr;
    // upload
    const int32_t* xyz = nullptr;
    const int32_t* lvl = nullptr;
    const float* val = nullptr;
    int64_t n = 0;
    bool uploaded = false;
    int lmin = 0, lmax = 0;
    int32_t origin[3] = {0, 0, 0};
    uint64_t level_count[kMaxLevel + 1] = {};
    uint64_t record_hint = 0;
    bool up_pending = false;       // upload verdict not read on the host yet
    bool up_captured = false;      // ... and not on its way either (enqueued inside a graph capture)
    int up_status = AMR_OK;
    hipEvent_t up_event = nullptr;  // recorded after the verdict's copy
    uint32_t last_cap = 0;          // table size of the last build, and its n
    int64_t last_n = -1;
    // index
    bool built = false;             // a build is enqueued (its verdict may still be on the device)
    bool build_tried = false;       // a build was enqueued since the last upload
    bool build_pending = false;     // its verdict has not been read by amr_build_status
    bool build_captured = false;    // it was enqueued inside a graph capture (no event to wait for)
    int build_status = AMR_OK;      // the verdict, once read
    hipEvent_t build_event = nullptr;
    uint32_t cap = 0;
    uint32_t grid_groups = 0;       // groups the extraction grids cover (a bound the build enforces)
    Record* rec = nullptr;
    int32_t* ids = nullptr;
    bool ids_ready = false;  // input indices filled in (on first use)
    int extractions = 0;     // extraction calls since the build (saturates at 2)
    uint64_t build_gen = 0;  // builds so far
    uint64_t upload_gen = 0;  // uploads so far
    // the sorted-cells index (amr_build_sorted_index), valid for upload srt_gen
    uint64_t srt_gen = ~0ull;
    const uint64_t* srt_keys = nullptr;
    const uint32_t* srt_cells = nullptr;
    int srt_bits = 0;
    int64_t srt_lo[kMaxLevel + 2] = {};
    uint64_t smp_gen = ~0ull;  // the build a dual-mesh sampler was made for
    float2* rng = nullptr;
    unsigned long long* dual_total = nullptr;
    uint32_t* clist = nullptr;              // group list of a list pass, its length,
    uint32_t* lcnt = nullptr;               // its triangle counts (lists from a count pass)
    unsigned long long* n_list = nullptr;   // and the dual count summed on the way
    unsigned long long* list_duals = nullptr;
    unsigned long long* ls0 = nullptr;      // candidate list: look-back states
    unsigned long long* ls1 = nullptr;
    int32_t* glist = nullptr;
    unsigned long long* gkey = nullptr;
    unsigned long long* tot = nullptr;   // extraction: per-tile totals
    unsigned long long* gcnt = nullptr;  // extraction: per-group totals
    unsigned long long* st_t = nullptr;  // extraction: per-tile prefixes
    unsigned long long* st_d = nullptr;
    unsigned long long* xs0 = nullptr;   // extraction scan: look-back states
    unsigned long long* xs1 = nullptr;
    unsigned long long* fs0 = nullptr;   // fused extraction: look-back states
    unsigned long long* fs1 = nullptr;
    unsigned long long* ct0 = nullptr;
    unsigned long long* ct1 = nullptr;
    Sched* sched = nullptr;
    // amr_time_kernel: the next launch of this kernel records these events
    int time_kernel = 0;
    hipEvent_t time_start = nullptr, time_stop = nullptr;
    const char* timed_name = "";  // the kernel the last armed timing went to
};

namespace {

// A launch that records the set's timing events around the kernel itself
// when amr_time_kernel armed them for `which` (once), else a plain launch.
template <typename... KArgs, typename... Args>
void launch(amr_set* s, int which, const char* name, void (*kernel)(KArgs...), dim3 grid, dim3 block,
            hipStream_t stream, Args... args) {
    if (s->time_kernel == which) {
        s->time_kernel = 0;
        s->timed_name = name;
        hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, s->time_start, s->time_stop, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, stream, args...);
    }
}

uint32_t table_cap(const amr_set* s) {
    uint64_t want = s->record_hint * 2;
    if (want < kRegion) want = kRegion;  // slot_of needs at least one whole region
    uint64_t cap = 1;
    while (cap < want) cap <<= 1;
    return cap > kMaxCap ? 0 : (uint32_t)cap;
}

struct Layout {
    size_t rec, ids, glist, gkey, gcnt, rng, clist, lcnt, tot, st_t, st_d, xs0, xs1, fs0, fs1, ct0, ct1, ls0, ls1,
        sched, dual_total, n_list, list_duals, total;
    uint32_t max_tiles, max_scan_tiles, compact_tiles, max_list_wgs;
    int compact_per;
};

Layout layout_for(uint32_t cap) {
    Layout L{};
    uint32_t max_groups = cap;  // at most one group per slot
    L.max_tiles = (max_groups + kGroupsPerTile - 1) / kGroupsPerTile + 1;
    // small tables: more, smaller compaction tiles (latency); large: fewer
    // tickets (measured with 256 threads per work-group: 2^16 slots 18 us
    // with 256 tiles against 28 us with 64; 2^20 slots 65 us with 1024 tiles
    // against 93 with 4096 and 77 with 512)
    L.compact_per = cap <= (1u << 17) ? 1 : cap <= (1u << 20) ? 4 : kCompactMaxPerThread;
    uint32_t ctile = (uint32_t)(kCompactBlock * L.compact_per);
    L.compact_tiles = (cap + ctile - 1) / ctile;
    size_t off = 0;
    L.rec = off;
    off = align256(off + (size_t)cap * sizeof(Record));
    L.ids = off;
    off = align256(off + (size_t)cap * 8 * sizeof(int32_t));
    L.glist = off;
    off = align256(off + (size_t)max_groups * sizeof(int32_t));
    L.gkey = off;
    off = align256(off + (size_t)max_groups * sizeof(unsigned long long));
    L.gcnt = off;
    off = align256(off + (size_t)max_groups * sizeof(unsigned long long));
    L.rng = off;
    off = align256(off + (size_t)max_groups * sizeof(float2));
    L.clist = off;
    off = align256(off + (size_t)max_groups * sizeof(uint32_t));
    L.lcnt = off;
    off = align256(off + ((size_t)max_groups + kGroupsPerTile) * sizeof(uint32_t));
    L.max_scan_tiles = (L.max_tiles + kBlock * kScanPer - 1) / (kBlock * kScanPer);
    L.tot = off;
    off = align256(off + (size_t)L.max_tiles * 8);
    L.st_t = off;
    off = align256(off + (size_t)L.max_tiles * 8);
    L.st_d = off;
    off = align256(off + (size_t)L.max_tiles * 8);
    L.xs0 = off;
    off = align256(off + (size_t)L.max_scan_tiles * 8);
    L.xs1 = off;
    off = align256(off + (size_t)L.max_scan_tiles * 8);
    L.fs0 = off;
    off = align256(off + (size_t)kFusedMaxTiles * 8);
    L.fs1 = off;
    off = align256(off + (size_t)kFusedMaxTiles * 8);
    L.ct0 = off;
    off = align256(off + (size_t)L.compact_tiles * 8);
    L.ct1 = off;
    off = align256(off + (size_t)L.compact_tiles * 8);
    L.sched = off;
    off = align256(off + sizeof(Sched));
    L.dual_total = off;
    off = align256(off + sizeof(unsigned long long));
    L.n_list = off;
    off = align256(off + sizeof(unsigned long long));
    L.list_duals = off;
    off = align256(off + sizeof(unsigned long long));
    L.max_list_wgs = (max_groups + kBlock * kListPer - 1) / (kBlock * kListPer);
    L.ls0 = off;
    off = align256(off + (size_t)L.max_list_wgs * 8);
    L.ls1 = off;
    off = align256(off + (size_t)L.max_list_wgs * 8);
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

// Most groups a good build can hold: the build fails when more than 3/4 of
// the slots are in use.
uint32_t max_groups_of(uint32_t cap) { return cap - cap / 4; }

// The input index of every cell beside its value in the table, filled in
// once per build, when a call first needs it.
int ensure_ids(amr_set* s, hipStream_t stream) {
    if (s->ids_ready || s->n == 0) return AMR_OK;
    hipLaunchKernelGGL(k_index_ids, dim3(grid_for(s->n, 256)), dim3(256), 0, stream, s->xyz, s->lvl, s->n, s->ctrl,
                       s->rec, s->ids);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "cell index map");
    s->ids_ready = true;
    return AMR_OK;
}

int launch_extract(amr_set* s, bool duals, float iso, float* tris, int32_t* tri_cells, int64_t* tri_dual,
                   int32_t* corner_level, int32_t* verts, float* dvals, int64_t cap, int64_t* counts,
                   hipStream_t stream) {
    if ((duals ? verts != nullptr : tri_cells != nullptr) && cap > 0) {
        // outputs name input indices
        const int st = ensure_ids(s, stream);
        if (st != AMR_OK) return st;
    }
    // The group count lives on the device; the grids cover the bound the
    // build enforced, and work-groups past the last tile leave at once.
    const uint32_t max_groups = s->grid_groups;
    uint32_t max_tiles = (max_groups + kGroupsPerTile - 1) / kGroupsPerTile;
    if (max_tiles == 0) max_tiles = 1;
    ExtractArgs a;
    a.rec = s->rec;
    a.ids = s->ids;
    a.glist = s->glist;
    a.gkey = s->gkey;
    a.ctrl = s->ctrl;
    a.iso = iso;
    a.tris = tris;
    a.tri_cells = tri_cells;
    a.tri_dual = tri_dual;
    a.corner_level = corner_level;
    a.verts = verts;
    a.dvals = dvals;
    a.cap = cap;
    a.counts = counts;
    a.tot = s->tot;
    a.gcnt = s->gcnt;
    a.pre_t = s->st_t;
    a.pre_d = s->st_d;
    a.sc0 = s->xs0;
    a.sc1 = s->xs1;
    a.sched = s->sched;
    a.n_scan_tiles = (max_tiles + kBlock * kScanPer - 1) / (kBlock * kScanPer);
    if (a.n_scan_tiles == 0) a.n_scan_tiles = 1;
    // The second extraction after a build records the group value ranges
    // (a set extracted once never pays for them); from the third on,
    // iso-surfaces use them unless triangles name their duals (whose
    // numbering needs every group's dual count).  The kernels cull only when
    // the device says the ranges of this build are there (a recording call
    // captured in a graph and never replayed leaves none).
    a.rng = s->rng;
    a.dual_total = s->dual_total;
    a.rng_mode = s->extractions == 0   ? kRngNone
                 : s->extractions == 1 ? kRngRecord
                 : (!duals && tri_dual == nullptr ? kRngCull : kRngNone);
    a.list_from_cull = 0;
    a.clist = nullptr;
    a.n_list = nullptr;
    a.lcnt = nullptr;
    a.list_duals = nullptr;
    const uint32_t n_wgs = (max_groups + kBlock * kListPer - 1) / (kBlock * kListPer);
    const uint32_t grid = ((max_tiles + kXcds - 1) / kXcds) * kXcds;
    // full count passes over large sets: one lane per group (k_count), 256
    // groups per work-group
    const bool lane_count = max_groups >= kLaneCountMinGroups;
    const uint32_t count_units = (max_groups + 255) / 256;
    const uint32_t count_grid = (count_units > 0 ? ((count_units + kXcds - 1) / kXcds) : 1) * kXcds;
    if (max_tiles <= kFusedMaxTiles) {
        // one fused pass (look-back states alternate parity between calls)
        a.sc0 = s->fs0;
        a.sc1 = s->fs1;
        if (duals)
            launch(s, AMR_KERNEL_EXTRACT, "k_extract<true, 2>", k_extract<true, kPassFused>, dim3(max_tiles), dim3(kBlock), stream, a);
        else
            launch(s, AMR_KERNEL_EXTRACT, "k_extract<false, 2>", k_extract<false, kPassFused>, dim3(max_tiles), dim3(kBlock), stream, a);
    } else if (a.rng_mode == kRngCull) {
        // list the candidate groups, then count, scan and write over the list
        const bool write = cap > 0 && (tris || tri_cells);
        hipLaunchKernelGGL(k_group_list, dim3(n_wgs), dim3(kBlock), 0, stream, s->rng, nullptr, s->ctrl, iso, n_wgs,
                           s->clist, nullptr, s->n_list, nullptr, s->ls0, s->ls1, s->sched);
        a.clist = s->clist;
        a.n_list = s->n_list;
        a.list_duals = s->dual_total;
        a.list_from_cull = 1;
        launch(s, AMR_KERNEL_EXTRACT, "k_extract_list<0>", k_extract_list<kPassCount>, dim3(grid), dim3(kBlock), stream, a);
        hipLaunchKernelGGL(k_tile_scan, dim3(a.n_scan_tiles), dim3(kBlock), 0, stream, a, 0);
        if (write) launch(s, AMR_KERNEL_WRITE, "k_extract_list<1>", k_extract_list<kPassWrite>, dim3(grid), dim3(kBlock), stream, a);
    } else if (!duals && tri_dual == nullptr && cap > 0 && (tris || tri_cells)) {
        // count pass over all groups, then list the groups with triangles (in
        // group order, with their counts) and scan and write over that list
        // only: most groups have none, and the write pass would otherwise
        // redo their neighbourhoods beside the few that have some
        if (lane_count)
            launch(s, AMR_KERNEL_EXTRACT, "k_count<false>", k_count<false>, dim3(count_grid), dim3(256), stream, a);
        else
            launch(s, AMR_KERNEL_EXTRACT, "k_extract<false, 0>", k_extract<false, kPassCount>, dim3(grid), dim3(kBlock), stream, a);
        hipLaunchKernelGGL(k_group_list, dim3(n_wgs), dim3(kBlock), 0, stream, nullptr, s->gcnt, s->ctrl, iso,
                           n_wgs, s->clist, s->lcnt, s->n_list, s->list_duals, s->ls0, s->ls1, s->sched);
        a.clist = s->clist;
        a.n_list = s->n_list;
        a.lcnt = s->lcnt;
        a.list_duals = s->list_duals;
        hipLaunchKernelGGL(k_tile_scan, dim3(a.n_scan_tiles), dim3(kBlock), 0, stream, a, 0);
        launch(s, AMR_KERNEL_WRITE, "k_extract_list<1>", k_extract_list<kPassWrite>, dim3(grid), dim3(kBlock), stream, a);
    } else {
        // count pass, scan, then the write pass only when something is written;
        // the grid is a multiple of the XCD count (see the tile mapping)
        const bool write = cap > 0 && (duals ? (corner_level || verts || dvals) : (tris || tri_cells || tri_dual));
        if (lane_count) {
            if (duals)
                launch(s, AMR_KERNEL_EXTRACT, "k_count<true>", k_count<true>, dim3(count_grid), dim3(256), stream, a);
            else
                launch(s, AMR_KERNEL_EXTRACT, "k_count<false>", k_count<false>, dim3(count_grid), dim3(256), stream, a);
        } else if (duals) {
            launch(s, AMR_KERNEL_EXTRACT, "k_extract<true, 0>", k_extract<true, kPassCount>, dim3(grid), dim3(kBlock), stream, a);
        } else {
            launch(s, AMR_KERNEL_EXTRACT, "k_extract<false, 0>", k_extract<false, kPassCount>, dim3(grid), dim3(kBlock), stream, a);
        }
        hipLaunchKernelGGL(k_tile_scan, dim3(a.n_scan_tiles), dim3(kBlock), 0, stream, a, duals ? 1 : 0);
        if (write) {
            if (duals)
                launch(s, AMR_KERNEL_WRITE, "k_extract<true, 1>", k_extract<true, kPassWrite>, dim3(grid), dim3(kBlock), stream, a);
            else
                launch(s, AMR_KERNEL_WRITE, "k_extract<false, 1>", k_extract<false, kPassWrite>, dim3(grid), dim3(kBlock), stream, a);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "extract launch");
    if (s->extractions < 2) ++s->extractions;
    return AMR_OK;
}

}  // namespace

struct amr_batch {
    int device = 0;
    int n_sets = 0;
    BatchSet* d_sets = nullptr;  // device table
    uint32_t max_groups = 0;     // the largest group bound of the sets (their extraction grids)
    uint32_t bound[kMaxSets] = {};  // each set's group bound
};

namespace {

int batch_check_shape(int block, int unit) {
    if (block != 128 && block != 256) return fail(AMR_EINVAL, "batched launch: block must be 128 or 256");
    if (unit < 64 || unit > kMaxUnit || (unit & (unit - 1)))
        return fail(AMR_EINVAL, "batched launch: unit must be a power of two in 64..%d groups", kMaxUnit);
    return AMR_OK;
}

int log2_of(int unit) {
    int k = 0;
    while ((1 << k) < unit) ++k;
    return k;
}

// units of the largest set (the per-job counts are kept per unit of the job's set)
int64_t batch_max_units(const amr_batch* b, int unit) {
    const int64_t t = ((int64_t)b->max_groups + unit - 1) / unit;
    return t > 0 ? t : 1;
}

// units of all sets together, at their bounds: the counting and writing grids
int64_t batch_all_units(const amr_batch* b, int unit) {
    int64_t n = 0;
    for (int i = 0; i < b->n_sets; ++i) n += ((int64_t)b->bound[i] + unit - 1) / unit;
    return n > 0 ? n : 1;
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
    // pinned, so that the read-backs of the verdicts are plain DMA
    hipError_t e = hipHostMalloc((void**)&s->host_ctrl, sizeof(Ctrl), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete s;
        return hipfail(e, "amr_create: host control block");
    }
    memset(s->host_ctrl, 0, sizeof(Ctrl));
    e = hipMalloc((void**)&s->ctrl, sizeof(Ctrl));
    if (e == hipSuccess) {
        // clean replicas for the first upload
        hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, 0, s->ctrl);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->up_event, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->build_event, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (s->ctrl) (void)hipFree(s->ctrl);
        if (s->up_event) (void)hipEventDestroy(s->up_event);
        (void)hipHostFree(s->host_ctrl);
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
        if (s->up_event) (void)hipEventDestroy(s->up_event);
        if (s->build_event) (void)hipEventDestroy(s->build_event);
    }
    (void)hipHostFree(s->host_ctrl);
    delete s;
}

namespace {

// True while `stream` records a graph: then nothing may wait on the host,
// and events and copies to the host are left out.
bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

}  // namespace

int amr_upload(amr_set* s, const int32_t* xyz, const int32_t* level, const float* value, int64_t n,
               hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_upload: set is NULL");
    if (n < 0) return fail(AMR_EINVAL, "amr_upload: negative n");
    if (n > 0 && (!xyz || !level || !value)) return fail(AMR_EINVAL, "amr_upload: NULL array");
    if (n >= (int64_t)1 << 31) return fail(AMR_ERANGE, "amr_upload: more than 2^31-1 cells");
    DeviceGuard dg(s->device);
    s->uploaded = false;
    s->built = false;
    s->build_tried = false;
    s->build_pending = false;
    s->xyz = xyz;
    s->lvl = level;
    s->val = value;
    s->n = n;
    ++s->upload_gen;
    for (int l = 0; l <= kMaxLevel; ++l) s->level_count[l] = 0;
    s->lmin = s->lmax = 0;
    s->origin[0] = s->origin[1] = s->origin[2] = 0;
    s->record_hint = 0;
    s->up_pending = false;
    s->up_captured = false;
    s->up_status = AMR_OK;
    // the replicas are clean: amr_create and every k_upload_finish leave them so
    if (n > 0) {
        launch(s, AMR_KERNEL_UPLOAD, "k_upload", k_upload, dim3(grid_for(n, 256)), dim3(256), stream, xyz, level, value, n,
               s->ctrl);
        hipLaunchKernelGGL(k_upload_finish, dim3(1), dim3(kReplicas), 0, stream, s->ctrl);
    } else {
        // an empty set: a clean verdict for the build's kernels
        hipLaunchKernelGGL(k_upload_finish, dim3(1), dim3(kReplicas), 0, stream, s->ctrl);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_upload: launch");
    if (capturing(stream)) {
        // inside a graph: the verdict stays on the device (the build reads it
        // there; amr_index_bytes fetches it once the graph has run)
        s->up_captured = true;
    } else {
        // the verdict travels to the host behind the kernels; whoever needs it
        // first (amr_index_bytes, amr_build_index, amr_build_status) waits for this event
        e = hipMemcpyAsync(&s->host_ctrl->res, &s->ctrl->res, sizeof(UpRes), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipEventRecord(s->up_event, stream);
        if (e != hipSuccess) return hipfail(e, "amr_upload: readback");
    }
    s->up_pending = true;
    s->uploaded = true;
    g_err[0] = 0;
    return AMR_OK;
}

namespace {

// Take over an upload verdict that has reached host_ctrl->res.
int apply_upload(amr_set* s) {
    const UpRes& u = s->host_ctrl->res;
    s->up_pending = false;
    s->up_captured = false;
    s->up_status = u.status;
    if (u.status != AMR_OK) {
        if (u.err >= 16)
            return fail(AMR_ERANGE, "amr_upload: extent %lld on axis %d too large for level %d (limit 2^20)",
                        (long long)u.hi[u.err - 16] - u.lo[u.err - 16], (int)(u.err - 16), u.lmax);
        const char* why = (u.err & kErrLevel)   ? "level outside [0, 20]"
                          : (u.err & kErrAlign) ? "lower corner not a multiple of 2^level"
                          : (u.err & kErrValue) ? "non-finite value"
                                                : "coordinate outside [-2^23, 2^23]";
        return fail(u.status, "amr_upload: cell %llu: %s", (unsigned long long)u.bad, why);
    }
    s->lmin = u.lmin;
    s->lmax = u.lmax;
    for (int a = 0; a < 3; ++a) s->origin[a] = u.origin[a];
    for (int l = 0; l <= kMaxLevel; ++l) s->level_count[l] = u.level_count[l];
    s->record_hint = u.record_hint;
    return AMR_OK;
}

// Wait for the upload verdict if it is still on its way (or, for an upload
// enqueued inside a graph capture, fetch it from the device).
int upload_verdict(amr_set* s) {
    if (s->up_pending) {
        hipError_t e;
        if (s->up_captured) {
            e = hipDeviceSynchronize();
            if (e == hipSuccess) e = hipMemcpy(&s->host_ctrl->res, &s->ctrl->res, sizeof(UpRes), hipMemcpyDeviceToHost);
        } else {
            e = hipEventSynchronize(s->up_event);
        }
        if (e != hipSuccess) return hipfail(e, "amr_upload: waiting for the verdict");
        return apply_upload(s);
    }
    if (s->up_status != AMR_OK) return apply_upload(s);  // the same error again
    return AMR_OK;
}

// Read the verdict of the last build (and of the upload before it) from the
// device, waiting for the build first; sets s->build_status and returns it.
int read_build_verdict(amr_set* s) {
    if (!s->build_pending) return s->build_status;
    DeviceGuard dg(s->device);
    hipError_t e = s->build_captured ? hipDeviceSynchronize() : hipEventSynchronize(s->build_event);
    const size_t tail = offsetof(Ctrl, overflow);
    if (e == hipSuccess)
        e = hipMemcpy((char*)s->host_ctrl + tail, (char*)s->ctrl + tail, sizeof(Ctrl) - tail, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hipfail(e, "amr_build_status: reading the verdict");
    s->build_pending = false;
    s->build_captured = false;
    const Ctrl& c = *s->host_ctrl;
    int st = c.status;
    if (s->up_pending) {
        // the copy above carried the upload verdict too
        int su = apply_upload(s);
        if (su != AMR_OK) {
            s->build_status = su;
            s->built = false;
            return su;
        }
    } else if (s->up_status != AMR_OK) {
        st = s->up_status;
    }
    if (st == AMR_OK) {
        s->build_status = AMR_OK;
        g_err[0] = 0;
        return AMR_OK;
    }
    s->built = false;
    s->build_status = st;
    if (st == AMR_ENOSPACE) {
        unsigned long long n_records = c.n_records;  // records at compaction time: the groups
        for (int r = 0; r < kReplicas; ++r) n_records += c.made[r * 16];
        uint64_t seen = n_records;
        s->record_hint = seen * 2 > s->record_hint * 4 ? seen * 2 : s->record_hint * 4;
        s->last_cap = 0;  // the next build sizes a new table and bound
        return fail(AMR_ENOSPACE, "amr_build_index: hash table too small (%u slots, %llu groups against a bound of %u); "
                    "query amr_index_bytes again", s->cap, (unsigned long long)c.n_groups, s->grid_groups);
    }
    if (st == AMR_EOVERLAP && c.overlap) {
        // bad_build holds slot * 8 + child of the coarse cell: name its input index
        const unsigned long long ref = c.bad_build;
        int32_t id = -1;
        hipLaunchKernelGGL(k_index_ids, dim3(grid_for(s->n, 256)), dim3(256), 0, 0, s->xyz, s->lvl, s->n, s->ctrl,
                           s->rec, s->ids);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpy(&id, s->ids + ref, sizeof(id), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hipfail(e, "amr_build_index: overlap report");
        return fail(AMR_EOVERLAP, "amr_build_index: cell %d contains finer cells", (int)id);
    }
    if (st == AMR_EOVERLAP) {
        // some cell was stored twice: find the lowest overwritten index
        hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, 0, s->ctrl);
        hipLaunchKernelGGL(k_index_ids, dim3(grid_for(s->n, 256)), dim3(256), 0, 0, s->xyz, s->lvl, s->n, s->ctrl,
                           s->rec, s->ids);
        hipLaunchKernelGGL(k_index_find_dup, dim3(grid_for(s->n, 256)), dim3(256), 0, 0, s->xyz, s->lvl, s->n, s->rec,
                           s->ids, s->ctrl);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpy((char*)s->host_ctrl + tail, (char*)s->ctrl + tail, sizeof(Ctrl) - tail,
                          hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hipfail(e, "amr_build_index: duplicate search");
        return fail(AMR_EOVERLAP, "amr_build_index: duplicate cell (index %llu)", s->host_ctrl->bad_build);
    }
    return fail(st, "amr_build_index: the build failed (status %d)", st);
}

}  // namespace

int amr_index_bytes(const amr_set* cs, size_t* bytes) {
    if (!cs || !bytes) return fail(AMR_EINVAL, "amr_index_bytes: NULL argument");
    amr_set* s = const_cast<amr_set*>(cs);  // reading a verdict updates the handle
    if (!s->uploaded) return fail(AMR_ESTATE, "amr_index_bytes: call amr_upload first");
    if (s->build_pending) (void)read_build_verdict(s);  // an AMR_ENOSPACE verdict grows the answer
    int st = upload_verdict(s);
    if (st != AMR_OK) return st;
    uint32_t cap = table_cap(s);
    if (!cap) return fail(AMR_ERANGE, "amr_index_bytes: more groups than the index supports");
    *bytes = layout_for(cap).total;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_build_index(amr_set* s, void* ws, size_t bytes, hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_build_index: set is NULL");
    if (!s->uploaded) return fail(AMR_ESTATE, "amr_build_index: call amr_upload first");
    s->built = false;
    s->build_pending = false;
    if (!ws || ((uintptr_t)ws & 255)) return fail(AMR_EINVAL, "amr_build_index: workspace NULL or not 256-B aligned");
    const bool cap_known = s->n == s->last_n && s->last_cap && bytes >= layout_for(s->last_cap).total;
    const bool in_graph = capturing(stream);
    uint32_t cap;
    if (s->up_pending && cap_known) {
        // a set of the same size as last time: build at once with the same
        // table; the kernels take the geometry from the upload verdict on the
        // device, and a table that turns out too small fails the build
        cap = s->last_cap;
    } else if (s->up_pending && in_graph) {
        return fail(AMR_ESTATE, "amr_build_index: the table size is unknown inside a graph capture (size it with "
                                "amr_index_bytes or an earlier build of as many cells first)");
    } else {
        int st = upload_verdict(s);
        if (st != AMR_OK) return st;
        cap = table_cap(s);
        if (!cap) return fail(AMR_ERANGE, "amr_build_index: more groups than the index supports");
    }
    Layout L = layout_for(cap);
    if (bytes < L.total)
        return fail(AMR_ENOSPACE, "amr_build_index: workspace of %zu bytes, need %zu", bytes, L.total);
    // The extraction grids cover this many groups; the build fails with
    // AMR_ENOSPACE if there are more.  A new table takes the upload's record
    // estimate with a quarter of headroom (about one record per group for
    // octrees and bricks); a rebuild of as many cells keeps the last bound.
    if (!(s->up_pending && cap_known)) {
        const uint64_t want = s->record_hint + s->record_hint / 4 + 256;
        s->grid_groups = (uint32_t)(want < (uint64_t)max_groups_of(cap) ? want : max_groups_of(cap));
    }
    if (s->grid_groups > max_groups_of(cap) || s->grid_groups == 0) s->grid_groups = max_groups_of(cap);
    DeviceGuard dg(s->device);
    char* base = (char*)ws;
    s->cap = cap;
    s->rec = (Record*)(base + L.rec);
    s->ids = (int32_t*)(base + L.ids);
    s->glist = (int32_t*)(base + L.glist);
    s->gkey = (unsigned long long*)(base + L.gkey);
    s->gcnt = (unsigned long long*)(base + L.gcnt);
    s->rng = (float2*)(base + L.rng);
    s->dual_total = (unsigned long long*)(base + L.dual_total);
    s->clist = (uint32_t*)(base + L.clist);
    s->lcnt = (uint32_t*)(base + L.lcnt);
    s->n_list = (unsigned long long*)(base + L.n_list);
    s->list_duals = (unsigned long long*)(base + L.list_duals);
    s->ls0 = (unsigned long long*)(base + L.ls0);
    s->ls1 = (unsigned long long*)(base + L.ls1);
    s->tot = (unsigned long long*)(base + L.tot);
    s->st_t = (unsigned long long*)(base + L.st_t);
    s->st_d = (unsigned long long*)(base + L.st_d);
    s->xs0 = (unsigned long long*)(base + L.xs0);
    s->xs1 = (unsigned long long*)(base + L.xs1);
    s->fs0 = (unsigned long long*)(base + L.fs0);
    s->fs1 = (unsigned long long*)(base + L.fs1);
    s->ct0 = (unsigned long long*)(base + L.ct0);
    s->ct1 = (unsigned long long*)(base + L.ct1);
    s->sched = (Sched*)(base + L.sched);
    int log2cap = 0;
    while ((1u << log2cap) < cap) ++log2cap;
    {
        uint32_t work = cap * 4u > L.compact_tiles ? cap * 4u : L.compact_tiles;  // a lane per record quarter
        if (work < kFusedMaxTiles) work = kFusedMaxTiles;
        launch(s, AMR_KERNEL_RESET, "k_build_reset", k_build_reset, dim3(grid_for(work, 256)), dim3(256), stream, s->rec, cap,
               64 - log2cap, s->sched, s->ct0, s->ct1, L.compact_tiles, s->fs0, s->fs1, s->ls0, s->ls1,
               L.max_list_wgs, s->ctrl);
    }
    if (s->n > 0)
        launch(s, AMR_KERNEL_INSERT, "k_index_insert", k_index_insert, dim3(grid_for(s->n, 256)), dim3(256), stream, s->xyz, s->lvl,
               s->val, s->n, s->rec, s->ctrl);
    // the group list only depends on the leaves, so it is compacted before
    // the ancestors are marked, and the marking runs over it; its last
    // work-group decides the verdict
    launch(s, AMR_KERNEL_COMPACT, "k_index_compact", k_index_compact, dim3(L.compact_tiles), dim3(kCompactBlock), stream, s->rec, cap,
           s->glist, s->gkey, s->ct0, s->ct1, s->sched, L.compact_tiles, L.compact_per, s->ctrl);
    {
        const int64_t most = s->n < (int64_t)cap ? s->n : (int64_t)cap;  // at least the number of groups
        launch(s, AMR_KERNEL_MARK, "k_index_mark", k_index_mark, dim3(grid_for(most, 256)), dim3(256), stream, s->rec, s->gkey,
               s->ctrl);
    }
    hipLaunchKernelGGL(k_index_verdict, dim3(1), dim3(64), 0, stream, s->n, cap, s->grid_groups, s->ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_build_index: launch");
    s->build_captured = in_graph;
    if (!in_graph) {
        e = hipEventRecord(s->build_event, stream);
        if (e != hipSuccess) return hipfail(e, "amr_build_index: event");
    }
    s->built = true;
    s->build_tried = true;
    s->build_pending = true;
    s->build_status = kStatusPending;
    s->ids_ready = false;
    s->extractions = 0;
    ++s->build_gen;
    s->last_cap = cap;
    s->last_n = s->n;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_build_status(amr_set* s) {
    if (!s) return fail(AMR_EINVAL, "amr_build_status: set is NULL");
    if (!s->build_tried) return fail(AMR_ESTATE, "amr_build_status: no build since the last upload");
    if (!s->build_pending) {
        // read before: the same answer again
        if (s->build_status == AMR_OK) {
            g_err[0] = 0;
            return AMR_OK;
        }
        return fail(s->build_status, "amr_build_status: the last build failed (status %d)", s->build_status);
    }
    return read_build_verdict(s);
}

int amr_dual_cells(amr_set* s, int32_t* corner_level, int32_t* verts, float* vals, int64_t cap, int64_t* counts,
                   hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_dual_cells: set is NULL");
    if (!s->built) return fail(AMR_ESTATE, "amr_dual_cells: call amr_build_index first");
    if (cap < 0 || (cap > 0 && !corner_level && !verts && !vals))
        return fail(AMR_EINVAL, "amr_dual_cells: bad capacity");
    DeviceGuard dg(s->device);
    return launch_extract(s, true, 0.0f, nullptr, nullptr, nullptr, corner_level, verts, vals, cap, counts, stream);
}

int amr_isosurface(amr_set* s, float iso, float* tris, int32_t* tri_cells, int64_t* tri_dual, int64_t cap,
                   int64_t* counts, hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_isosurface: set is NULL");
    if (!s->built) return fail(AMR_ESTATE, "amr_isosurface: call amr_build_index first");
    if (!isfinite(iso)) return fail(AMR_EINVAL, "amr_isosurface: iso is not finite");
    if (cap < 0) return fail(AMR_EINVAL, "amr_isosurface: negative capacity");
    DeviceGuard dg(s->device);
    return launch_extract(s, false, iso, tris, tri_cells, tri_dual, nullptr, nullptr, nullptr, cap, counts, stream);
}


int amr_batch_create(amr_batch** out, amr_set* const* sets, int n_sets) {
    if (!out) return fail(AMR_EINVAL, "amr_batch_create: out is NULL");
    *out = nullptr;
    if (!sets || n_sets < 1 || n_sets > kMaxSets) return fail(AMR_EINVAL, "amr_batch_create: need 1..%d sets", kMaxSets);
    int dev = sets[0] ? sets[0]->device : -1;
    BatchSet* host = (BatchSet*)calloc((size_t)n_sets, sizeof(BatchSet));
    if (!host) return fail(AMR_ENOMEM, "amr_batch_create: out of host memory");
    uint32_t mg = 0;
    for (int i = 0; i < n_sets; ++i) {
        const amr_set* s = sets[i];
        if (!s || s->device != dev) {
            free(host);
            return fail(AMR_EINVAL, "amr_batch_create: set %d is NULL or on another device", i);
        }
        if (!s->built) {
            free(host);
            return fail(AMR_ESTATE, "amr_batch_create: set %d has no index", i);
        }
        host[i].rec = s->rec;
        host[i].glist = s->glist;
        host[i].gkey = s->gkey;
        host[i].ctrl = s->ctrl;
        host[i].rng = s->rng;
        host[i].rng_ok = &s->sched->rng_ok;
        host[i].bound = s->grid_groups;
        if (s->grid_groups > mg) mg = s->grid_groups;
    }
    DeviceGuard dg(dev);
    amr_batch* b = new (std::nothrow) amr_batch();
    if (!b) {
        free(host);
        return fail(AMR_ENOMEM, "amr_batch_create: out of host memory");
    }
    b->device = dev;
    b->n_sets = n_sets;
    b->max_groups = mg;
    for (int i = 0; i < n_sets; ++i) b->bound[i] = host[i].bound;
    hipError_t e = hipMalloc((void**)&b->d_sets, sizeof(BatchSet) * (size_t)n_sets);
    if (e == hipSuccess) e = hipMemcpy(b->d_sets, host, sizeof(BatchSet) * (size_t)n_sets, hipMemcpyHostToDevice);
    free(host);
    if (e != hipSuccess) {
        if (b->d_sets) (void)hipFree(b->d_sets);
        delete b;
        return hipfail(e, "amr_batch_create");
    }
    *out = b;
    g_err[0] = 0;
    return AMR_OK;
}

void amr_batch_destroy(amr_batch* b) {
    if (!b) return;
    {
        DeviceGuard dg(b->device);
        if (b->d_sets) (void)hipFree(b->d_sets);
    }
    delete b;
}

int amr_batch_workspace_bytes(const amr_batch* b, int max_jobs, int block, int unit, size_t* bytes) {
    if (!b || !bytes) return fail(AMR_EINVAL, "amr_batch_workspace_bytes: NULL argument");
    if (max_jobs < 1 || max_jobs > kMaxJobs) return fail(AMR_EINVAL, "amr_batch_workspace_bytes: 1..%d jobs", kMaxJobs);
    const int st = batch_check_shape(block, unit);
    if (st != AMR_OK) return st;
    const size_t per = (size_t)max_jobs * (size_t)batch_max_units(b, unit) * sizeof(uint32_t);
    *bytes = align256(sizeof(BatchTab)) + 2 * align256(per);
    g_err[0] = 0;
    return AMR_OK;
}

int amr_batch_isosurface(amr_batch* b, const amr_iso_job* jobs, int n_jobs, float* tris, int64_t* counts, void* ws,
                         size_t bytes, int block, int unit, hipStream_t stream) {
    if (!b || !jobs || !counts) return fail(AMR_EINVAL, "amr_batch_isosurface: NULL argument");
    size_t need = 0;
    int st = amr_batch_workspace_bytes(b, n_jobs, block, unit, &need);
    if (st != AMR_OK) return st;
    if (!ws || ((uintptr_t)ws & 255)) return fail(AMR_EINVAL, "amr_batch_isosurface: workspace NULL or unaligned");
    if (bytes < need) return fail(AMR_ENOSPACE, "amr_batch_isosurface: workspace %zu bytes, need %zu", bytes, need);
    const int64_t grid = batch_all_units(b, unit);
    if (grid > 0x7FFFFFFF) return fail(AMR_EINVAL, "amr_batch_isosurface: %lld units, too many", (long long)grid);
    DeviceGuard dg(b->device);
    const size_t per = align256((size_t)n_jobs * (size_t)batch_max_units(b, unit) * sizeof(uint32_t));
    char* w = (char*)ws;
    BatchArgs a;
    a.sets = b->d_sets;
    a.n_sets = b->n_sets;
    a.jobs = jobs;
    a.n_jobs = n_jobs;
    a.unit = unit;
    a.unit_shift = log2_of(unit);
    a.tris = tris;
    a.counts = counts;
    a.tab = (BatchTab*)w;
    a.tcnt = (uint32_t*)(w + align256(sizeof(BatchTab)));
    a.tpre = (uint32_t*)((char*)a.tcnt + per);
    hipLaunchKernelGGL(k_batch_prep, dim3(1), dim3(256), 0, stream, a);
    if (block == 128)
        hipLaunchKernelGGL(k_batch_count<16>, dim3((unsigned)grid), dim3(128), 0, stream, a);
    else
        hipLaunchKernelGGL(k_batch_count<32>, dim3((unsigned)grid), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_batch_scan, dim3(n_jobs), dim3(256), 0, stream, a);
    if (block == 128)
        hipLaunchKernelGGL(k_batch_write<16>, dim3((unsigned)grid), dim3(128), 0, stream, a);
    else
        hipLaunchKernelGGL(k_batch_write<32>, dim3((unsigned)grid), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AMR_OK : hipfail(e, "amr_batch_isosurface: launch");
}

namespace {
struct WeldLayout {
    uint32_t cap;
    uint32_t n_tiles;
    size_t key, first, vid, cslot, s0, s1, sched, total;
};

bool weld_layout(int64_t n_tris, WeldLayout& L) {
    if (n_tris < 0 || n_tris >= ((int64_t)1 << 29)) return false;
    int64_t corners = 3 * n_tris;
    uint64_t cap = 1024;
    while (cap < (uint64_t)(2 * corners)) cap <<= 1;  // load <= 1/2 even with no sharing
    L.cap = (uint32_t)cap;
    L.n_tiles = (uint32_t)((corners + kWeldTile - 1) / kWeldTile);
    size_t off = 0;
    L.key = off;
    off = align256(off + cap * 8);
    L.first = off;
    off = align256(off + cap * 4);
    L.vid = off;
    off = align256(off + cap * 4);
    L.cslot = off;
    off = align256(off + (size_t)corners * 4 + 4);
    L.s0 = off;
    off = align256(off + ((size_t)L.n_tiles + 1) * 8);
    L.s1 = off;
    off = align256(off + ((size_t)L.n_tiles + 1) * 8);
    L.sched = off;
    off = align256(off + sizeof(Sched));
    L.total = off;
    return true;
}
}  // namespace

int amr_indexed_mesh_bytes(int64_t n_tris, size_t* bytes) {
    if (!bytes) return fail(AMR_EINVAL, "amr_indexed_mesh_bytes: NULL argument");
    WeldLayout L;
    if (!weld_layout(n_tris, L)) return fail(AMR_ERANGE, "amr_indexed_mesh_bytes: n_tris out of range");
    *bytes = L.total;
    return AMR_OK;
}

namespace {
// The weld of an indexed mesh into the workspace at `base` (layout L).
int weld_into(const float* tris, const int32_t* tri_cells, int64_t n_tris, float* verts, int32_t* idx,
              int64_t cap_verts, int64_t* n_verts, char* base, const WeldLayout& L, hipStream_t stream,
              const char* who) {
    if (n_tris == 0) {
        hipLaunchKernelGGL(k_weld_empty, dim3(1), dim3(64), 0, stream, n_verts);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? AMR_OK : hipfail(e, who);
    }
    WeldWs w;
    w.key = (unsigned long long*)(base + L.key);
    w.first = (unsigned int*)(base + L.first);
    w.vid = (unsigned int*)(base + L.vid);
    w.cslot = (unsigned int*)(base + L.cslot);
    w.s0 = (unsigned long long*)(base + L.s0);
    w.s1 = (unsigned long long*)(base + L.s1);
    w.sched = (Sched*)(base + L.sched);
    w.cap = L.cap;
    int log2cap = 0;
    while ((1u << log2cap) < L.cap) ++log2cap;
    w.shift = 64 - log2cap;
    int64_t corners = 3 * n_tris;
    hipLaunchKernelGGL(k_weld_init, dim3(grid_for(L.cap, 256)), dim3(256), 0, stream, w, L.n_tiles);
    hipLaunchKernelGGL(k_weld_insert, dim3(grid_for(corners, 256)), dim3(256), 0, stream, tri_cells, corners, w);
    hipLaunchKernelGGL(k_weld_scan, dim3(L.n_tiles), dim3(kBlock), 0, stream, tris, corners, w, L.n_tiles, verts,
                       cap_verts, n_verts);
    hipLaunchKernelGGL(k_weld_index, dim3(grid_for(corners, 256)), dim3(256), 0, stream, corners, w, idx);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AMR_OK : hipfail(e, who);
}
}  // namespace

int amr_indexed_mesh(const float* tris, const int32_t* tri_cells, int64_t n_tris, float* verts, int32_t* idx,
                     int64_t cap_verts, int64_t* n_verts, void* ws, size_t bytes, hipStream_t stream) {
    WeldLayout L;
    if (!weld_layout(n_tris, L)) return fail(AMR_ERANGE, "amr_indexed_mesh: n_tris out of range");
    if (!n_verts || (n_tris > 0 && (!tris || !tri_cells || !idx)) || cap_verts < 0 || (cap_verts > 0 && !verts))
        return fail(AMR_EINVAL, "amr_indexed_mesh: bad argument");
    if (!ws || ((uintptr_t)ws & 255)) return fail(AMR_EINVAL, "amr_indexed_mesh: workspace NULL or unaligned");
    if (bytes < L.total) return fail(AMR_ENOSPACE, "amr_indexed_mesh: workspace %zu bytes, need %zu", bytes, L.total);
    return weld_into(tris, tri_cells, n_tris, verts, idx, cap_verts, n_verts, (char*)ws, L, stream,
                     "amr_indexed_mesh");
}

namespace {
// Scratch of amr_indexed_mesh_noalloc: the weld's workspace for up to
// kWeldScratchTris triangles, one copy on every GPU the library runs on,
// held until the process ends.  In host code `weld_scratch` names a host
// stand-in, not device memory: its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int64_t kWeldScratchTris = 1 << 18;
constexpr size_t kWeldScratchBytes = (size_t)40 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char weld_scratch[kWeldScratchBytes];

std::mutex g_weld_scratch_lock;
char* g_weld_scratch[kMaxDevices] = {};

// The scratch of the current device (nullptr and a message on failure).
char* weld_scratch_of_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        fail(AMR_EHIP, "amr_indexed_mesh_noalloc: no current HIP device (or more than %d)", kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_weld_scratch_lock);
    if (!g_weld_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(weld_scratch));
        if (e != hipSuccess || !ptr) {
            hipfail(e, "amr_indexed_mesh_noalloc: scratch address");
            return nullptr;
        }
        g_weld_scratch[dev] = (char*)ptr;
    }
    return g_weld_scratch[dev];
}
}  // namespace

int amr_indexed_mesh_noalloc(const float* tris, const int32_t* tri_cells, int64_t n_tris, float* verts,
                             int32_t* idx, int64_t cap_verts, int64_t* n_verts, hipStream_t stream) {
    WeldLayout L;
    if (n_tris < 0 || n_tris > kWeldScratchTris || !weld_layout(n_tris, L) || L.total > kWeldScratchBytes)
        return fail(AMR_ERANGE, "amr_indexed_mesh_noalloc: n_tris must lie in [0, %lld] (a %zu-byte scratch per GPU)",
                    (long long)kWeldScratchTris, kWeldScratchBytes);
    if (!n_verts || (n_tris > 0 && (!tris || !tri_cells || !idx)) || cap_verts < 0 || (cap_verts > 0 && !verts))
        return fail(AMR_EINVAL, "amr_indexed_mesh_noalloc: bad argument");
    char* base = weld_scratch_of_current_device();
    if (!base) return AMR_EHIP;
    return weld_into(tris, tri_cells, n_tris, verts, idx, cap_verts, n_verts, base, L, stream,
                     "amr_indexed_mesh_noalloc");
}

namespace {
// Sampler workspace: per cell the offset of its dual list (int64, n + 1),
// per cell a counter (uint32), the lists (uint32 dual indices, at most 8 per
// dual), per dual its bounding box (2 x float4) and the work-group sums of
// the offset scan.
struct SmpLayout {
    int64_t nb;
    size_t off, cur, ent, box, bsum, total;
};

bool smp_layout(int64_t n, int64_t m, SmpLayout& L) {
    if (n < 0 || m < 0 || m > (int64_t)0xFFFFFFFFll) return false;
    L.nb = (n + 256 * kSmpPer - 1) / (256 * kSmpPer);
    if (L.nb < 1) L.nb = 1;
    size_t o = 0;
    L.off = o;
    o = align256(o + (size_t)(n + 1) * 8);
    L.cur = o;
    o = align256(o + (size_t)n * 4 + 4);
    L.ent = o;
    o = align256(o + (size_t)m * 8 * 4 + 4);
    L.box = o;
    o = align256(o + (size_t)m * 32 + 32);
    L.bsum = o;
    o = align256(o + (size_t)(L.nb + 1) * 8);
    L.total = o;
    return true;
}
}  // namespace

int amr_sampler_bytes(const amr_set* s, int64_t n_duals, size_t* bytes) {
    if (!s || !bytes) return fail(AMR_EINVAL, "amr_sampler_bytes: NULL argument");
    SmpLayout L;
    if (!smp_layout(s->n, n_duals, L)) return fail(AMR_ERANGE, "amr_sampler_bytes: n_duals out of range");
    *bytes = L.total;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_sampler_build(amr_set* s, const int32_t* verts, int64_t n_duals, void* ws, size_t bytes,
                      hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_sampler_build: set is NULL");
    if (!s->built) return fail(AMR_ESTATE, "amr_sampler_build: call amr_build_index first");
    SmpLayout L;
    if (!smp_layout(s->n, n_duals, L)) return fail(AMR_ERANGE, "amr_sampler_build: n_duals out of range");
    if (n_duals > 0 && !verts) return fail(AMR_EINVAL, "amr_sampler_build: verts is NULL");
    if (!ws || ((uintptr_t)ws & 255)) return fail(AMR_EINVAL, "amr_sampler_build: workspace NULL or not 256-B aligned");
    if (bytes < L.total)
        return fail(AMR_ENOSPACE, "amr_sampler_build: workspace of %zu bytes, need %zu", bytes, L.total);
    DeviceGuard dg(s->device);
    int st = ensure_ids(s, stream);
    if (st != AMR_OK) return st;
    char* b = (char*)ws;
    int64_t* off = (int64_t*)(b + L.off);
    uint32_t* cur = (uint32_t*)(b + L.cur);
    uint32_t* ent = (uint32_t*)(b + L.ent);
    int64_t* bsum = (int64_t*)(b + L.bsum);
    const int64_t n = s->n;
    hipLaunchKernelGGL(k_smp_clear, dim3(grid_for(n, 256)), dim3(256), 0, stream, cur, n);
    if (n_duals > 0)
        hipLaunchKernelGGL(k_smp_count, dim3(grid_for(n_duals, 256)), dim3(256), 0, stream, verts, n_duals, n, s->xyz,
                           s->lvl, cur, (float4*)(b + L.box));
    hipLaunchKernelGGL(k_smp_block_sums, dim3(L.nb), dim3(256), 0, stream, cur, n, bsum);
    hipLaunchKernelGGL(k_smp_scan_sums, dim3(1), dim3(256), 0, stream, bsum, L.nb);
    hipLaunchKernelGGL(k_smp_offsets, dim3(L.nb), dim3(256), 0, stream, cur, n, bsum, L.nb, off);
    if (n_duals > 0)
        hipLaunchKernelGGL(k_smp_fill, dim3(grid_for(n_duals, 256)), dim3(256), 0, stream, verts, n_duals, n, off,
                           cur, ent);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_sampler_build: launch");
    s->smp_gen = s->build_gen;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_sample(amr_set* s, const int32_t* corner_level, const int32_t* verts, int64_t n_duals, const void* ws,
               size_t bytes, const float* points, int64_t n_points, float* values, int64_t* dual,
               hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_sample: set is NULL");
    if (!s->built || s->smp_gen != s->build_gen)
        return fail(AMR_ESTATE, "amr_sample: no sampler built for the current index (amr_sampler_build)");
    SmpLayout L;
    if (!smp_layout(s->n, n_duals, L)) return fail(AMR_ERANGE, "amr_sample: n_duals out of range");
    if (n_points < 0) return fail(AMR_EINVAL, "amr_sample: negative n_points");
    if (n_points > 0 && (!points || !values)) return fail(AMR_EINVAL, "amr_sample: NULL points or values");
    if (n_duals > 0 && (!corner_level || !verts)) return fail(AMR_EINVAL, "amr_sample: NULL dual arrays");
    if (!ws || ((uintptr_t)ws & 255)) return fail(AMR_EINVAL, "amr_sample: workspace NULL or not 256-B aligned");
    if (bytes < L.total) return fail(AMR_ENOSPACE, "amr_sample: workspace of %zu bytes, need %zu", bytes, L.total);
    if (n_points == 0) {
        g_err[0] = 0;
        return AMR_OK;
    }
    DeviceGuard dg(s->device);
    const char* b = (const char*)ws;
    SampleArgs a;
    a.rec = s->rec;
    a.ids = s->ids;
    a.ctrl = s->ctrl;
    a.xyz = s->xyz;
    a.lvl = s->lvl;
    a.val = s->val;
    a.n = s->n;
    a.corner_level = corner_level;
    a.verts = verts;
    a.off = (const int64_t*)(b + L.off);
    a.ent = (const uint32_t*)(b + L.ent);
    a.box = (const float4*)(b + L.box);
    a.pts = points;
    a.n_pts = n_points;
    a.out = values;
    a.dual = dual;
    launch(s, AMR_KERNEL_SAMPLE, "k_smp_query", k_smp_query, dim3(grid_for(n_points, 256)), dim3(256), stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_sample: launch");
    g_err[0] = 0;
    return AMR_OK;
}

namespace {
// Sorted-index workspace: keys and cell indices twice (the passes
// alternate), the digit histograms of the tiles and their offsets, and the
// work-group sums of the offset scan.
struct SortLayout {
    uint32_t n_tiles;
    int64_t n_hist, nb;
    size_t ka, kb, va, vb, hist, off, bsum, total;
};

SortLayout sort_layout(int64_t n) {
    SortLayout L{};
    L.n_tiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
    if (L.n_tiles == 0) L.n_tiles = 1;
    L.n_hist = (int64_t)256 * L.n_tiles;
    L.nb = (L.n_hist + 256 * kSmpPer - 1) / (256 * kSmpPer);
    size_t o = 0;
    L.ka = o;
    o = align256(o + (size_t)n * 8 + 8);
    L.kb = o;
    o = align256(o + (size_t)n * 8 + 8);
    L.va = o;
    o = align256(o + (size_t)n * 4 + 4);
    L.vb = o;
    o = align256(o + (size_t)n * 4 + 4);
    L.hist = o;
    o = align256(o + (size_t)L.n_hist * 4);
    L.off = o;
    o = align256(o + (size_t)(L.n_hist + 1) * 8);
    L.bsum = o;
    o = align256(o + (size_t)(L.nb + 1) * 8);
    L.total = o;
    return L;
}

SortedIndex sorted_view(const amr_set* s) {
    SortedIndex si;
    si.keys = s->srt_keys;
    si.cells = s->srt_cells;
    for (int l = 0; l < kMaxLevel + 2; ++l) si.lo[l] = s->srt_lo[l];
    si.lmin = s->lmin;
    si.lmax = s->lmax;
    si.bits = s->srt_bits;
    si.ox = s->origin[0];
    si.oy = s->origin[1];
    si.oz = s->origin[2];
    return si;
}

// the index a locate call names: AMR_ESTATE when it has not been built
int index_ready(amr_set* s, int kind, const char* who, hipStream_t stream) {
    if (kind == AMR_INDEX_HASH) {
        if (!s->built) return fail(AMR_ESTATE, "%s: call amr_build_index first", who);
        return ensure_ids(s, stream);
    }
    if (kind == AMR_INDEX_SORTED) {
        if (!s->uploaded || s->srt_gen != s->upload_gen)
            return fail(AMR_ESTATE, "%s: call amr_build_sorted_index first", who);
        return AMR_OK;
    }
    return fail(AMR_EINVAL, "%s: unknown index %d", who, kind);
}
}  // namespace

int amr_sorted_index_bytes(amr_set* s, size_t* bytes) {
    if (!s || !bytes) return fail(AMR_EINVAL, "amr_sorted_index_bytes: NULL argument");
    if (!s->uploaded) return fail(AMR_ESTATE, "amr_sorted_index_bytes: call amr_upload first");
    DeviceGuard dg(s->device);
    const int st = upload_verdict(s);
    if (st != AMR_OK) return st;
    *bytes = sort_layout(s->n).total;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_build_sorted_index(amr_set* s, void* ws, size_t bytes, hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_build_sorted_index: set is NULL");
    if (!s->uploaded) return fail(AMR_ESTATE, "amr_build_sorted_index: call amr_upload first");
    if (!ws || ((uintptr_t)ws & 255))
        return fail(AMR_EINVAL, "amr_build_sorted_index: workspace NULL or not 256-B aligned");
    DeviceGuard dg(s->device);
    int st = upload_verdict(s);  // the geometry comes from the host copy of the verdict
    if (st != AMR_OK) return st;
    const SortLayout L = sort_layout(s->n);
    if (bytes < L.total)
        return fail(AMR_ENOSPACE, "amr_build_sorted_index: workspace of %zu bytes, need %zu", bytes, L.total);
    // bits per axis of the offset coordinates, and of the level above lmin
    int64_t span = 1;
    for (int a = 0; a < 3; ++a) {
        const int64_t e = (int64_t)s->host_ctrl->res.hi[a] - s->origin[a];
        if (e > span) span = e;
    }
    int bits = 0;
    while (((int64_t)1 << bits) < span) ++bits;
    int lbits = 0;
    while ((1 << lbits) < s->lmax - s->lmin + 1) ++lbits;
    if (3 * bits + lbits > 64)
        return fail(AMR_ERANGE, "amr_build_sorted_index: %d bits per axis and %d level bits exceed a 64-bit key", bits,
                    lbits);
    const int passes = s->n > 0 ? (3 * bits + lbits + 7) / 8 : 0;
    char* b = (char*)ws;
    uint64_t* k0 = (uint64_t*)(b + L.ka);
    uint64_t* k1 = (uint64_t*)(b + L.kb);
    uint32_t* v0 = (uint32_t*)(b + L.va);
    uint32_t* v1 = (uint32_t*)(b + L.vb);
    uint32_t* hist = (uint32_t*)(b + L.hist);
    int64_t* off = (int64_t*)(b + L.off);
    int64_t* bsum = (int64_t*)(b + L.bsum);
    if (s->n > 0)
        hipLaunchKernelGGL(k_sort_keys, dim3(grid_for(s->n, 256)), dim3(256), 0, stream, s->xyz, s->lvl, s->n,
                           s->origin[0], s->origin[1], s->origin[2], s->lmin, bits, k0, v0);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_sort_hist, dim3(L.n_tiles), dim3(256), 0, stream, k0, s->n, 8 * p, L.n_tiles, hist);
        hipLaunchKernelGGL(k_smp_block_sums, dim3(L.nb), dim3(256), 0, stream, hist, L.n_hist, bsum);
        hipLaunchKernelGGL(k_smp_scan_sums, dim3(1), dim3(256), 0, stream, bsum, L.nb);
        hipLaunchKernelGGL(k_smp_offsets, dim3(L.nb), dim3(256), 0, stream, hist, L.n_hist, bsum, L.nb, off);
        hipLaunchKernelGGL(k_sort_scatter, dim3(L.n_tiles), dim3(256), 0, stream, k0, v0, s->n, 8 * p, L.n_tiles,
                           off, k1, v1);
        uint64_t* tk = k0;
        k0 = k1;
        k1 = tk;
        uint32_t* tv = v0;
        v0 = v1;
        v1 = tv;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_build_sorted_index: launch");
    // level l's keys follow those of the finer levels (the level is the top digit)
    int64_t acc = 0;
    for (int l = 0; l <= kMaxLevel + 1; ++l) {
        s->srt_lo[l] = acc;
        if (l <= kMaxLevel) acc += (int64_t)s->level_count[l];
    }
    s->srt_keys = k0;
    s->srt_cells = v0;
    s->srt_bits = bits;
    s->srt_gen = s->upload_gen;
    g_err[0] = 0;
    return AMR_OK;
}

int amr_locate(amr_set* s, int index, const int32_t* points, int64_t n, int32_t* cells, hipStream_t stream) {
    if (!s) return fail(AMR_EINVAL, "amr_locate: set is NULL");
    if (n < 0 || (n > 0 && (!points || !cells))) return fail(AMR_EINVAL, "amr_locate: bad arguments");
    DeviceGuard dg(s->device);
    const int st = index_ready(s, index, "amr_locate", stream);
    if (st != AMR_OK) return st;
    if (n == 0) {
        g_err[0] = 0;
        return AMR_OK;
    }
    const SortedIndex si = sorted_view(s);
    if (index == AMR_INDEX_SORTED)
        hipLaunchKernelGGL(k_locate<true>, dim3(grid_for(n, 256)), dim3(256), 0, stream, s->rec, s->ids, s->ctrl, si,
                           points, n, cells);
    else
        hipLaunchKernelGGL(k_locate<false>, dim3(grid_for(n, 256)), dim3(256), 0, stream, s->rec, s->ids, s->ctrl,
                           si, points, n, cells);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_locate: launch");
    g_err[0] = 0;
    return AMR_OK;
}

int amr_snap_count(amr_set* s, int index, uint64_t* out, hipStream_t stream) {
    if (!s || !out) return fail(AMR_EINVAL, "amr_snap_count: NULL argument");
    DeviceGuard dg(s->device);
    const int st = index_ready(s, index, "amr_snap_count", stream);
    if (st != AMR_OK) return st;
    const SortedIndex si = sorted_view(s);
    unsigned long long* o = (unsigned long long*)out;
    hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, stream, o);
    const int grid = s->n > 0 ? (grid_for(s->n, 256) < 1024 ? grid_for(s->n, 256) : 1024) : 1;
    if (index == AMR_INDEX_SORTED)
        launch(s, AMR_KERNEL_SNAP, "k_snap<true>", k_snap<true>, dim3(grid), dim3(256), stream, s->xyz, s->lvl, s->n, s->rec, s->ids,
               s->ctrl, si, o);
    else
        launch(s, AMR_KERNEL_SNAP, "k_snap<false>", k_snap<false>, dim3(grid), dim3(256), stream, s->xyz, s->lvl, s->n, s->rec,
               s->ids, s->ctrl, si, o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "amr_snap_count: launch");
    g_err[0] = 0;
    return AMR_OK;
}

int amr_time_kernel(amr_set* s, int kernel, hipEvent_t start, hipEvent_t stop) {
    if (!s) return fail(AMR_EINVAL, "amr_time_kernel: set is NULL");
    if (kernel < 0 || kernel > AMR_KERNEL_SNAP) return fail(AMR_EINVAL, "amr_time_kernel: unknown kernel %d", kernel);
    if (kernel != 0 && (!start || !stop)) return fail(AMR_EINVAL, "amr_time_kernel: NULL event");
    s->time_kernel = kernel;
    s->time_start = start;
    s->time_stop = stop;
    if (kernel != 0) s->timed_name = "";
    g_err[0] = 0;
    return AMR_OK;
}

const char* amr_timed_kernel_name(const amr_set* s) { return s ? s->timed_name : ""; }

const char* amr_last_error(void) { return g_err; }

}  // extern "C"
