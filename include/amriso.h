/*
 * amriso.h -- C ABI of libamriso.so: dual cells and crack-free iso-surfaces
 * of AMR data on an AMD Instinct MI355X (gfx950).
 *
 * Method: I. Wald, "A Simple, General, and GPU Friendly Method for Computing
 * Dual Mesh and Iso-Surfaces of Adaptive Mesh Refinement (AMR) Data"
 * (arXiv 2004.08475).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Cells (paper sec. 3.1): an AMR data set is a flat, unsorted list of
 *    cells (i,j,k;l).  Level 0 is the finest; a level-l cell has width 2^l, a
 *    lower corner that is a multiple of 2^l and covers [lo, lo + 2^l) on
 *    each axis.  Cells carry one float value at their centre lo + 2^l/2.
 *    No hierarchy, bricks or level balance are assumed (sec. 3.1, sec. 6):
 *    any level jumps and holes are allowed; cells must not overlap.
 *  - Memory: every pointer marked "device" is device memory of the set's
 *    GPU, owned by the caller (for instance a torch tensor).  The library
 *    only borrows it.  The library itself allocates one small control block
 *    per set (a few KB, freed by amr_destroy).
 *  - Streams: every call enqueues its work on the given HIP stream.  Calls
 *    on one set must be issued on one stream at a time (they share the
 *    set's scratch space inside the index workspace).
 *  - Errors: functions return an amr_status; they never abort or throw.
 *    amr_last_error() gives a message for the calling thread.  Problems
 *    with the cells themselves (bad fields, overlaps, a hash table too
 *    small) are found by kernels; they are reported by the next call that
 *    waits on the host for them (amr_build_status, amr_index_bytes), and
 *    extractions enqueued after a failed build write -1 into their counts
 *    and nothing else.
 *  - Graph capture: amr_upload, amr_build_index (for as many cells as an
 *    earlier build of the set, or after amr_index_bytes sized the table),
 *    amr_dual_cells, amr_isosurface, amr_batch_isosurface and
 *    amr_indexed_mesh do no host synchronisation and can be captured in a
 *    HIP graph together.
 *  - Limits: 0 <= level <= 20; every coordinate c satisfies
 *    -2^23 <= c and c + 2^level <= 2^23 (cell centres are then exact in
 *    float32); per axis, max(c + 2^level) - min(c) + 2^(Lmax+3) <= 2^20
 *    finest units, Lmax being the coarsest level present.  Outside:
 *    AMR_ERANGE.
 */
#ifndef AMRISO_H
#define AMRISO_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amr_set amr_set; /* opaque, library-owned host handle */

typedef enum amr_status {
    AMR_OK = 0,
    AMR_EINVAL = -1,   /* bad argument, misaligned corner, level < 0, non-finite value */
    AMR_ERANGE = -2,   /* outside the coordinate / level limits above */
    AMR_EOVERLAP = -3, /* two cells overlap (duplicates or nested cells) */
    AMR_ENOSPACE = -4, /* a caller buffer or the index workspace is too small */
    AMR_ESTATE = -5,   /* call out of order (e.g. extraction before amr_build_index) */
    AMR_EHIP = -6,     /* a HIP runtime call failed */
    AMR_ENOMEM = -7    /* host or control-block allocation failed */
} amr_status;

/* Create an empty set bound to HIP device `hip_device`.  *out receives the
   handle.  Returns AMR_EINVAL for a bad device, AMR_EHIP / AMR_ENOMEM on
   allocation failure. */
int amr_create(amr_set** out, int hip_device);

/* Destroy a set (NULL is allowed).  Waits for nothing: the caller must have
   synchronised the set's stream. */
void amr_destroy(amr_set* set);

/* Input stage (paper sec. 3.1; the cell list of the pipeline in the figure
   of its sec. 5.2).  Borrows n cells in structure-of-arrays form:
     xyz   device int32 [n][3]  lower corners, in finest-level units
     level device int32 [n]     levels
     value device float [n]     cell values
   The arrays must stay alive and unchanged until the set is destroyed or
   re-uploaded.  Enqueues the validation of every cell on the device (level
   range, alignment of the corner to 2^level, finite value, coordinate
   limits) and the reduction of the bounding box and per-level counts, and
   returns without waiting.  The verdict stays on the device for the build's
   kernels; the host reads it in amr_index_bytes, amr_build_index (only
   when it must size a new table) or amr_build_status, which return
   AMR_EINVAL / AMR_ERANGE for bad cells (the message names the lowest
   offending index).  This call itself only rejects bad arguments.  n == 0
   is allowed (an empty set).  Invalidates any index built before. */
int amr_upload(amr_set* set, const int32_t* xyz, const int32_t* level, const float* value, int64_t n,
               hipStream_t stream);

/* Bytes of device workspace amr_build_index needs for the uploaded set (no
   GPU work; waits for the upload's verdict if it has not been read yet, and
   returns its AMR_EINVAL / AMR_ERANGE).  It also reads the verdict of a
   build still unread: after a build that failed with AMR_ENOSPACE the
   answer grows to fit the set. */
int amr_index_bytes(const amr_set* set, size_t* bytes);

/* Cell-location index (paper sec. 3.2: the paper sorts the cells by their
   integer coordinates and binary-searches per level; this library stores
   the cells of each level in an open-addressing hash keyed by the integer
   coordinates of their 2x2x2 sibling block, so one probe returns up to
   eight same-level cells).  `workspace` is caller-owned device memory of at
   least amr_index_bytes() bytes, 256-byte aligned; it must stay alive while
   the set is used.  Enqueues the build and returns without waiting: the
   kernels also check that no two cells overlap and decide the verdict on
   the device, where the extraction kernels read it.  The host waits only
   to size a new table: when neither amr_index_bytes nor an earlier build of
   as many cells (whose table the workspace still fits) has done so, the
   call waits for the upload's verdict first.  Returns at once the upload's
   AMR_EINVAL / AMR_ERANGE when that verdict was read and bad, AMR_ENOSPACE
   for a workspace below the table's size, AMR_ESTATE before amr_upload (or
   when the table would have to be sized inside a graph capture).  The
   build's own verdict comes from amr_build_status. */
int amr_build_index(amr_set* set, void* workspace, size_t bytes, hipStream_t stream);

/* Verdict of the last amr_build_index (paper sec. 3.1 assumes valid,
   non-overlapping cells; this is where bad ones are reported).  Waits on the
   host until that build has run, then returns AMR_OK, the upload's
   AMR_EINVAL / AMR_ERANGE for bad cells, AMR_EOVERLAP for duplicate or
   nested cells (the message names one of them), AMR_ENOSPACE if the hash
   table was too small (query amr_index_bytes again and rebuild with a
   larger workspace), or AMR_ESTATE when no build followed the last upload.
   A build enqueued inside a graph capture is waited for with a device-wide
   synchronisation.  Calling it again returns the same verdict. */
int amr_build_status(amr_set* set);

/* Dual cells (paper sec. 4.2-4.4).  For every cell and each of its 8
   corners, the logical same-level dual centred on that corner is snapped to
   the actual cells around it and emitted unless a vertex is missing
   (rule 1), lies on a finer level (rule 2) or is a same-level cell that
   precedes the generating one (rule 3), so every dual is emitted once.
   Outputs (device, may be NULL when cap == 0):
     corner_level int32 [cap][4]  (P.x, P.y, P.z, l): the dual's centre
                                  vertex P (a cell corner) and its level
     verts        int32 [cap][8]  indices (into the uploaded arrays) of the
                                  cells at slots s = ex + 2*ey + 4*ez,
                                  i.e. the cells containing P + (e - 1)*2^l
     vals         float [cap][8]  the values of those cells (so that later
                                  passes over the duals read them in order)
   counts: device int64 [2]; counts[0] = counts[1] = number of emitted duals
   (-1 if the build failed).  Records past cap are not written.  Asynchronous: the caller reads counts
   and re-runs with a larger buffer when counts[0] > cap.  The order of the
   records is fixed for a given index.  Returns AMR_ESTATE before
   amr_build_index. */
int amr_dual_cells(amr_set* set, int32_t* corner_level, int32_t* verts, float* vals, int64_t cap,
                   int64_t* counts, hipStream_t stream);

/* Iso-surface (paper sec. 5): every emitted dual, degenerate or not, is a
   hexahedron with its vertices at the centres of its 8 cells and goes
   through Marching Cubes (bit s of the case is set when the value at slot s
   is >= iso).  Triangles whose three vertices are not distinct (two of
   their hexahedron edges join the same pair of cells) are dropped.  On a
   cut edge, A is the end with value < iso and B the end with value >= iso;
   the vertex is fmaf(t, cB - cA, cA) with t = (iso - vA) / (vB - vA) in
   IEEE float32.  The surface is crack-free: faces shared by two duals yield
   identical vertices.
   Outputs (device, each may be NULL; all NULL with cap == 0 counts only):
     tris      float [cap][3][3]  vertex positions, ordered so that the
                                  right-hand normal points into the >= iso
                                  side
     tri_cells int32 [cap][3][2]  per vertex, the (A, B) cell indices of its
                                  edge (a weld key for an indexed mesh)
     tri_dual  int64 [cap]        index of the generating dual in the order
                                  amr_dual_cells writes them (64 bits: a set
                                  may emit more than 2^31 duals)
   counts: device int64 [2]; counts[0] = triangles, counts[1] = emitted
   duals (both -1 if the build failed).  Triangles past cap are not
   written.  Asynchronous and free of host synchronisation, so it can be
   captured in a HIP graph (a captured call stays valid until the set is
   built again).  Returns AMR_EINVAL for a non-finite iso, AMR_ESTATE before
   amr_build_index.
   Range culling (not part of the paper; outputs are identical with or
   without it): the second extraction after a build (this call or
   amr_dual_cells) also records, per 2x2x2 group of cells, the minimum and
   maximum cell value of the group's 4x4x4 neighbourhood (8 bytes per group,
   inside the index workspace) and the set's dual count; a set extracted
   only once never pays for that.  From the third extraction on, calls that
   pass tri_dual == NULL skip every group whose range lies entirely below
   iso or entirely at or above it: all its duals have Marching Cubes case 0
   or 255. */
int amr_isosurface(amr_set* set, float iso, float* tris, int32_t* tri_cells, int64_t* tri_dual, int64_t cap,
                   int64_t* counts, hipStream_t stream);

/* ---------------------------------------------------------------------------
   Batched iso-surfaces (many iso-values and/or many sets in one enqueue).
   The dual cells do not depend on the field (paper sec. 4), so a batched
   run reads each unit of a set's groups and their neighbourhoods once per
   pass and runs Marching Cubes (paper sec. 5) for every job on that set
   against them; groups whose neighbourhood value range straddles no job's
   iso are skipped (before their neighbourhood is read when the set has
   recorded ranges, see amr_isosurface).  A counting pass over all units of
   all sets, a per-job scan and a writing pass handle all jobs.  For a job
   on set s with iso v, the triangles, their order and every bit of their
   positions equal those of amr_isosurface(s, v) (no cell pairs or dual
   indices are written here).
   --------------------------------------------------------------------------- */

typedef struct amr_batch amr_batch; /* opaque, library-owned host handle */

/* One job of a batch; the array of jobs lives in device memory, so iso-values
   can be changed between launches (e.g. between replays of a HIP graph). */
typedef struct amr_iso_job {
    float iso;          /* iso-value (finite; otherwise the job counts -1) */
    int32_t set;        /* index into the batch's sets (otherwise the job counts -1) */
    int64_t out_offset; /* first triangle slot of this job in the output */
    int64_t out_cap;    /* triangles this job may write (more are counted only) */
} amr_iso_job;

/* Create a batch over n_sets (1..256) indexed sets of one device.  The
   batch reads each set's index in place: the sets must not be uploaded or
   built again while the batch is used.  Allocates a small device table
   (freed by amr_batch_destroy); synchronous.  Returns AMR_ESTATE if a set
   has no index, AMR_EINVAL for bad arguments. */
int amr_batch_create(amr_batch** out, amr_set* const* sets, int n_sets);

void amr_batch_destroy(amr_batch* batch);

/* Device workspace bytes for up to max_jobs jobs with `block` threads per
   work-group (128 or 256: chunks of 16 or 32 groups of 2x2x2 cells, eight
   threads each) and `unit` groups of a set per work-group (a power of two,
   64..1024): 2 x 4 bytes per (job, unit of the largest set) plus 10 KB.
   AMR_EINVAL for any other shape. */
int amr_batch_workspace_bytes(const amr_batch* batch, int max_jobs, int block, int unit, size_t* bytes);

/* Enqueue the batched run of n_jobs jobs (1 <= n_jobs <= 256): four kernel
   launches on `stream` (job layout, per-unit counts, per-job scan, writes).
     jobs      device amr_iso_job [n_jobs]
     tris      device float [..][3][3]: job j writes triangles
               out_offset .. out_offset + min(count, out_cap) - 1 (NULL:
               nothing is written; give out_cap 0 to skip the writing pass)
     counts    device int64 [n_jobs]: full triangle count of each job (-1
               for an invalid job or a set whose build failed)
     workspace device, >= amr_batch_workspace_bytes(n_jobs, block, unit),
               256-byte aligned, no initial contents needed; runs that share
               a workspace must not overlap in time.
     block     128 or 256;  unit 64, 128, .., 1024
   No host synchronisation, no memset, no allocation: capturable in a HIP
   graph. */
int amr_batch_isosurface(amr_batch* batch, const amr_iso_job* jobs, int n_jobs, float* tris, int64_t* counts,
                         void* workspace, size_t bytes, int block, int unit, hipStream_t stream);

/* ---------------------------------------------------------------------------
   Indexed face set (paper sec. 5.2): the fat triangles share vertices; each
   shared vertex gets one index.  The paper sorts the vertices by position
   and numbers the first of every run; here a vertex is identified by the
   (A, B) cell pair of its edge (amr_isosurface's tri_cells output), an exact
   integer key -- equal keys always have bit-identical positions.  Vertices
   are numbered in order of first appearance (triangle-major, corner-minor),
   so the result does not depend on scheduling.
   --------------------------------------------------------------------------- */

/* Workspace bytes for n_tris triangles (host-only). */
int amr_indexed_mesh_bytes(int64_t n_tris, size_t* bytes);

/* tris      device float [n_tris][3][3], tri_cells device int32 [n_tris][3][2]
   verts     device float [cap_verts][3]: unique vertices, first appearance order
   idx       device int32 [n_tris][3]: vertex index of every corner
   n_verts   device int64 [1]: number of unique vertices (verts past cap_verts
             are not written; idx is always complete)
   workspace device, >= amr_indexed_mesh_bytes(n_tris), 256-byte aligned;
             no initial contents needed.
   No host synchronisation.  Returns AMR_ERANGE unless 0 <= n_tris < 2^29,
   AMR_EINVAL for NULL arrays or an unaligned workspace, AMR_ENOSPACE for a
   workspace below amr_indexed_mesh_bytes. */
int amr_indexed_mesh(const float* tris, const int32_t* tri_cells, int64_t n_tris, float* verts, int32_t* idx,
                     int64_t cap_verts, int64_t* n_verts, void* workspace, size_t bytes, hipStream_t stream);

/* The same weld without allocating anything and without a workspace, for
   callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid allocation).  The weld's
   scratch is a 40 MiB array in the library's device code, one per GPU
   (held until the process ends), found on each device's first call with
   that device current; the call runs on the current device.  Every call on
   one GPU shares that array: calls that overlap in time on one GPU race
   (use one stream, or order them).  Arguments as amr_indexed_mesh; returns
   AMR_ERANGE unless 0 <= n_tris <= 262144, AMR_EINVAL for NULL arrays,
   AMR_EHIP if the scratch's address cannot be had.  No host
   synchronisation, no allocation. */
int amr_indexed_mesh_noalloc(const float* tris, const int32_t* tri_cells, int64_t n_tris, float* verts,
                             int32_t* idx, int64_t cap_verts, int64_t* n_verts, hipStream_t stream);

/* ---------------------------------------------------------------------------
   Dual-mesh interpolant.  The paper names the dual mesh as an interpolant of
   the cell values (sec. 5, after Moran et al.) and leaves volume rendering
   over it to future work (sec. 7) without defining the interpolant.  Here a
   dual (from amr_dual_cells) is the trilinear hexahedron over the centres
   of its 8 vertex cells, slot s = ex + 2*ey + 4*ez at parameter
   (ex, ey, ez), carrying the trilinear interpolant of their values.  A
   point takes the value of the dual whose map reaches it; where several
   reach it (shared faces, and duals that overlap when their cells span
   three or more levels) the dual with the smallest (level, P.z, P.y, P.x)
   wins.  The map sends each cube corner to its slot's cell centre exactly,
   so a dual reaches the centres of its vertex cells (there the value is
   that cell's).  The candidates of a point are the duals having the point's
   cell as a vertex; elsewhere the inverse map is Newton's method in float64 from the
   dual's centre (40 steps, each clamped to [-1/2, 3/2] per axis), and a
   dual reaches the point when every Jacobian on the way had |det| > 1e-14,
   the final residual is below 1e-9 and the parameter lies in
   [-1e-9, 1 + 1e-9] on every axis.
   --------------------------------------------------------------------------- */

/* Workspace bytes of a sampler over n_duals duals of the set's n cells
   (host-only): int64 [n+1] list offsets, uint32 [n] counters, uint32
   [8*n_duals] lists, a few KB of scan sums.  AMR_ERANGE for n_duals outside
   [0, 2^32). */
int amr_sampler_bytes(const amr_set* set, int64_t n_duals, size_t* bytes);

/* Build the map from every cell to the duals that have it as a vertex.
     verts     device int32 [n_duals][8]: vertex cells of the duals, as
               amr_dual_cells writes them (entries outside [0, n) are ignored)
     workspace device, >= amr_sampler_bytes(n_duals), 256-byte aligned; no
               initial contents needed; owned by the caller and read by
               amr_sample
   Asynchronous, no host synchronisation.  The sampler stays valid until the
   set is uploaded or built again.  Returns AMR_ESTATE before
   amr_build_index, AMR_ENOSPACE for a short workspace. */
int amr_sampler_build(amr_set* set, const int32_t* verts, int64_t n_duals, void* workspace, size_t bytes,
                      hipStream_t stream);

/* Interpolated values at n_points points.
     corner_level, verts  device int32 [n_duals][4], [n_duals][8]: the same
               dual list the sampler was built over (unchanged since)
     workspace the sampler's workspace (amr_sampler_build)
     points    device float [n_points][3], in finest-level units (the
               coordinates of the cells)
     values    device float [n_points]: the interpolant evaluated in float64
               and rounded to float32; NaN where no dual reaches the point
     dual      device int64 [n_points] or NULL: index of the winning dual in
               the list, -1 where none
   Asynchronous, no host synchronisation.  Returns AMR_ESTATE when no
   sampler was built for the current index, AMR_EINVAL for bad arguments. */
int amr_sample(amr_set* set, const int32_t* corner_level, const int32_t* verts, int64_t n_duals,
               const void* workspace, size_t bytes, const float* points, int64_t n_points, float* values,
               int64_t* dual, hipStream_t stream);

/* ---------------------------------------------------------------------------
   Point location: the index above against the paper's own scheme (sec. 3.2:
   the cells sorted by their integer coordinates, a binary search per
   level, a hit counting only when its level matches), built here with a
   radix sort of (level, Morton code of the level-l coordinates).  Both
   answer the same queries; amr_snap_count runs the snap queries of every
   cell through either, which is how the extraction's index was chosen.
   --------------------------------------------------------------------------- */
enum amr_index_kind {
    AMR_INDEX_HASH = 0,   /* the index of amr_build_index */
    AMR_INDEX_SORTED = 1  /* the index of amr_build_sorted_index */
};

/* Workspace bytes of the sorted index of the uploaded set: 24 bytes per
   cell plus 3 KB per 4096 cells.  Waits for the upload's verdict (and
   returns its AMR_EINVAL / AMR_ERANGE). */
int amr_sorted_index_bytes(amr_set* set, size_t* bytes);

/* Build the sorted index into `workspace` (device, caller-owned, >=
   amr_sorted_index_bytes, 256-byte aligned, kept alive while it is used).
   Waits on the host for the upload's verdict, then enqueues the sort
   without waiting.  Valid until the next amr_upload.  Independent of
   amr_build_index. */
int amr_build_sorted_index(amr_set* set, void* workspace, size_t bytes, hipStream_t stream);

/* The cell containing each point.
     points device int32 [n][3]: positions in finest-level units (a cell of
            level l at lower corner c contains [c, c + 2^l) on each axis)
     cells  device int32 [n]: input index of the containing cell, -1 where
            no cell contains the point
   index: AMR_INDEX_HASH (after amr_build_index) or AMR_INDEX_SORTED
   (after amr_build_sorted_index); AMR_ESTATE when that index is not built.
   Both give the same answer.  Asynchronous. */
int amr_locate(amr_set* set, int index, const int32_t* points, int64_t n, int32_t* cells, hipStream_t stream);

/* The snap queries of the paper's method (sec. 4.4) for every cell: the 27
   points lo + o * 2^l, o in {-1, 0, 1}^3 (the slot points of the cell's 8
   corner duals), each located through `index`.  out: device uint64 [2]:
   out[0] = points found in some cell, out[1] = the sum over them of (cell
   index + 1); both indexes give the same.  Asynchronous. */
int amr_snap_count(amr_set* set, int index, uint64_t* out, hipStream_t stream);

/* ---------------------------------------------------------------------------
   Measurement: HIP events around one kernel.  The next launch of the named
   kernel for this set is made with hipExtLaunchKernelGGL, which records
   `start` just before the kernel runs and `stop` just after it, on the
   stream the kernel runs on; hipEventElapsedTime then gives the kernel's own
   duration, without the gaps between launches.  One-shot: later launches
   are plain again.  kernel == 0 disarms.  The events are the caller's.
   --------------------------------------------------------------------------- */
enum amr_kernel {
    AMR_KERNEL_UPLOAD = 1,   /* validation and reduction of the cells (amr_upload) */
    AMR_KERNEL_RESET = 2,    /* clearing of the hash table (amr_build_index) */
    AMR_KERNEL_INSERT = 3,   /* insertion of every cell into the table (amr_build_index) */
    AMR_KERNEL_COMPACT = 4,  /* group list of the table (amr_build_index) */
    AMR_KERNEL_MARK = 5,     /* ancestor marks and the build's verdict (amr_build_index) */
    AMR_KERNEL_EXTRACT = 6,  /* first extraction pass of a call: the fused pass or the count pass */
    AMR_KERNEL_WRITE = 7,    /* write pass of a call that has one */
    AMR_KERNEL_SAMPLE = 8,   /* point queries of amr_sample */
    AMR_KERNEL_SNAP = 9      /* snap queries of amr_snap_count */
};

int amr_time_kernel(amr_set* set, int kernel, hipEvent_t start, hipEvent_t stop);

/* Name of the kernel the last armed timing of this set was applied to, as
   rocprofv3 shows it without its arguments ("k_count<false>",
   "k_extract<false, 0>", ...); "" while a timing is armed and has not run
   yet, and before any.  The string is static. */
const char* amr_timed_kernel_name(const amr_set* set);

/* Message describing the last error on the calling thread ("" if none). */
const char* amr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AMRISO_H */
