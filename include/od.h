/*
 * od.h -- C ABI of the overdecomposed 3D Jacobi library (libod.so).
 *
 * The library runs one GPU's share of an overdecomposed structured-grid
 * computation: a 3D grid split into many more blocks ("chares") than GPUs
 * (Section III, "Managing Overdecomposition"), each chare holding its own
 * storage and doing a 7-point Jacobi sweep (the stencil workload of
 * Section V, Jacobi2D, extended to three dimensions) with halo pack,
 * exchange and unpack between neighbouring chares done device-side
 * (Section IV, intra-process transport: device-to-device, no host round
 * trip).
 *
 * Arithmetic (identical in every execution mode, every decomposition and
 * every tuned variant):
 *   u'(i,j,k) = (((((u[i-1] + u[i+1]) + u[j-1]) + u[j+1]) + u[k-1]) + u[k+1]) / 6
 * each addition rounded to the grid's type, the division correctly rounded,
 * no fused multiply-add, no flush of subnormals.  The residual of a sweep
 * is max over interior points of |u' - u|.
 *
 * Conventions for every function:
 *   - Return value: OD_OK (0) or a negative od_status.  No exception or
 *     signal crosses this boundary.  On error, od_last_error() gives a
 *     message (thread-local, valid until the next od_* call on the thread).
 *   - Device memory is caller-owned: the workspace / arena pointers are
 *     device allocations (e.g. from PyTorch) that the library carves up
 *     and never frees.  The library itself allocates no device memory.
 *   - Handles (od_grid*, od_server*) are owned by the library from the
 *     create call until the matching destroy call.
 *   - Streams are borrowed: `hip_stream` is a hipStream_t (NULL = the
 *     default stream) that must outlive the handle.
 *   - Global field layout (od_read / od_write): a dense array of the
 *     grid's type with shape (nz+2, ny+2, nx+2), x fastest.  Interior point
 *     (i,j,k), 0 <= i < nx, sits at ((k+1)*(ny+2) + (j+1))*(nx+2) + (i+1);
 *     the shell at index -1 and n holds the Dirichlet values; shell edges
 *     and corners are never read and read back as 0.
 */
#ifndef OD_H
#define OD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OD_OK = 0,
    OD_EINVAL = -22,      /* bad argument, size or configuration            */
    OD_ENOMEM = -12,      /* workspace / arena too small for the request    */
    OD_EAGAIN = -11,      /* server queue full: retry later                 */
    OD_ENOTREADY = -61,   /* request still queued or running                */
    OD_ECANCELED = -125,  /* request cancelled (server shut down)           */
    OD_ETIMEDOUT = -110,  /* a device-side wait exceeded its bound           */
    OD_ESCHED = -71,      /* a message-driven schedule check failed (a tile's
                             step counter did not advance by one, or a tile
                             ran while a neighbour was not within one step) */
    OD_EHIP = -1000       /* HIP runtime error; message in od_last_error()  */
} od_status;

typedef enum { OD_F32 = 4, OD_F64 = 8 } od_dtype;   /* value = bytes per element */

/* How od_iterate advances the grid (Section III; the per-chare mode is the
 * paper's one-kernel-sequence-per-chare execution, the others are the
 * batched forms). */
typedef enum {
    OD_PER_CHARE = 0,   /* per chare and iteration: pack kernel, D2D copies of
                           the face messages, unpack kernel, sweep kernel, on
                           a pool of non-blocking streams with events        */
    OD_FUSED = 1,       /* one launch per iteration over every chare's tiles;
                           halo exchange fused into the sweep               */
    OD_GRAPH = 2,       /* OD_FUSED launches captured once in a hipGraph and
                           replayed                                          */
    OD_PERSISTENT = 3,  /* one cooperative launch for all n iterations with a
                           device-wide barrier between iterations            */
    OD_MSGDRIVEN = 4    /* one cooperative launch per od_iterate call (split
                           every 2^23 tile-steps and 65535 steps; at most
                           2^23 - 1 tiles); each tile advances as soon
                           as the tiles it reads halos from have finished the
                           previous step (message-driven, no global barrier) */
} od_exec;

typedef struct {
    int32_t origin[3];  /* global interior coordinates of the block's first cell */
    int32_t extent[3];  /* cells along x, y, z (each >= 1)                   */
} od_block;

typedef struct {
    int64_t n[3];         /* global interior extents nx, ny, nz (each >= 1)       */
    int64_t block[3];     /* regular chare extents; {0,0,0} => derive from odf    */
    int32_t odf;          /* chares on this GPU when block is {0,0,0}; a cube k^3
                             splits k ways per dimension, otherwise a balanced
                             3-factor split with the largest factor on z         */
    const od_block* blocks; /* optional explicit (uneven, AMR-like) blocks that
                               tile the domain exactly; overrides block/odf;
                               origins/extents must share a granularity g with
                               (nx/g)(ny/g)(nz/g) <= 2^26                         */
    int32_t nblocks;
    od_dtype dtype;
    double bc[6];         /* Dirichlet values of faces x-,x+,y-,y+,z-,z+          */
    uint64_t seed;        /* interior ~ U[0,1): value at global linear index
                             g = (k*ny + j)*nx + i is the (g+1)-th SplitMix64
                             output of `seed`, top 53 (f64) / 24 (f32) bits      */
    od_exec exec;
    int32_t tile[3];      /* tile shape (x, y, z) of the fused sweep; {0,0,0} =
                             the built-in or autotuned default for the block shape */
    /* Load imbalance (the dynamic imbalance that motivates overdecomposition,
     * Section I; the configuration with 10 % of chares doing 1 to 4 extra
     * sweeps).  At every step t, round(imbalance_pct / 100 * chares) chares
     * re-run their sweep 1..imbalance_max_extra extra times: the chares
     * taken first in a pseudo-random order of chare ids drawn from
     * (seed, t), each re-run count drawn from SplitMix64 at (seed, t,
     * chare); od_extra_sweeps reports the draw.  A re-run recomputes the
     * same values, so results do not change, only the time.  Where steps
     * run in pairs, a chare re-runs extra(t) + extra(t + 1) one-step sweeps
     * before the pass of steps t and t + 1.  0 = off. */
    int32_t imbalance_pct;
    int32_t imbalance_max_extra;
    /* Implementation hints, 0 = defaults; none of them changes a result.
     * bit 0: write the sweep's output with non-temporal (streaming) stores;
     * bit 1: launch tiles in plain spatial order instead of grouping
     * spatial neighbours on one XCD;
     * bit 2 (OD_MSGDRIVEN): schedule check: seeded delays before each task
     * publishes its finish and before each claim, and seeded start
     * positions of the per-XCD cursors, perturb the order in which tiles
     * run, and every task checks that each tile it reads halos from is
     * within one step of it (a failure raises the error flag: reads then
     * return OD_ESCHED).  Every message-driven task also checks, in any
     * mode, that its tile's step counter advances by exactly one;
     * bit 3 (OD_PERSISTENT): record the timeline read by od_timeline;
     * bit 4 (OD_PERSISTENT): take tiles from per-XCD-group counters, each
     * workgroup its next tile when the current one ends (the default for
     * two-step passes, under imbalance and with uneven blocks); uniform
     * one-step work defaults to a fixed stride per workgroup;
     * bit 5 (OD_PERSISTENT): counters, with each XCD group's last tiles
     * cut into z-ranges so the end of an iteration waits less (with two
     * steps per pass only the group's partial last round of tiles);
     * bits 6 / 7 (OD_MSGDRIVEN): claim ready tiles from each XCD's cursor /
     * from ready queues (default: cursor with >= 4 tiles per workgroup);
     * bits 9 / 10 (OD_MSGDRIVEN): one publisher workgroup per XCD / none
     * (default: a publisher on XCDs with >= 8 workgroups and >= 2 tasks
     * per workgroup and step);
     * bit 11 (OD_PERSISTENT): fixed schedule with contiguous runs of each
     * XCD group's tiles per workgroup;
     * bit 13 (OD_PERSISTENT): the fixed stride per workgroup, also where
     * counters are the default;
     * bit 12 (OD_FUSED, OD_GRAPH, OD_PERSISTENT, OD_MSGDRIVEN): one step
     * per pass.  By default these forms run iterations in pairs where they
     * can (blocks at one resolution, a tile shape with a two-step variant,
     * under load imbalance the 3D stencil: a heavy chare's re-runs are
     * one-step sweeps before its pass; OD_PERSISTENT with the 3D stencil, the
     * fixed-stride or counter schedule, with or without the guided tail,
     * and no timeline; OD_MSGDRIVEN with the 3D stencil, each task then a
     * pass of its tile, waiting for the tiles within two cells): one pass
     * reads the field once and writes it two steps later, the first step
     * kept on chip (the same values as two single sweeps, bit for bit);
     * od_iterate(n) with odd n ends with a single sweep.  With explicit
     * blocks the tiles are also cut so that every line of cells a pair
     * reads lies in one block.
     * od_plan_info.steps_per_pass tells which is in use.
     * Bit 8 is reserved.  Other bits are ignored. */
    int32_t hints;
    /* 7 (or 0): 3D 7-point stencil.  5: the 2D 5-point stencil of the
     * paper's Jacobi2D workload, u' = (((u[i-1] + u[i+1]) + u[k-1]) + u[k+1]) / 4,
     * on a grid with n[1] == 1: the 2D plane is (x, z), its second direction
     * stored as z; bc[2] and bc[3] (the y faces) are not read. */
    int32_t stencil;
    /* Multi-resolution blocks (explicit blocks only; NULL = every block has
     * unit cells, the uniform grid).  block_cell[b] is the cell edge of
     * block b in grid units, a power of two in [1, 1024]; the block's
     * origin and extent must be multiples of it and it holds extent/cell
     * cells per dimension.  Interior cell (i,j,k) of block b starts at unit
     * q = origin + (i,j,k)*cell and is initialised from SplitMix64 at unit
     * index (q_z*ny + q_y)*nx + q_x.  Every iteration first fills the ghost
     * cells of faces where the resolution changes: from a coarser
     * neighbour, the value of the neighbour cell containing the ghost
     * cell (injection); from a finer one (ratio r), the mean of the r x r
     * neighbour cells of the layer touching the face, summed with the
     * second tangential axis outer and the first inner (tangential axes in
     * x, y, z order) and divided by r*r.  Across such a face the finer
     * block's tangential origin and extent must be multiples of the coarser
     * cell, else OD_EINVAL.  Supported with OD_FUSED and OD_GRAPH (the
     * fill and the sweep as two launches per iteration) and OD_PERSISTENT
     * (both in one cooperative launch per od_iterate call, a device-wide
     * barrier after each; tiles from per-XCD counters, so hints bits 3, 5,
     * 11 and 13 and imbalance are refused); the global od_read / od_write /
     * od_read_points calls are refused, use od_read_block / od_write_block. */
    const int32_t* block_cell;
    /* Bound, in seconds, on every device-side wait of the persistent and
     * message-driven launches (barriers, ready queues); 0 = 10 s.  A wait
     * that reaches it raises the grid's error flag and every workgroup
     * leaves (reads then return OD_ETIMEDOUT).  Tests use a tiny bound to
     * exercise that path. */
    double wait_s;
} od_config;

struct od_grid;
struct od_server;

/* Defaults: n = 64^3, odf = 8, f64, bc = {1,0,0,0,0,0}, seed 12734,
 * OD_GRAPH, everything else 0. */
void od_config_default(od_config* cfg);

/* Bytes of caller-owned device workspace od_create needs for cfg. */
od_status od_workspace_bytes(const od_config* cfg, size_t* bytes);

/* Decompose, build halo maps, carve the workspace, upload descriptors and
 * initialise the field on the device (interior from seed, shell from bc).
 * The decomposition is the paper's overdecomposition: the grid's work and
 * data are split into many more chares than GPUs, each with its own
 * storage (Section II, Charm++ and Overdecomposition; Section III,
 * Managing Overdecomposition); every chare face's halo source is resolved
 * here, once, as with the pre-filled location table that lets a sender
 * pick the transport (Section IV, Portable Communication Layer).
 * Synchronises the stream before returning.  `dev_workspace` must be at
 * least od_workspace_bytes() bytes and 256-byte aligned. */
od_status od_create(const od_config* cfg, void* hip_stream, void* dev_workspace,
                    size_t workspace_bytes, struct od_grid** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * grid as od_create, but only the field storage is caller memory.
 * dev_fields (256-byte aligned) holds at least od_plan_info.field_bytes
 * bytes, the leading part of od_create's workspace; the descriptors and
 * device state (residual slots, barrier and step counters, queues) live in
 * a static device array of the library, 16 MiB per GPU, which every GPU the
 * library runs on holds until the process ends.  This call allocates no
 * device memory (no hipMalloc, no library allocator); it synchronises the
 * stream before returning.
 *   - exec must be OD_FUSED, OD_PERSISTENT or OD_MSGDRIVEN (OD_EINVAL
 *     otherwise: the graph and per-chare forms create graphs and streams
 *     when they first iterate).
 *   - Descriptor room is reserved for the planned tiles only: od_autotune
 *     then tries only tile shapes with no more tiles than planned.
 *   - OD_ENOMEM if the grid's control state exceeds 16 MiB (e.g. 512^3 at
 *     4096 chares needs about 1 MB fused, 3.3 MB persistent) or
 *     dev_fields is too small.
 *   - Every call shares its GPU's array, which keeps the last call's
 *     contents: the call rewrites every descriptor and clears the state it
 *     needs zeroed.  A grid made earlier on the same GPU by this call is
 *     superseded: its od_iterate, od_residual and reads return OD_EINVAL.
 *     Grids of this kind used concurrently on one GPU (other threads) race.
 * The handle is used and destroyed like od_create's; the field buffer stays
 * the caller's. */
od_status od_create_static(const od_config* cfg, void* hip_stream, void* dev_fields, size_t field_bytes,
                           struct od_grid** out);

/* Enqueue n >= 0 Jacobi iterations on the grid's stream (asynchronous, like
 * a kernel launch).  One iteration is the stencil application's step:
 * every chare exchanges halos with its neighbours and sweeps its block
 * (Section V, Jacobi2D, here with the 3D 7-point stencil), in the form
 * cfg.exec names (Section III for the per-chare form and the fused and
 * graph-captured mitigations cited in Section I).  Where the grid runs
 * iterations in pairs (od_plan_info.steps_per_pass == 2, hints bit 12) a
 * pass does two of them, with identical results.  Allocates nothing and
 * does not synchronise, except in OD_PER_CHARE mode whose host loop itself
 * issues the work. */
od_status od_iterate(struct od_grid* g, int64_t n);

/* Synchronise the stream; *r = residual of the last sweep (0 before any):
 * max over interior points of |u_new - u_old|.  The paper runs its
 * stencil for a fixed count without convergence checks (Section V,
 * Jacobi2D); the residual is this library's addition (a max norm, so its
 * value does not depend on the decomposition or the order of reduction).
 * od_residual and the reads below (od_read, od_read_points, od_read_block)
 * return OD_ETIMEDOUT instead of a result if a device-side wait of an
 * earlier persistent or message-driven launch gave up; the grid's state is
 * then undefined until od_write. */
od_status od_residual(struct od_grid* g, double* r);

/* Iterations done since od_create (or the last od_write). */
od_status od_iterations(struct od_grid* g, int64_t* iters);

/* Copy the whole padded global field (layout above) to host memory; syncs. */
od_status od_read(struct od_grid* g, void* host_dst, size_t bytes);

/* Set interior and Dirichlet shell from a padded global host array; resets
 * the iteration count and residual; syncs. */
od_status od_write(struct od_grid* g, const void* host_src, size_t bytes);

/* Read `count` interior values at global linear interior indices
 * idx[i] = (k*ny + j)*nx + i into host_dst (grid type); syncs. */
od_status od_read_points(struct od_grid* g, const int64_t* idx, int64_t count, void* host_dst);

/* Block-level I/O for any grid (regular, uneven or multi-resolution):
 * chare `b`'s interior cells, x fastest, shape (cells[2], cells[1],
 * cells[0]) as reported by od_block_cells; od_write_block sets them in the
 * current iterate (the iteration count and residual are kept).  Both sync. */
od_status od_block_cells(struct od_grid* g, int32_t b, int32_t cells[3]);
od_status od_read_block(struct od_grid* g, int32_t b, void* host_dst, size_t bytes);
od_status od_write_block(struct od_grid* g, int32_t b, const void* host_src, size_t bytes);

/* Host-only plan: decomposition, tiles and halo maps for cfg, with no
 * device work and no workspace.  The handle supports od_plan,
 * od_tile_info_get, od_chare_get and od_destroy; the other calls return
 * OD_EINVAL on it. */
od_status od_plan_create(const od_config* cfg, struct od_grid** out);

/* Introspection of the decomposition (host data, no device access):
 * chares, tiles, and algorithmic bytes moved per iteration
 * (s * (2*interior + ghost cells read from other chares)). */
typedef struct {
    int32_t nchares, ntiles, npseudo;
    int64_t interior, halo_cells;   /* halo_cells: ghost cells filled from other chares */
    int64_t bytes_per_iter;         /* algorithmic HBM bytes of one sweep            */
    int32_t tile[3];                /* tile shape in use                              */
    int32_t grid_wgs;               /* workgroups of the persistent / msg-driven launch */
    int32_t schedule;               /* OD_PERSISTENT: 1 fixed stride, 2 per-XCD counters,
                                       3 counters with a guided tail, 4 fixed
                                       contiguous runs; OD_MSGDRIVEN:
                                       bits 0-1 claims (0 automatic, 1 cursor, 2 ready
                                       queues), bits 2-3 publisher (0 automatic, 1 on,
                                       2 off); else 0                                  */
    int32_t coop_waves;             /* waves-per-SIMD cap of the cooperative grid
                                       (0 = default)                                   */
    int64_t field_bytes;            /* leading part of the workspace holding the field
                                       storage (the buffer od_create_static takes)    */
    int64_t control_bytes;          /* rest of the workspace: descriptors and device
                                       state, for this handle's plan                 */
    int32_t steps_per_pass;         /* 2: iterations run in pairs (OD_FUSED, OD_GRAPH,
                                       OD_PERSISTENT, OD_MSGDRIVEN; hints bit 12);
                                       else 1                                          */
    int64_t bytes_per_pass;         /* algorithmic HBM bytes of one pass: one sweep, or
                                       with two steps per pass s * (2*interior + cells
                                       of other chares within two steps' reach)       */
} od_plan_info;
od_status od_plan(struct od_grid* g, od_plan_info* info);

/* Per-tile descriptor export for host-side checks (brute-force halo maps):
 * for tile t: its chare, origin in the chare, extent, and for each face
 * (x-,x+,y-,y+,z-,z+) the source it reads its ghost slab from:
 * src_kind 0 = a chare (src = chare id), 1 = a Dirichlet face of the domain
 * (src = face 0..5), 2 = the ghost buffer of a resolution-change face of
 * the tile's own chare (src = face 0..5); src_origin = the coordinates of
 * the ghost slab's first cell in cells of the chare's size (global interior
 * coordinates for unit cells). */
typedef struct {
    int32_t chare, origin[3], extent[3];
    int32_t src_kind[6], src[6], src_origin[6][3];
} od_tile_info;
od_status od_tile_info_get(struct od_grid* g, int32_t t, od_tile_info* out);

/* Dependency list of tile t of an OD_MSGDRIVEN grid or plan (host data):
 * the tiles whose cells tile t's task reads, which are also the tiles that
 * read tile t's cells (the relation is symmetric): every other tile within
 * one cell (tasks of one step) or two cells in L1 distance (two-step tasks,
 * od_plan_info.steps_per_pass == 2) of the tile's box.  Up to cap indices
 * are written to out (ascending); *count = the list's length.  OD_EINVAL for
 * other exec modes or t out of range. */
od_status od_tile_deps(struct od_grid* g, int32_t t, int32_t* out, int32_t cap, int32_t* count);

/* Timeline of the last od_iterate of an OD_PERSISTENT grid created with
 * hints bit 3, for its first min(n, 1024, max_iters) iterations: out[4*i + k]
 * = microseconds (device wall clock) from the first workgroup's start of
 * iteration 0 to, for iteration i: k = 0 the first and k = 1 the last
 * workgroup starting it (leaving the previous barrier), k = 2 the first and
 * k = 3 the last workgroup finishing its tiles (arriving at the barrier).
 * *n_iters = iterations reported.  Syncs; OD_EINVAL for other grids. */
od_status od_timeline(struct od_grid* g, double* out, int32_t max_iters, int32_t* n_iters);

/* The load-imbalance draw of step `step` (0-based count of iterations since
 * od_create): out[c] = extra re-runs of chare c's sweep, for the n ==
 * nchares chares (all 0 without imbalance).  Host-only: it evaluates the
 * same definition the kernels evaluate on the device. */
od_status od_extra_sweeps(struct od_grid* g, int64_t step, int32_t* out, int32_t n);

/* Chare geometry: origin and extent of chare c in grid units (for
 * multi-resolution blocks: the block as given; cells = extent / cell). */
od_status od_chare_get(struct od_grid* g, int32_t c, od_block* out);

/* Wait for all work on the grid's stream, release host-side resources.
 * The workspace is not touched afterwards and stays the caller's. */
od_status od_destroy(struct od_grid* g);

/* Measured HBM copy ceiling: copy `bytes` between two caller-owned device
 * buffers `iters` times on `hip_stream` with each of the library's
 * streaming-copy kernel variants; *seconds = elapsed time (hipEvents) of the
 * fastest variant's `iters` copies. */
od_status od_stream_copy(void* hip_stream, void* dst, const void* src, size_t bytes,
                         int32_t iters, double* seconds);

/* Measured HBM ceilings by access kind: kind 0 = copy (as od_stream_copy,
 * 2 * bytes moved per pass), 1 = read-only (src is read, nothing is
 * stored; dst must be device memory of at least 16 bytes, its first word
 * may be modified), 2 = write-only (dst is overwritten with a pattern; src
 * is not read but must be non-NULL).  Each of the streaming kernel
 * variants runs `iters` passes over `bytes` (a positive multiple of 16);
 * *seconds = the fastest variant's elapsed time (hipEvents), *variant its
 * index (may be NULL).  Buffers are caller-owned device memory. */
od_status od_stream_bench(void* hip_stream, void* dst, const void* src, size_t bytes, int32_t iters,
                          int32_t kind, double* seconds, int32_t* variant);

/* Time n iterations with hipEvents on the grid's stream: *seconds = elapsed
 * device time between events recorded before and after od_iterate(n). */
od_status od_time_iterate(struct od_grid* g, int64_t n, double* seconds);

/* -------------------------------------------------------------------------
 * Launch-cost microbenchmark (Section III-A, Managing Overdecomposition:
 * the kernel-overlap experiment with streams gated on one flag).  It runs
 * on the current HIP device and creates and destroys its own non-blocking
 * streams (default priority).
 */
typedef struct {
    int64_t total_threads;
    int32_t nkernels;
    int32_t nstreams;     /* streams actually used: min(nstreams, nkernels) */
    int32_t work;
    int32_t pad;
    double makespan_us;   /* device: earliest workgroup start -> latest workgroup end */
    double host_us;       /* host: release enqueued -> every stream's event complete  */
    double enqueue_us;    /* host: time to enqueue the gates, kernels and events      */
} od_overlap_result;

/* Workspace for od_launch_overlap: 256 bytes of timestamps followed by
 * total_threads uint32 outputs.  0 if total_threads <= 0. */
size_t od_launch_overlap_bytes(int64_t total_threads);

/* Split total_threads threads (each `work` dependent 32-bit multiply-adds
 * x <- x*1664525 + 1013904223 from x = thread_index ^ 0x9E3779B9, stored to
 * outputs[thread_index]) into nkernels near-equal kernels of 256-thread
 * workgroups, round-robin over nstreams streams.  Each stream first runs a
 * one-wave gate kernel polling a flag in pinned host memory (allocated once
 * per device and kept until the process ends); after every kernel is
 * enqueued the host raises the flag and all streams start together.  A gate
 * gives up after 10 s (OD_ETIMEDOUT).  Blocks until every kernel has
 * completed (bounded: OD_ETIMEDOUT after 60 s).
 * dev_ws: caller-owned device memory, 256-byte aligned, at least
 * od_launch_overlap_bytes(total_threads).  Limits: total_threads in
 * [1, 2^31], nkernels in [1, min(65536, total_threads)], nstreams in
 * [1, 256], work in [0, 2^24]; otherwise OD_EINVAL. */
od_status od_launch_overlap(void* dev_ws, size_t ws_bytes, int64_t total_threads, int32_t nkernels,
                            int32_t nstreams, int32_t work, od_overlap_result* out);


/* -------------------------------------------------------------------------
 * Autotuning: tile shape and schedule.  Every candidate computes the same
 * arithmetic; only the tile shape, the schedule and the launch shape
 * differ.  OD_FUSED and OD_GRAPH grids time `iters` fused passes per tile
 * candidate, per step (a shape with a two-step variant is timed as pairs
 * of steps, as the grid would run it; each pass writes only the spare
 * parity, so the field is unchanged).  OD_PERSISTENT grids time a launch of 2 * iters iterations
 * for every tile candidate under each schedule (fixed stride, fixed runs,
 * per-XCD counters, counters with a guided tail) and waves-per-SIMD cap (the
 * kernel's register limit or one less).  OD_MSGDRIVEN grids keep their tile
 * and time their scheduler choices (cursor or ready-queue claims,
 * publisher or none, waves cap) over 2 * iters steps each.  For these two,
 * the field, the device state and the iteration count are saved to pinned
 * host memory first and restored afterwards.  The fastest choice is applied and cached per (dtype, mode,
 * grid and chare shapes, hints, imbalance).  OD_PER_CHARE: OD_EINVAL.
 * `out_tile` receives the chosen shape; od_plan reports the schedule. */
od_status od_autotune(struct od_grid* g, int32_t iters, int32_t out_tile[3]);

/* -------------------------------------------------------------------------
 * Serving: independent Jacobi solves of different sizes admitted as they
 * arrive under a device-memory budget and run concurrently by the
 * message-driven device scheduler (continuous batching).  Each solve's
 * result equals that of the same solve run alone.
 *
 * Not from the paper: the paper schedules chares of one application from
 * a message queue (Section II, asynchronous method invocation), and this
 * layer carries that execution model over to many independent solves
 * sharing one GPU.  Every call below is this library's own interface.
 */
typedef struct {
    int64_t n;            /* cubic interior extent                       */
    od_dtype dtype;
    int32_t odf;          /* chares for this solve (1, 8, 64, ...)       */
    double tol;           /* stop when residual < tol at a check step    */
    int64_t max_iters;    /* hard cap                                    */
    int32_t check_every;  /* residual checked at multiples of this       */
    uint64_t seed;
    double bc[6];
    double t_arrival;     /* when the request arrived, CLOCK_MONOTONIC
                             seconds (the clock of od_info's stamps); 0 =
                             the od_submit time.  Must not lie in the
                             future (OD_EINVAL).  Latency = t_done -
                             t_arrival, so time a caller spent before
                             submitting counts.                          */
} od_request;

enum { OD_REQ_QUEUED = 0, OD_REQ_RUNNING = 1, OD_REQ_DONE = 2, OD_REQ_CANCELED = 3 };

typedef struct {
    int32_t state;
    int64_t iters;       /* iterations done when it stopped             */
    double residual;     /* residual of its last sweep                  */
    double t_submit, t_admit, t_done;   /* host monotonic seconds       */
    double t_arrival;    /* the request's t_arrival (t_submit if it was 0) */
} od_info;

/* `dev_arena` of `arena_bytes` (caller-owned, 256-byte aligned) is the
 * memory budget: a fixed control region for `max_slots` slots, the rest
 * holds the resident solves.  At most `max_slots` solves are resident at
 * once.  Starts the worker thread that owns `hip_stream`; timestamps are
 * CLOCK_MONOTONIC seconds. */
od_status od_server_create(void* hip_stream, void* dev_arena, size_t arena_bytes,
                           int32_t max_slots, struct od_server** out);
/* Kernel hints of the server's later scheduling epochs: 0 or 4 (bit 2, the
 * schedule check of od_config.hints: seeded delays and cursor start
 * positions from `seed` perturb the device schedule, and every task checks
 * its neighbours' step counters; a failure cancels the running requests
 * with OD_ECANCELED and a message naming the check).  OD_EINVAL for other
 * bits.  Results never depend on it. */
od_status od_server_set_hints(struct od_server* s, int32_t hints, uint64_t seed);
/* Bytes of the fixed control region od_server_create carves from the
 * start of the arena for `max_slots` slots. */
od_status od_server_control_bytes(int32_t max_slots, size_t* bytes);
/* Bytes a request needs in the arena (besides the control region). */
od_status od_request_bytes(const od_request* req, size_t* bytes);
/* Queue a request; never blocks.  OD_ENOMEM if it can never fit the arena,
 * OD_EAGAIN if the submission queue is full, OD_EINVAL for bad fields. */
od_status od_submit(struct od_server* s, const od_request* req, uint64_t* ticket);
/* The server's worker thread drives the device (admission, scheduling
 * epochs); a second thread retires finished solves (copies each field to
 * host memory, frees its slot and arena space).  This reports how many
 * requests are resident
 * (`active`) and waiting (`queued`); OD_ECANCELED once the server has
 * stopped after a device error. */
od_status od_server_step(struct od_server* s, int32_t* active, int32_t* queued);

/* Where the server's threads spent their time so far (host clock): the
 * worker inside scheduling epochs (launch to completion), admitting
 * requests (planning, descriptor upload, field initialisation) and waiting
 * for work; the retire thread copying finished fields to host memory
 * (retire_s, which overlaps the epochs). */
typedef struct {
    int64_t epochs;
    double epoch_s, admit_s, retire_s, idle_s;
} od_server_stats;
od_status od_server_stats_get(struct od_server* s, od_server_stats* out);
/* State of a request; OD_ENOTREADY while queued or running. */
od_status od_poll(struct od_server* s, uint64_t ticket, od_info* out);
/* Copy a finished request's padded global field (global layout above) to
 * host_dst and forget the request.  OD_ENOTREADY while it runs. */
od_status od_fetch(struct od_server* s, uint64_t ticket, void* host_dst, size_t bytes);
od_status od_server_destroy(struct od_server* s);

/* Thread-local message of the last failing call on this thread. */
const char* od_last_error(void);

/* Library version string. */
const char* od_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OD_H */
