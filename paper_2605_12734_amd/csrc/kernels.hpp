// Launchers of the HIP kernels of libod (host-callable, C++ linkage).
#pragma once

#include <hip/hip_runtime.h>

#include "od_internal.hpp"

namespace od {

// Device-side owner lookup: which chare holds a global interior cell.
struct LookupDev {
    int32_t regular;
    int32_t k[3];               // regular: chares per dimension
    const int32_t* cidx[3];     // regular: chare coordinate of each global x / y / z
    const int32_t* owner;       // explicit: owner grid (og z, og y, og x)
    int32_t gran;
    int32_t og[3];
    const int32_t* corigin;     // chare origins, 3 per chare
    const int32_t* dir_pb;      // Dirichlet pseudo-block of (chare, face), 6 per chare, -1 if none
};

struct GridDev {
    void* arena;                // element base of every BlockDev offset
    const BlockDev* blocks;
    LookupDev lk;
    int64_t n[3];
};

// Seeded load imbalance (one definition for the host and the device).  At
// step t the chares are put in the order of a pseudo-random permutation of
// their ids drawn from (seed, t); the first `heavy` of them re-run their
// sweep 1..maxe extra times, the count drawn from SplitMix64 at
// (seed, t, chare).  The permutation is a four-round Feistel network on
// the smallest even number of bits covering the chare count, with cycle
// walking back into [0, nchares), so exactly `heavy` chares are drawn at
// every step and the draw is fresh at every step (no table, no period).
struct ImbDev {
    uint64_t seed;
    int32_t nchares;
    int32_t heavy;     // chares drawn per step (0 = no imbalance)
    int32_t maxe;      // largest number of extra re-runs
    int32_t pad_;
};

__host__ __device__ inline uint64_t imb_mix(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Position of chare c in step t's order (a permutation of [0, nchares)).
__host__ __device__ inline uint32_t imb_rank(const ImbDev& m, int64_t t, uint32_t c) {
    int half = 1;
    while ((1ull << (2 * half)) < (uint64_t)m.nchares) ++half;
    const uint32_t mask = (1u << half) - 1u;
    const uint64_t key = imb_mix(m.seed ^ 0x696D62616C616E63ull, (uint64_t)t);
    uint32_t y = c;
    do {
        uint32_t l = y >> half, r = y & mask;
        for (uint32_t round = 0; round < 4; ++round) {
            const uint32_t f = (uint32_t)imb_mix(key, ((uint64_t)round << 32) | r) & mask;
            const uint32_t nl = r;
            r = l ^ f;
            l = nl;
        }
        y = (l << half) | r;
    } while (y >= (uint32_t)m.nchares);
    return y;
}

// Extra re-runs of chare c's sweep at step t (0 for most chares).
__host__ __device__ inline int32_t imb_extra(const ImbDev& m, int64_t t, int32_t c) {
    if (m.heavy <= 0 || m.maxe <= 0) return 0;
    if (imb_rank(m, t, (uint32_t)c) >= (uint32_t)m.heavy) return 0;
    const uint64_t h = imb_mix(m.seed ^ 0x6578747261ull, (uint64_t)t * (uint64_t)m.nchares + (uint64_t)c);
    return 1 + (int32_t)((h >> 32) % (uint64_t)m.maxe);
}

// hints bit 2: message-driven schedule check.  Seeded delays before each
// task publishes its finish and before each claim, and seeded start
// offsets of the per-XCD cursors, perturb the order in which tiles run;
// every task checks that each tile it reads halos from is within one step
// of it.  In every message-driven launch a task also checks that its
// tile's step counter advances by exactly one.  A failed check raises
// kErrSchedule in the error flag (the launch then ends; no trap).
constexpr int kHintCheck = 4;
constexpr unsigned int kErrSchedule = 4u;

// Sweep-kernel variant: tile shape (x, y) compiled in; z extent is per tile.
struct SweepVariant {
    int tx, ty;
    int threads;
};
// Variants compiled for a dtype (bytes 4 or 8).
const SweepVariant* sweep_variants(int dtype_bytes, int* count);
bool sweep_variant_ok(int dtype_bytes, int tx, int ty);
int sweep_threads(int dtype_bytes, int tx, int ty);

// Fused sweep over tiles[0..ntiles): one workgroup per tile, reading parity
// `parity`, writing parity^1.  Residual of tile t goes (atomic max of the
// value's bit pattern) into res[2*rslot + (parity^1)]; workgroup 0 first
// zeroes res[2*s + parity] for s in [zero_lo, zero_hi).  `imb`, `step`:
// the load-imbalance draw of this step (imb.heavy == 0: none).
// xexp (may be null): multi-resolution x-column exports (XExpDev, per chare).
struct XExpDev;
struct FillSeg;
hipError_t launch_sweep(int dtype_bytes, int tx, int ty, hipStream_t st, void* arena,
                        const BlockDev* blocks, const TileDev* tiles, int32_t ntiles, int parity,
                        unsigned long long* res, int32_t zero_lo, int32_t zero_hi,
                        const ImbDev& imb, int64_t step, int hints, const XExpDev* xexp = nullptr);

// Two Jacobi steps per pass (regular grids at one resolution, 3D 7-point
// stencil): each tile reads the time-t field once, computes the first step
// on itself and on a one-cell ring around it in registers and LDS, and
// writes only the second step.  Besides the six face slabs (TileDev::f) it
// reads the slabs two cells out and the cells of twelve lines around the
// tile, each given like a FaceDev (block and local coordinates of its first
// cell; a ghost-shell cell maps to the Dirichlet pseudo-block of its face,
// any cell of which holds the face's value; a cell that is never read maps
// to the tile's own chare):
//   r2[f]     slab of face f two cells out (x-, x+, y-, y+, z-, z+)
//   e[0..3]   (x, y) = (-1,-1), (nx,-1), (-1,ny), (nx,ny), z = 0..nz-1 (along z)
//   e[4..7]   x = -1 / nx, z = -1: e[4] x-, e[5] x+; z = nz: e[6] x-, e[7] x+ (along y)
//   e[8..11]  y = -1 / ny, z = -1: e[8] y-, e[9] y+; z = nz: e[10] y-, e[11] y+ (along x)
// dir: bit f set when face f of the tile is a Dirichlet face of the domain
// (its first step is the boundary value itself).
struct Tile2Dev {
    FaceDev e[12];
    FaceDev r2[6];
    int32_t dir, pad_[3];
};
static_assert(sizeof(Tile2Dev) == 304, "Tile2Dev layout");
// Two-step variants compiled for a dtype: 3D tiles (x extent >= 2 vectors,
// y >= 2), or with `flat` the 2D 5-point stencil's row tiles (ty == 1).
bool sweep2_variant_ok(int dtype_bytes, int tx, int ty, bool flat = false);
// Reads parity `parity`, writes the field two steps later into parity^1;
// the residual (of the second step) and res zeroing as launch_sweep.
// hints bit 8 (the 2D stencil) selects the row kernel (no imbalance).
// imb.heavy > 0: chares drawn heavy at step `step` or step + 1 first re-run
// their sweep the drawn number of extra times (the result is unchanged).
hipError_t launch_sweep2(int dtype_bytes, int tx, int ty, hipStream_t st, void* arena, const BlockDev* blocks,
                         const TileDev* tiles, const Tile2Dev* tiles2, int32_t ntiles, int parity,
                         unsigned long long* res, int32_t zero_lo, int32_t zero_hi, int hints, const ImbDev& imb,
                         int64_t step);

// Persistent form of a multi-resolution grid: `iters` iterations in one
// cooperative launch, each the resolution-change ghost fill of the nseg
// rectangles (from parity p), the per-XCD barrier, the sweep of every tile
// (tiles from per-XCD-group counters; boundary x-columns exported through
// xexp) and the barrier again; bar / err as launch_persistent.
hipError_t launch_persistent_mr(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, void* arena,
                                const BlockDev* blocks, const TileDev* tiles, int32_t ntiles, int parity,
                                int64_t iters, unsigned long long* res, int32_t nres, unsigned int* bar,
                                unsigned int* err, int64_t wait_ticks, int hints, const FillSeg* segs, int32_t nseg,
                                const XExpDev* xexp);

// Persistent form of the two-step pass: `passes` passes (2 * passes steps)
// in one cooperative launch of `grid` workgroups, the per-XCD barrier
// between passes; dyn != 0: tiles from per-XCD-group counters, else the
// fixed stride; bar / err as launch_persistent; pass k covers steps
// iter_base + 2k and iter_base + 2k + 1 of the imbalance draw imb.
hipError_t launch_persistent2(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, void* arena,
                              const BlockDev* blocks, const TileDev* tiles, const Tile2Dev* tiles2, int32_t ntiles,
                              int parity, int64_t passes, unsigned long long* res, int32_t nres, unsigned int* bar,
                              unsigned int* err, int hints, int64_t wait_ticks, int dyn, const ImbDev& imb,
                              int64_t iter_base);

// Persistent cooperative sweep: all `iters` iterations in one launch with a
// device-wide barrier between them.  dyn != 0: workgroups take tiles from
// per-XCD-group counters (load balance under imbalance and uneven blocks);
// dyn == 0: workgroup w takes tiles w, w + grid, ... (uniform work).
// `bar` = kBarWords zeroed uint32: [0] arrivals, [1] generation, [2] exits,
// [32..40) per-XCD barrier arrivals, [40..48) workgroups per XCD, from
// word 64 the tile counters (8 XCD groups x 2 step parities, 32 words
// apart); the kernel leaves them zeroed.  Between iterations, one L2 write-back per XCD publishes its
// workgroups' results (the XCD's workgroups share that L2).  `err` = error
// flag.  `imb`: load-imbalance draw, iteration `it` of the launch is step
// iter_base + it.
// chunked (fixed-stride form): each workgroup takes a contiguous run of its
// XCD group's positions instead of every G/8-th one.
// `stamps` (may be null): timeline of the first kStampIters iterations, 4
// wall-clock words per iteration (first / last workgroup to start it,
// first / last to finish its tiles), prepared by launch_stamp_init.
constexpr int kStampIters = 1024;
constexpr int kBarWords = 1024;
hipError_t launch_persistent(int dtype_bytes, int tx, int ty, hipStream_t st, int grid,
                             void* arena, const BlockDev* blocks, const TileDev* tiles,
                             int32_t ntiles, int parity, int64_t iters,
                             unsigned long long* res, int32_t nres, unsigned int* bar,
                             unsigned int* err, const ImbDev& imb, int64_t iter_base, int hints, int dyn,
                             int64_t wait_ticks, unsigned long long* stamps = nullptr, int chunked = 0);
hipError_t launch_stamp_init(hipStream_t st, unsigned long long* stamps, int32_t n);
// hints bit 3 (persistent form): record the timeline above.
constexpr int kHintTimeline = 8;
// Register usage of a kernel of the compiled library (demangled name without the
// return type and parameters); false if the compile recorded none.
bool kernel_resources(const char* name, int* sgprs, int* vgprs, int* lds);
// Waves per SIMD that a kernel's scalar registers allow on gfx950: residency
// probes (256-thread workgroups holding their CU) held 8 waves at 78 SGPRs,
// 7 at 86 and 6 at 99-108, which a budget of 704 SGPRs per SIMD at a
// granularity of 16 reproduces (the occupancy query counts SGPRs more
// generously; VGPRs and LDS it counts exactly).
inline int waves_by_sgprs(int sgprs) {
    const int a = (sgprs + 15) / 16 * 16;
    const int w = a > 0 ? 704 / a : 8;
    return w > 8 ? 8 : (w < 1 ? 1 : w);
}
// Wall-clock ticks in `seconds` (bound of every device-side wait).
int64_t device_wait_ticks(double seconds = 10.0);
// Max co-resident workgroups of a cooperative kernel: kind 0 = persistent
// with the static tile stride, 2 = persistent with tile counters (dyn),
// 1 = message-driven, 3 / 4 = persistent two-step passes with the static
// stride / with counters, 5 = message-driven two-step tasks, 6 = persistent
// multi-resolution (ghost fill and sweep per iteration); at most
// max_waves waves per SIMD (0 = the default choice: 5 for kind 2, else as
// many as the registers allow).
int persistent_max_grid(int dtype_bytes, int tx, int ty, int kind, int max_waves = 0);
// Waves per SIMD the kernel's recorded scalar registers allow.
int coop_waves_limit(int dtype_bytes, int tx, int ty, int kind);

// Message-driven cooperative sweep: per-tile step counters `done`,
// dependency lists (CSR: dep_ptr[ntiles+1], dep_idx; symmetric), counters
// of finishes per tile and step parity, and per-XCD ready queues.
struct MsgArgs {
    const int32_t* tile_list;   // serving: launch position -> tile id (-1 = padding)
    const int32_t* solve_dtype; // serving: bytes per element of each solve
    void* arena;
    const BlockDev* blocks;
    const TileDev* tiles;
    const Tile2Dev* tiles2;     // plain grid with two-step tasks: each tile's extra lines
    int32_t ntiles;             // launch positions (plain grid: tiles)
    const int32_t* dep_ptr;
    const int32_t* dep_idx;
    int32_t* done;              // steps completed per tile (monotone), by tile id
    const int32_t* target;      // per-solve target step (for a plain grid: 1 entry)
    const int32_t* tile_solve;  // serving: solve of each tile
    unsigned long long* res;    // plain grid: 2 slots (step parity); serving: 1 slot per solve
    unsigned int* err;
    ImbDev imb;                 // load-imbalance draw (heavy == 0: none)
    // plain grids: scheduler step k draws the imbalance of step imb_base + k
    // (one-step tasks) or imb_base + 2k and + 2k + 1 (two-step tasks)
    int64_t imb_base;
    int64_t wait_ticks;         // bound on every device-side wait (wall-clock ticks)
    int32_t hints;              // od_config.hints (bit 2: schedule check, see kHintCheck)
    // plain grids: scheduler choice, bits 0-1 claim mode (0 = automatic,
    // 1 = cursor, 2 = ready queues), bits 2-3 publisher (0 = automatic,
    // 1 = one per XCD with at least two workgroups, 2 = none)
    int32_t sched;
    uint64_t seed;              // schedule check: seed of the perturbation
    int64_t pert_ticks;         // schedule check: largest delay (wall-clock ticks)
    // serving only
    int32_t* solve_count;       // per solve: tiles that finished the current decision step
    int32_t* gate;              // per solve: highest step whose check passed
    const int32_t* solve_ntiles;
    const int32_t* check_every;
    const double* tol;
    int32_t* final_step;        // per solve: step at which it stopped (0 = running)
    volatile int32_t* host_done;     // pinned host: per solve final step when done
    volatile unsigned long long* host_res;
    volatile int32_t* yield_flag;   // pinned host: nonzero => stop after current tasks
    int32_t* yield_dev;             // device copy of the yield flag (zeroed before the launch):
                                    // workgroup 0 polls the host flag at most every
                                    // yield_poll_ticks and raises this word, which every
                                    // workgroup reads (no host-memory poll per task)
    int64_t yield_poll_ticks;
    const int32_t* tile_pos;    // serving: tile id -> launch position
    const int32_t* solve_base;  // serving: launch position of each solve's first tile
    int32_t nlive;              // serving: running solves in the launch
    // per launch position: bit 0 = some tile that reads it is queued on
    // another XCD (its finish needs an L2 write-back); serving, bit 1 =
    // ready at launch start
    uint8_t* xpub;
    unsigned int* bar;          // 2 words for the launch-start barriers (count, generation)
    // pend = 2 counters per tile; qslots, pslots = 2 * ntiles + 8
    // ready-queue and cross-list slots; qhead = 64 control words (heads,
    // tails, present-XCD mask, workgroups per XCD, list tails, cross tiles
    // per XCD, running solves; 8 each except the mask and the count);
    // qsteps = steps a plain-grid launch runs
    int32_t* pend;
    int32_t* ready;             // cursor scheduler: per tile, next step - d0 + 1 (0 = not ready)
    unsigned long long* qslots;
    unsigned long long* pslots;
    unsigned int* qhead;
    int32_t qsteps;
};
hipError_t launch_msgdriven(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, const MsgArgs& a);
// The same scheduler with tasks of two steps (a.tiles2 set; a scheduler
// step is one two-step pass: the field's parity flips once per step).
hipError_t launch_msgdriven2(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, const MsgArgs& a);
// Clear the control words of a dependency-counting message-driven launch
// (the launch itself lays out and fills its queues); a plain grid also
// stores its target step in *target_word and zeroes res_clear[0..2) (both
// may be null), so no host buffer has to outlive the call.
hipError_t launch_queue_init(hipStream_t st, const MsgArgs& a, int32_t target = 0, int32_t* target_word = nullptr,
                             unsigned long long* res_clear = nullptr);
// Serving: for every launch position q of list[0..n) holding a tile id v
// (-1 = padding), tpos[v] = q, and sbase[v / stride] = q when v is a
// solve's first tile (v % stride == 0).  Entries of tiles not in the list
// are left as they are.
hipError_t launch_serve_positions(hipStream_t st, const int32_t* list, int32_t n, int32_t stride, int32_t* tpos,
                                  int32_t* sbase);

// Serving kernel: fp64 tiles of (kServeTx8, kServeTy8) and fp32 tiles of
// (kServeTx4, kServeTy4) columns, same thread count, one cooperative launch.
#ifndef OD_SERVE_TY8
#define OD_SERVE_TY8 16    // rows of an fp64 serving tile (fp32 tiles have twice as many)
#endif
constexpr int kServeTx8 = 32, kServeTy8 = OD_SERVE_TY8, kServeTx4 = 32, kServeTy4 = 2 * OD_SERVE_TY8;
int serve_max_grid();
hipError_t launch_serve(hipStream_t st, int grid, const MsgArgs& a);

// Multi-resolution ghost fill: one rectangle of a chare face's ghost buffer
// read from one neighbour chare of another cell size.  Ghost cell (c1, c2)
// of the rectangle (tangential axes t1 < t2 of the face's normal axis d)
// lies at neighbour-relative unit offsets (r1 + c1*hc, r2 + c2*hc); the
// neighbour cell edge is 2^lhn units.  A coarser or equal neighbour gives
// its cell containing that point, a finer one the mean of the
// (hc >> lhn)^2 cells of its layer `lay` covering the ghost cell's face.
struct FillSeg {
    int32_t dst;            // ghost pseudo-block (block table index)
    int32_t src;            // neighbour chare
    int32_t d;              // normal axis
    int32_t lay;            // neighbour cell index along d
    int32_t a1, a2;         // rectangle origin in the face's ghost cells
    int32_t n1, n2;         // rectangle extent
    int32_t r1, r2;         // neighbour-relative unit offset of ghost cell (a1, a2)
    int32_t hc, lhn;        // ghost cell edge (units), log2 neighbour cell edge
    int64_t first;          // index of the rectangle's first ghost cell over all rectangles
    // x-normal faces (d == 0): the neighbour's exported column of layer
    // `lay` for each parity (element offsets, see XExpDev) and its y extent;
    // the values are read from there, y fastest, instead of one per row of
    // the neighbour's storage
    int64_t eoff[2];
    int32_t ey, pad_;
};
static_assert(sizeof(FillSeg) == 80, "FillSeg layout");

// Multi-resolution grids: a chare's boundary x-column (x = 0 or ex - 1)
// that a neighbour of another cell size fills its ghosts from.  The fused
// sweep writes it, for the parity it produces, into a contiguous (y, z)
// array (y fastest) while the values are in registers, so the ghost fill
// reads whole sectors instead of one value per 64-byte row.  Element
// offsets from the arena base, -1 where no neighbour reads that column.
struct XExpDev {
    int64_t off[2][2];   // [side: 0 = x-, 1 = x+][parity]
};
// Copy the x-columns of parity `parity` into their exports (after the field
// is initialised or written from the host).
hipError_t launch_xexp_refresh(int dtype_bytes, hipStream_t st, void* arena, const BlockDev* blocks,
                               const XExpDev* xexp, int32_t nchares, int parity);

// Fill every resolution-change ghost buffer from parity `parity` of the
// chares: one single-wave workgroup per rectangle segs[0..nseg); `total` (ghost cells
// over all rectangles) only skips an empty launch.
hipError_t launch_amr_fill(int dtype_bytes, hipStream_t st, void* arena, const BlockDev* blocks,
                           const FillSeg* segs, int32_t nseg, int64_t total, int parity);

// Multi-resolution initialisation of parity 0: chare c's cell (i,j,k)
// starts at unit corigin_c + (i,j,k)*ccell[c] and takes the SplitMix64
// value of that unit's global index.
hipError_t launch_init_cells(int dtype_bytes, hipStream_t st, const GridDev& g, const int32_t* ccell,
                             int32_t nchares, uint64_t seed);

// Initialise parity 0 of every chare from seed, Dirichlet pseudo-blocks from bc.
// `interior` = false: only the Dirichlet pseudo-blocks (the chares are
// initialised by launch_init_cells).
hipError_t launch_init(int dtype_bytes, hipStream_t st, const GridDev& g, int32_t nchares,
                       uint64_t seed, int32_t npb, const int32_t* pb_face, const int32_t* pb_block,
                       const double* bc_dev, bool interior = true);

// Gather planes [kz_lo, kz_hi) of the padded global array into dst (device- or
// host-mapped), plane kz_lo at dst[0].  scatter: the inverse.
hipError_t launch_gather(int dtype_bytes, hipStream_t st, const GridDev& g, int parity,
                         int64_t kz_lo, int64_t kz_hi, void* dst);
hipError_t launch_scatter(int dtype_bytes, hipStream_t st, const GridDev& g, int parity,
                          int64_t kz_lo, int64_t kz_hi, const void* src);
hipError_t launch_points(int dtype_bytes, hipStream_t st, const GridDev& g, int parity,
                         const int64_t* idx, int64_t count, void* dst);

// Per-chare baseline: pack the six faces of one chare into messages / unpack
// six messages into its ghost pseudo-blocks.  msg[f] = device pointers (may
// be null for faces without a neighbour), elements of face f = cnt[f].
struct FaceSet {
    void* p[6];
    int64_t cnt[6];
};
hipError_t launch_pack_b(int dtype_bytes, hipStream_t st, void* arena, const BlockDev& B, int parity,
                         const FaceSet& out);
hipError_t launch_unpack(int dtype_bytes, hipStream_t st, FaceSet in, FaceSet ghost);

// Streaming copy of `bytes` (multiple of 16) from src to dst with copy
// kernel variant `variant` (0 .. copy_variant_count()-1).
int copy_variant_count();
hipError_t launch_copy(hipStream_t st, void* dst, const void* src, size_t bytes, int variant);
// The same variants as a read-only (kind 1: loads src, writes nothing; a
// 4-byte `sink` is written only for a data pattern that does not occur)
// or write-only (kind 2: stores a pattern to dst) stream; kind 0 = copy.
hipError_t launch_stream(hipStream_t st, void* dst, const void* src, size_t bytes, int variant, int kind,
                         uint32_t* sink);

}  // namespace od
