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
// zeroes res[2*s + parity] for s in [zero_lo, zero_hi).  `extra` (may be
// null): per-chare count of extra re-runs of the sweep for this step.
hipError_t launch_sweep(int dtype_bytes, int tx, int ty, hipStream_t st, void* arena,
                        const BlockDev* blocks, const TileDev* tiles, int32_t ntiles, int parity,
                        unsigned long long* res, int32_t zero_lo, int32_t zero_hi,
                        const uint8_t* extra, int hints);

// Persistent cooperative sweep: all `iters` iterations in one launch with a
// device-wide barrier between them.  `bar` = 2 zeroed uint32 (count,
// generation); `err` = error flag.  `extra` (may be null): table of
// [period][nchares] extra re-runs, row (iter_base + it) % period.
hipError_t launch_persistent(int dtype_bytes, int tx, int ty, hipStream_t st, int grid,
                             void* arena, const BlockDev* blocks, const TileDev* tiles,
                             int32_t ntiles, int parity, int64_t iters,
                             unsigned long long* res, int32_t nres, unsigned int* bar,
                             unsigned int* err, const uint8_t* extra, int32_t extra_period,
                             int32_t nchares, int64_t iter_base, int hints);
// Wall-clock ticks in `seconds` (bound of every device-side wait).
int64_t device_wait_ticks(double seconds = 10.0);
// Max co-resident workgroups of the persistent / message-driven kernels.
int persistent_max_grid(int dtype_bytes, int tx, int ty, int kind);

// Message-driven cooperative sweep (see sched kernels): per-tile step
// counters `done`, dependency lists (CSR: dep_ptr[ntiles+1], dep_idx).
struct MsgArgs {
    const int32_t* tile_list;   // launch's tiles (global ids); null => 0..ntiles-1
    const int32_t* solve_dtype; // serving: bytes per element of each solve
    void* arena;
    const BlockDev* blocks;
    const TileDev* tiles;
    int32_t ntiles;             // tiles in this launch
    const int32_t* dep_ptr;
    const int32_t* dep_idx;
    int32_t* done;              // steps completed per tile (monotone), by global id
    const int32_t* target;      // per-solve target step (for a plain grid: 1 entry)
    const int32_t* tile_solve;  // solve of each tile (null => solve 0)
    unsigned long long* res;    // plain grid: 2 slots (step parity); serving: 1 slot per solve
    unsigned int* err;
    const uint8_t* extra;       // [period][nchares] or null
    int32_t extra_period;
    int32_t nchares;
    int64_t wait_ticks;         // bound on a workgroup's idle wait (wall-clock ticks)
    int32_t final_only;         // plain grid: record the residual only at the target step
    int32_t hints;              // od_config.hints
    // serving only (null for a plain grid)
    int32_t* solve_count;       // per solve: tiles that finished the current decision step
    int32_t* gate;              // per solve: highest step whose check passed
    const int32_t* solve_ntiles;
    const int32_t* check_every;
    const double* tol;
    int32_t* final_step;        // per solve: step at which it stopped (0 = running)
    volatile int32_t* host_done;     // pinned host: per solve final step when done
    volatile unsigned long long* host_res;
    volatile int32_t* yield_flag;   // pinned host: nonzero => stop after current tasks
};
hipError_t launch_msgdriven(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, const MsgArgs& a);

// Serving kernel: fp64 tiles of (kServeTx8, kServeTy8) and fp32 tiles of
// (kServeTx4, kServeTy4) columns, same thread count, one cooperative launch.
constexpr int kServeTx8 = 32, kServeTy8 = 8, kServeTx4 = 32, kServeTy4 = 16;
int serve_max_grid();
hipError_t launch_serve(hipStream_t st, int grid, const MsgArgs& a);

// Initialise parity 0 of every chare from seed, Dirichlet pseudo-blocks from bc.
hipError_t launch_init(int dtype_bytes, hipStream_t st, const GridDev& g, int32_t nchares,
                       uint64_t seed, int32_t npb, const int32_t* pb_face, const int32_t* pb_block,
                       const double* bc_dev);

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

}  // namespace od
