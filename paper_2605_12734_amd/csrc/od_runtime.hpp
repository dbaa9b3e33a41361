// libod runtime internals: the grid object behind od_grid*.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "od_internal.hpp"

namespace od {

extern thread_local std::string g_last_error;
od_status fail(od_status s, const std::string& msg);
uint64_t host_sm64(uint64_t seed, uint64_t idx);

// Byte offsets of the workspace regions.
struct Layout {
    size_t blocks = 0, tiles = 0, cidx[3] = {0, 0, 0}, owner = 0, corigin = 0, dir_pb = 0;
    size_t pb_face = 0, pb_block = 0, bc = 0, res = 0, bar = 0, err = 0, done = 0, target = 0;
    size_t dep_ptr = 0, dep_idx = 0, field_end = 0, total = 0;
    // [0, field_end): field storage (chares, face pseudo-blocks, messages),
    // addressed from Grid::base; [ctrl_begin, total): descriptors and
    // device state, addressed through Grid::cp (ctrl_begin == field_end)
    size_t ctrl_begin = 0;
    size_t ccell = 0, segs = 0, xpub = 0, xexp = 0, tiles2 = 0;
    size_t pend = 0, qslots = 0, qctl = 0;   // message-driven dependency counters and XCD queues
    size_t stamps = 0;                       // persistent timeline (hints bit 3)
};

// Per-chare baseline message buffers (byte offsets): outgoing face messages
// for both parities, incoming message per face.
struct MsgBufs {
    size_t out[2][6] = {{0}};
    size_t in[6] = {0};
    int64_t cnt[6] = {0, 0, 0, 0, 0, 0};
};

struct Grid {
    od_config cfg{};
    Plan plan;
    int s = 8;                       // bytes per element
    Layout L;
    std::vector<BlockDev> blocks_h;
    std::vector<TileDev> tiles_h;
    std::vector<int32_t> cpy;        // row pitch per chare
    std::vector<int32_t> dir_pb, ghost_pb, pb_face, pb_block;
    std::vector<int32_t> amr_pb;     // multi-resolution ghost buffer of (chare, face), -1 if none
    std::vector<FillSeg> segs_h;     // multi-resolution ghost fill rectangles
    int64_t fill_total = 0;          // ghost cells filled per iteration
    std::vector<XExpDev> xexp_h;     // per-chare x-column exports (empty: none)
    // two steps per pass (fused, graph, persistent and message-driven
    // forms, see two_step_possible): decided with the tile list; the
    // tiles' extra line descriptors
    bool two_step = false;
    std::vector<Tile2Dev> tiles2_h;
    int64_t halo2_cells = 0;         // cells of other chares within two steps of each chare
    std::vector<int32_t> dep_ptr, dep_idx;
    ImbDev imb{};                    // load-imbalance draw (heavy == 0: none)
    // Persistent schedule: 0 = automatic (counters for two-step passes,
    // under imbalance and with uneven blocks that keep one step per pass;
    // the fixed stride for other uniform one-step work), 1 = fixed
    // stride, 2 = tiles
    // from per-XCD-group counters, 3 = counters with the last tiles of each
    // group cut into z-ranges (guided_tail), 4 = fixed contiguous runs per
    // workgroup.  hints bits 4, 5, 11 and 13 force 2, 3, 4 and 1; the
    // autotuner may choose.
    int persist_sched = 0;
    int persist_waves = 0;           // cooperative waves per SIMD cap (0 = default)
    int msg_sched = 0;               // message-driven scheduler choice (MsgArgs::sched)
    int sched() const {
        if (cfg.hints & 2048) return 4;
        if (cfg.hints & 8192) return 1;
        if (cfg.hints & 32) return 3;
        if (cfg.hints & 16) return 2;
        if (persist_sched) return persist_sched;
        // counters, claimed as each tile ends, measured faster than the
        // stride for two-step passes at every ODF (512^3 fp64: 278-287 vs
        // 288-308 us per iteration) and under imbalance; the stride stays
        // for uniform one-step work
        if (imb.heavy > 0 || (!plan.regular && !plan.two_step_lines)) return 2;
        return two_step ? 2 : 1;
    }
    bool persistent_dyn() const { return sched() == 2 || sched() == 3; }
    // cooperative-kernel kind for persistent_max_grid
    int coop_kind() const {
        if (cfg.exec == OD_MSGDRIVEN) return two_step ? 5 : 1;
        if (plan.multires) return 6;
        return two_step ? (persistent_dyn() ? 4 : 3) : (persistent_dyn() ? 2 : 0);
    }
    std::vector<TileHost> base_tiles;   // the planner's tile list before schedule-specific cuts
    std::vector<MsgBufs> msg;
    int32_t nres = 1;
    size_t tile_cap = 0;             // tile descriptors the workspace has room for
    size_t tile2_cap = 0;            // two-step line descriptors it has room for

    // device state
    hipStream_t st = nullptr;
    hipStream_t cap_st = nullptr;
    char* base = nullptr;            // field storage
    char* ctrl = nullptr;            // control regions (L.ctrl_begin maps here)
    size_t ws_bytes = 0;
    // build_layout reserves descriptor room for every autotune candidate's
    // tiles (false: only the planned tiles)
    bool tune_room = true;
    // grids made by od_create_static: their control regions live in the
    // device's static array; a later od_create_static on the same device
    // supersedes them (static_gen no longer current)
    int static_dev = -1;
    uint64_t static_gen = 0;
    char* cp(size_t off) const { return ctrl + (off - L.ctrl_begin); }
    GridDev gdev{};
    int parity = 0;
    int64_t iters = 0;
    // message-driven grids: scheduler steps run so far, the value every
    // tile's step counter holds between launches (a two-step task is one
    // step), so parity == flips & 1
    int64_t flips = 0;
    bool msg_final = false;
    int32_t stamp_iters = 0;         // iterations of the last persistent launch with a timeline
    int grid_wgs = 0;
    std::map<std::pair<int, int64_t>, hipGraphExec_t> graphs;
    // per-chare baseline
    std::vector<hipStream_t> pool;
    std::vector<hipEvent_t> packed;
    hipEvent_t join_ev = nullptr;
    std::vector<int32_t> tile_lo;
    bool faces_packed = false;
    // host staging for I/O
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    bool pinned_borrowed = false;    // staging owned by someone else (serving)

    ~Grid();
    // kernel mode bits: od_config.hints, plus bit 8 for the 5-point stencil
    int mode() const { return (cfg.hints & ~0x100) | (cfg.stencil == 5 ? 0x100 : 0); }
    // message-driven scheduler bits (MsgArgs::sched): hints bits 6/7 force
    // cursor / ready-queue claims, bits 9/10 a publisher on / off; else the
    // tuner's choice (0 = automatic)
    int msg_sched_bits() const {
        int claim = (cfg.hints & 64) ? 1 : ((cfg.hints & 128) ? 2 : (msg_sched & 3));
        int pub = (cfg.hints & 512) ? 1 : ((cfg.hints & 1024) ? 2 : ((msg_sched >> 2) & 3));
        return claim | (pub << 2);
    }
    od_status upload();
    od_status reset_state();
    od_status init_field();
    od_status refresh_xexp(int par);   // x-column exports of field par from the chares
    const XExpDev* xexp_dev();         // device export table, nullptr without exports
    od_status ensure_pinned(size_t bytes);
    unsigned long long* res_ptr();
    od_status fused_one(hipStream_t s2, int par, int64_t step);
    od_status fused_two(hipStream_t s2, int par, int64_t step);   // steps step, step + 1: parity par -> par ^ 1
    od_status upload_tiles();                      // tile descriptors (and two-step lines) to the device
    int64_t bytes_per_pass() const;
    od_status graph_run(int64_t n);
    od_status persistent_run(int64_t n);
    od_status msgdriven_run(int64_t n);
    od_status msgdriven_launch(int64_t n, bool pairs);   // n scheduler steps (pairs: two-step tasks)
    od_status per_chare_run(int64_t n);
    od_status iterate(int64_t n);
    od_status residual(double* r);
    // sync the grid's stream; OD_ETIMEDOUT if a device-side wait gave up
    od_status device_error();
    od_status io(void* host, size_t bytes, bool to_host);
    od_status read_points(const int64_t* idx, int64_t count, void* host_dst);
    od_status block_io(int32_t b, void* host, size_t bytes, bool to_host);
    od_status retile(const int32_t tile[3]);
    // Cooperative forms: size the grid (workgroups that are co-resident)
    // and build the persistent form's tile list for its schedule (the
    // guided tail cuts the last tiles of each XCD group, see guided_tail);
    // uploads the tiles.  fresh_plan: plan.tiles was just planned (else the
    // list is rebuilt from base_tiles, e.g. after a schedule change).
    od_status setup_cooperative(bool fresh_plan = true);
};

std::string build_layout(const od_config& cfg, Grid& G);
std::string fill_tile_descs(Grid& G);
void decide_two_step(Grid& G);
// Smallest tile extents any autotune candidate uses for a dtype.
void tune_min_tile(int dtype_bytes, int32_t ey_max, int32_t m[3]);
od_status autotune(Grid& G, int32_t iters, int32_t out_tile[3]);
std::string build_tile_deps(const Plan& p, std::vector<int32_t>& ptr, std::vector<int32_t>& idx, bool reach2 = false);

}  // namespace od
