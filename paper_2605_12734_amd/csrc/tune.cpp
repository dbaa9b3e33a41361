// Autotuner: tile shape and, for the cooperative forms, the schedule.
//
// A tile candidate is a compiled (TX, TY) kernel variant plus a z-column
// length TZ.  Every candidate evaluates each lattice point with the same
// expression in the same order, so tuning can change the time but never a
// bit of the result.  Fused and graph grids time their fused sweep,
// repeating one sweep from the current parity into the spare parity (the
// field is never overwritten).  Persistent grids time real multi-iteration
// launches of their persistent kernel under each schedule (fixed stride,
// counters, counters with a guided tail) and waves-per-SIMD cap (the
// kernel's register limit or one less); message-driven grids keep their
// tile (the dependency lists are built for it) and time their scheduler
// choices over real steps.  For both, the grid's state is saved to host
// memory before the search and restored after it.  Results are cached per (dtype, exec
// mode, grid and chare-shape histogram) in the process and, if
// OD_TUNE_CACHE names a file, on disk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "od_runtime.hpp"

namespace od {

namespace {

std::mutex g_cache_mu;
std::map<std::string, std::array<int32_t, 5>> g_cache;   // tile x, y, z, schedule, waves cap
bool g_cache_loaded = false;

const int32_t kTz[] = {8, 16, 32, 64, 128};
// single-row (2D) tiles march their second direction: longer columns
const int32_t kTz2d[] = {8, 32, 128, 512, 2048};

std::string signature(const Grid& G) {
    std::map<std::array<int32_t, 3>, int64_t> hist;
    for (const Chare& c : G.plan.chares) hist[{c.e[0], c.e[1], c.e[2]}]++;
    std::ostringstream os;
    os << "s" << G.s << "/e" << (int)G.cfg.exec << "/n" << G.plan.n[0] << "x" << G.plan.n[1] << "x" << G.plan.n[2];
    for (const auto& kv : hist) os << "/" << kv.first[0] << "x" << kv.first[1] << "x" << kv.first[2] << ":" << kv.second;
    // message-driven grids tune the scheduler at their own tile; schedule
    // checks and load imbalance change what is timed
    if (G.cfg.exec == OD_MSGDRIVEN)
        os << "/t" << G.plan.tile[0] << "x" << G.plan.tile[1] << "x" << G.plan.tile[2] << (G.two_step ? "/p2" : "");
    os << "/h" << (G.cfg.hints & ~1) << "/i" << G.cfg.imbalance_pct << "x" << G.cfg.imbalance_max_extra;
    return os.str();
}

void load_file_cache() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char* path = std::getenv("OD_TUNE_CACHE");
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string key;
        std::array<int32_t, 5> v = {0, 0, 0, 0, 0};
        if (!(ls >> key >> v[0] >> v[1] >> v[2])) continue;
        ls >> v[3] >> v[4];   // schedule and waves cap (absent in older entries: 0 = automatic)
        g_cache[key] = v;
    }
}

void store_file_cache(const std::string& key, const std::array<int32_t, 5>& t) {
    const char* path = std::getenv("OD_TUNE_CACHE");
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << t[0] << " " << t[1] << " " << t[2] << " " << t[3] << " " << t[4] << "\n";
}

}  // namespace

// Candidates for chares of at most ey_max rows: single-row variants only for
// grids one cell thick in y (the 2D stencil), multi-row ones otherwise.
static bool candidate_ok(const SweepVariant& v, int32_t ey_max) { return (v.ty == 1) == (ey_max == 1); }

void tune_min_tile(int dtype_bytes, int32_t ey_max, int32_t m[3]) {
    int n = 0;
    const SweepVariant* v = sweep_variants(dtype_bytes, &n);
    m[0] = m[1] = 1 << 30;
    for (int i = 0; i < n; ++i) {
        if (!candidate_ok(v[i], ey_max)) continue;
        m[0] = std::min(m[0], v[i].tx);
        m[1] = std::min(m[1], v[i].ty);
    }
    m[2] = kTz[0];
}

od_status Grid::retile(const int32_t tile[3]) {
    if (!sweep_variant_ok(s, tile[0], tile[1]) || tile[2] < 1)
        return fail(OD_EINVAL, "tile (" + std::to_string(tile[0]) + "," + std::to_string(tile[1]) + "," +
                                   std::to_string(tile[2]) + ") is not a compiled variant");
    int32_t old[3] = {plan.tile[0], plan.tile[1], plan.tile[2]};
    for (int d = 0; d < 3; ++d) plan.tile[d] = tile[d];
    std::string e = plan_tiles(plan);
    if (e.empty() && plan.tiles.size() > tile_cap) e = "tiles exceed the workspace's tile capacity";
    if (e.empty()) e = fill_tile_descs(*this);
    if (!e.empty()) {
        for (int d = 0; d < 3; ++d) plan.tile[d] = old[d];
        plan_tiles(plan);
        fill_tile_descs(*this);
        // the cooperative forms' list (and the persistent form's balanced
        // last round) is rebuilt for the old shape, matching the device copy
        if (cfg.exec == OD_PERSISTENT || cfg.exec == OD_MSGDRIVEN) setup_cooperative();
        return fail(OD_EINVAL, e);
    }
    od_status us = upload_tiles();
    if (us != OD_OK) return us;
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
    if (cfg.exec == OD_PERSISTENT || cfg.exec == OD_MSGDRIVEN) {
        od_status cs = setup_cooperative();
        if (cs != OD_OK) return cs;
    }
    for (int d = 0; d < 3; ++d) cfg.tile[d] = plan.tile[d];
    return OD_OK;
}

// Schedule state of a grid (persistent: schedule and waves cap;
// message-driven: scheduler bits and waves cap) as cached.
static void apply_schedule(Grid& G, int32_t sched, int32_t waves) {
    if (G.cfg.exec == OD_MSGDRIVEN)
        G.msg_sched = sched;
    else
        G.persist_sched = sched;
    G.persist_waves = waves;
}

// The grid's whole device state (field storage and control regions) and
// its iteration state, kept in host memory while tuning candidates run real
// iterations on the grid, then put back.
struct SavedState {
    std::vector<char> ctrl;
    size_t fbytes = 0;
    int64_t iters = 0, flips = 0;
    int parity = 0;
    bool msg_final = false;
};

static od_status save_state(Grid& G, SavedState& S) {
    hipError_t he = hipStreamSynchronize(G.st);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("sync: ") + hipGetErrorString(he));
    S.fbytes = G.L.field_end;
    S.ctrl.resize(G.L.total - G.L.ctrl_begin);
    od_status st = G.ensure_pinned(S.fbytes);
    if (st != OD_OK) return st;
    he = hipMemcpy(G.pinned, G.base, S.fbytes, hipMemcpyDeviceToHost);
    if (he == hipSuccess) he = hipMemcpy(S.ctrl.data(), G.ctrl, S.ctrl.size(), hipMemcpyDeviceToHost);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("save state: ") + hipGetErrorString(he));
    S.iters = G.iters;
    S.flips = G.flips;
    S.parity = G.parity;
    S.msg_final = G.msg_final;
    return OD_OK;
}

static hipError_t restore_state(Grid& G, const SavedState& S) {
    hipError_t he = hipStreamSynchronize(G.st);
    if (he == hipSuccess) he = hipMemcpy(G.base, G.pinned, S.fbytes, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(G.ctrl, S.ctrl.data(), S.ctrl.size(), hipMemcpyHostToDevice);
    G.iters = S.iters;
    G.flips = S.flips;
    G.parity = S.parity;
    G.msg_final = S.msg_final;
    return he;
}

// Message-driven grids: the scheduler choices (claims from the per-XCD
// cursor or from ready queues; a publisher workgroup per XCD or none) and
// the waves-per-SIMD cap, at the grid's tile.  Each candidate runs a launch
// of 2 * iters steps on the grid itself, between save_state and
// restore_state.
static od_status tune_msgdriven(Grid& G, int32_t iters, std::array<int32_t, 5>& best) {
    SavedState S;
    od_status st = save_state(G, S);
    if (st != OD_OK) return st;
    hipError_t he = hipSuccess;
    const int limit = coop_waves_limit(G.s, G.plan.tile[0], G.plan.tile[1], G.coop_kind());
    hipEvent_t a = nullptr, b = nullptr;
    he = hipEventCreate(&a);
    if (he == hipSuccess) he = hipEventCreate(&b);
    float best_ms = 1e30f;
    for (int claim = 1; claim <= 2 && he == hipSuccess && st == OD_OK; ++claim)
        for (int pub = 1; pub <= 2 && he == hipSuccess && st == OD_OK; ++pub)
            for (int w = limit; w >= std::max(1, limit - 1) && he == hipSuccess && st == OD_OK; --w) {
                apply_schedule(G, claim | (pub << 2), w);
                st = G.setup_cooperative(false);
                if (st != OD_OK) break;
                st = G.msgdriven_run(2);   // warm-up
                if (st != OD_OK) break;
                he = hipEventRecord(a, G.st);
                if (he == hipSuccess) st = G.msgdriven_run(2 * (int64_t)iters);
                if (he == hipSuccess && st == OD_OK) he = hipEventRecord(b, G.st);
                if (he == hipSuccess && st == OD_OK) he = hipEventSynchronize(b);
                float ms = 0;
                if (he == hipSuccess && st == OD_OK) he = hipEventElapsedTime(&ms, a, b);
                if (he == hipSuccess && st == OD_OK) st = G.device_error();
                if (he == hipSuccess && st == OD_OK && ms < best_ms) {
                    best_ms = ms;
                    best = {G.plan.tile[0], G.plan.tile[1], G.plan.tile[2], claim | (pub << 2), w};
                }
            }
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    // restore the grid as it was, with the chosen schedule
    hipError_t he2 = restore_state(G, S);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("tuning launch: ") + hipGetErrorString(he));
    if (he2 != hipSuccess) return fail(OD_EHIP, std::string("restore state: ") + hipGetErrorString(he2));
    if (st != OD_OK) return st;
    apply_schedule(G, best[3], best[4]);
    return G.setup_cooperative(false);
}

od_status autotune(Grid& G, int32_t iters, int32_t out_tile[3]) {
    if (G.cfg.exec == OD_PER_CHARE)
        return fail(OD_EINVAL, "autotune does not apply to OD_PER_CHARE grids; create them with cfg.tile set to a "
                               "tuned shape");
    if (iters < 1) return fail(OD_EINVAL, "iters must be >= 1");
    const std::string key = signature(G);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        load_file_cache();
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            const std::array<int32_t, 5> c = it->second;
            apply_schedule(G, c[3], c[4]);
            od_status s = G.cfg.exec == OD_MSGDRIVEN ? G.setup_cooperative(false) : G.retile(c.data());
            if (s == OD_OK && out_tile)
                for (int d = 0; d < 3; ++d) out_tile[d] = G.plan.tile[d];
            return s;
        }
    }
    if (G.cfg.exec == OD_MSGDRIVEN) {
        // the dependency lists are built for the planned tiles: the tile
        // stays, the scheduler is tuned
        std::array<int32_t, 5> best = {G.plan.tile[0], G.plan.tile[1], G.plan.tile[2], 0, 0};
        od_status s = tune_msgdriven(G, iters, best);
        if (s != OD_OK) return s;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_cache[key] = best;
            store_file_cache(key, best);
        }
        if (out_tile)
            for (int d = 0; d < 3; ++d) out_tile[d] = G.plan.tile[d];
        return OD_OK;
    }
    hipError_t he = hipStreamSynchronize(G.st);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("sync: ") + hipGetErrorString(he));
    // keep the residual slots: tuning launches overwrite them
    std::vector<unsigned long long> saved((size_t)(2 * G.nres + 2));
    he = hipMemcpy(saved.data(), G.cp(G.L.res), saved.size() * 8, hipMemcpyDeviceToHost);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("save residual: ") + hipGetErrorString(he));

    int32_t emax[3] = {1, 1, 1};
    for (const Chare& c : G.plan.chares)
        for (int d = 0; d < 3; ++d) emax[d] = std::max(emax[d], c.e[d]);
    std::vector<std::array<int32_t, 3>> cands;
    int nv = 0;
    const SweepVariant* v = sweep_variants(G.s, &nv);
    const int32_t vx = 16 / G.s;
    for (int i = 0; i < nv; ++i) {
        if (!candidate_ok(v[i], emax[1])) continue;
        if (v[i].tx > 2 * ((emax[0] + vx - 1) / vx * vx) && v[i].tx > 16) continue;   // mostly idle lanes
        if (v[i].ty > 2 * emax[1] && v[i].ty > 4) continue;
        std::vector<int32_t> tzs;
        if (emax[1] == 1) {
            for (int32_t tz : kTz2d)
                if (tz < emax[2]) tzs.push_back(tz);
        } else {
            for (int32_t tz : kTz)
                if (tz < emax[2]) tzs.push_back(tz);
        }
        tzs.push_back(emax[2]);
        for (int32_t tz : tzs) cands.push_back({v[i].tx, v[i].ty, tz});
    }
    hipEvent_t a = nullptr, b = nullptr;
    he = hipEventCreate(&a);
    if (he == hipSuccess) he = hipEventCreate(&b);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("event: ") + hipGetErrorString(he));
    od_status st = OD_OK;
    const int32_t start_tile[3] = {G.plan.tile[0], G.plan.tile[1], G.plan.tile[2]};
    const int32_t start_sched = G.persist_sched, start_waves = G.persist_waves;
    float best_ms = 1e30f;
    std::array<int32_t, 5> best = {start_tile[0], start_tile[1], start_tile[2], start_sched, start_waves};
    st = OD_OK;
    const bool pers = G.cfg.exec == OD_PERSISTENT;
    // persistent schedules: fixed stride (1), counters (2), counters with a
    // guided tail (3), fixed runs (4); hints bits 4/5/11/13 fix the schedule
    std::vector<int32_t> scheds = {0};
    // (multi-resolution grids always take tiles from counters)
    if (pers) scheds = (G.cfg.hints & (48 | 2048 | 8192)) || G.plan.multires ? std::vector<int32_t>{0}
                                                                            : std::vector<int32_t>{1, 2, 3, 4};
    // persistent candidates run real launches of 2 * iters iterations (the
    // barriers and counter resets are part of what is timed), so the grid's
    // state is saved first and restored after the search
    SavedState saved_state;
    if (pers) {
        st = save_state(G, saved_state);
        if (st != OD_OK) {
            hipEventDestroy(a);
            hipEventDestroy(b);
            return st;
        }
    }
    auto time_it = [&](float* ms_out) -> hipError_t {
        if (pers) {
            od_status ps = G.persistent_run(2);   // warm-up
            hipError_t e = ps == OD_OK ? hipEventRecord(a, G.st) : hipErrorLaunchFailure;
            if (e == hipSuccess) ps = G.persistent_run(2 * (int64_t)iters);
            if (ps != OD_OK) return hipErrorLaunchFailure;
            e = hipEventRecord(b, G.st);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            if (e == hipSuccess) e = hipEventElapsedTime(ms_out, a, b);
            if (e == hipSuccess && G.device_error() != OD_OK) e = hipErrorLaunchFailure;
            return e;
        }
        // a candidate with a two-step variant is timed as the grid would run
        // it (pairs of steps per pass), per step
        auto launch = [&]() {
            if (G.two_step)
                return launch_sweep2(G.s, G.plan.tile[0], G.plan.tile[1], G.st, G.base,
                                     reinterpret_cast<const BlockDev*>(G.cp(G.L.blocks)),
                                     reinterpret_cast<const TileDev*>(G.cp(G.L.tiles)),
                                     reinterpret_cast<const Tile2Dev*>(G.cp(G.L.tiles2)), (int32_t)G.tiles_h.size(),
                                     G.parity, G.res_ptr(), 0, 1, G.mode(), ImbDev{}, 0);
            return launch_sweep(G.s, G.plan.tile[0], G.plan.tile[1], G.st, G.base,
                                reinterpret_cast<const BlockDev*>(G.cp(G.L.blocks)),
                                reinterpret_cast<const TileDev*>(G.cp(G.L.tiles)), (int32_t)G.tiles_h.size(),
                                G.parity, G.res_ptr(), 0, 1, ImbDev{}, 0, G.mode(), G.xexp_dev());
        };
        hipError_t e = launch();   // warm-up
        if (e == hipSuccess) e = hipEventRecord(a, G.st);
        for (int32_t i = 0; i < iters && e == hipSuccess; ++i) e = launch();
        if (e == hipSuccess) e = hipEventRecord(b, G.st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(ms_out, a, b);
        if (e == hipSuccess && G.two_step) *ms_out *= 0.5f;
        return e;
    };
    for (const auto& c : cands) {
        if (G.retile(c.data()) != OD_OK) continue;   // e.g. over the tile capacity
        for (int32_t sc : scheds) {
            const int kind = (sc == 2 || sc == 3) ? 2 : 0;
            const int limit = pers ? coop_waves_limit(G.s, G.plan.tile[0], G.plan.tile[1], kind) : 0;
            for (int w = limit; w >= (pers ? std::max(1, limit - 1) : 0); --w) {
                if (pers) {
                    apply_schedule(G, sc, w);
                    if (G.setup_cooperative(false) != OD_OK) continue;
                }
                float ms = 0;
                he = time_it(&ms);
                if (he != hipSuccess) {
                    st = fail(OD_EHIP, std::string("tuning launch: ") + hipGetErrorString(he));
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = {c[0], c[1], c[2], pers ? sc : 0, pers ? w : 0};
                }
                if (!pers) break;
            }
            if (st != OD_OK) break;
        }
        if (st != OD_OK) break;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (pers) {
        he = restore_state(G, saved_state);
        if (he != hipSuccess && st == OD_OK) st = fail(OD_EHIP, std::string("restore state: ") + hipGetErrorString(he));
    }
    if (st != OD_OK) {
        apply_schedule(G, start_sched, start_waves);
        G.retile(start_tile);
        return st;
    }
    apply_schedule(G, best[3], best[4]);
    st = G.retile(best.data());
    if (st != OD_OK) return st;
    he = hipMemcpy(G.cp(G.L.res), saved.data(), saved.size() * 8, hipMemcpyHostToDevice);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("restore residual: ") + hipGetErrorString(he));
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache[key] = best;
        store_file_cache(key, best);
    }
    if (out_tile)
        for (int d = 0; d < 3; ++d) out_tile[d] = best[d];
    return OD_OK;
}

}  // namespace od
