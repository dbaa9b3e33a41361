// Tile-shape autotuner for the fused sweep.
//
// A candidate is a compiled (TX, TY) kernel variant plus a z-column length
// TZ.  Every candidate evaluates each lattice point with the same
// expression in the same order, so tuning can change the time but never a
// bit of the result.  Candidates are timed on the grid itself by repeating
// one sweep from the current parity into the spare parity (the current
// field is never overwritten).  Results are cached per (dtype, exec mode,
// chare-shape histogram) in the process and, if OD_TUNE_CACHE names a file,
// on disk.
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
std::map<std::string, std::array<int32_t, 3>> g_cache;
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
    return os.str();
}

void load_file_cache() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char* path = std::getenv("OD_TUNE_CACHE");
    if (!path) return;
    std::ifstream in(path);
    std::string key;
    int32_t a, b, c;
    while (in >> key >> a >> b >> c) g_cache[key] = {a, b, c};
}

void store_file_cache(const std::string& key, const std::array<int32_t, 3>& t) {
    const char* path = std::getenv("OD_TUNE_CACHE");
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << t[0] << " " << t[1] << " " << t[2] << "\n";
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
    hipError_t he = hipMemcpyAsync(cp(L.tiles), tiles_h.data(), tiles_h.size() * sizeof(TileDev),
                                   hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("tile upload: ") + hipGetErrorString(he));
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
    if (cfg.exec == OD_PERSISTENT || cfg.exec == OD_MSGDRIVEN) {
        od_status cs = setup_cooperative();
        if (cs != OD_OK) return cs;
    }
    for (int d = 0; d < 3; ++d) cfg.tile[d] = plan.tile[d];
    return OD_OK;
}

od_status autotune(Grid& G, int32_t iters, int32_t out_tile[3]) {
    if (G.cfg.exec != OD_FUSED && G.cfg.exec != OD_GRAPH && G.cfg.exec != OD_PERSISTENT)
        return fail(OD_EINVAL, "autotune applies to OD_FUSED, OD_GRAPH and OD_PERSISTENT grids; create other "
                               "modes with cfg.tile set to a tuned shape");
    const std::string key = signature(G);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        load_file_cache();
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            od_status s = G.retile(it->second.data());
            if (s == OD_OK && out_tile)
                for (int d = 0; d < 3; ++d) out_tile[d] = G.plan.tile[d];
            return s;
        }
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
    const int32_t start_tile[3] = {G.plan.tile[0], G.plan.tile[1], G.plan.tile[2]};
    float best_ms = 1e30f;
    std::array<int32_t, 3> best = {start_tile[0], start_tile[1], start_tile[2]};
    od_status st = OD_OK;
    for (const auto& c : cands) {
        if (G.retile(c.data()) != OD_OK) continue;   // e.g. over the tile capacity
        auto launch = [&]() {
            return launch_sweep(G.s, G.plan.tile[0], G.plan.tile[1], G.st, G.base,
                                reinterpret_cast<const BlockDev*>(G.cp(G.L.blocks)),
                                reinterpret_cast<const TileDev*>(G.cp(G.L.tiles)), (int32_t)G.tiles_h.size(),
                                G.parity, G.res_ptr(), 0, 1, ImbDev{}, 0, G.mode());
        };
        he = launch();   // warm-up
        if (he == hipSuccess) he = hipEventRecord(a, G.st);
        for (int32_t i = 0; i < iters && he == hipSuccess; ++i) he = launch();
        if (he == hipSuccess) he = hipEventRecord(b, G.st);
        if (he == hipSuccess) he = hipEventSynchronize(b);
        float ms = 0;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, a, b);
        if (he != hipSuccess) {
            st = fail(OD_EHIP, std::string("tuning launch: ") + hipGetErrorString(he));
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (st != OD_OK) {
        G.retile(start_tile);
        return st;
    }
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
