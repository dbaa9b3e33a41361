// extern "C" entry points of libod (declared in include/od.h).  Argument
// checking and error reporting live here; the work is done by od::Grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "od_runtime.hpp"

using od::fail;
using od::Grid;

struct od_grid {
    Grid g;
};

// Control regions (descriptors, residual slots, barrier and step counters,
// queues) of grids made by od_create_static, for callers that cannot
// allocate device memory.  Each GPU holds its own copy of the array until
// the process ends; host code addresses it only through the per-device
// pointer from hipGetSymbolAddress, never through the array's name.
constexpr size_t kStaticControlBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticControlBytes];

namespace {

od_status plan_only(const od_config* cfg, Grid& G) {
    if (cfg == nullptr) return fail(OD_EINVAL, "cfg is NULL");
    std::string err = od::build_layout(*cfg, G);
    if (!err.empty()) return fail(OD_EINVAL, err);
    return OD_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char* g_static_ptr[kMaxDevices] = {};
std::atomic<uint64_t> g_static_gen[kMaxDevices];

// Device address of this device's static control array (looked up once per
// device, with the device current).
od_status static_control(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(OD_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return fail(OD_EHIP, std::string("hipGetSymbolAddress(static control array): ") + hipGetErrorString(e));
        if (reinterpret_cast<uintptr_t>(ptr) % od::kAlign != 0)
            return fail(OD_EHIP, "static control array is not 256-byte aligned");
        g_static_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = g_static_ptr[dev];
    return OD_OK;
}

bool static_superseded(const Grid& G) {
    return G.static_gen != 0 && g_static_gen[G.static_dev].load(std::memory_order_acquire) != G.static_gen;
}

#define OD_GUARD_BEGIN try {
#define OD_GUARD_END                                                              \
    }                                                                             \
    catch (const std::bad_alloc&) {                                               \
        return fail(OD_ENOMEM, "host allocation failed");                         \
    }                                                                             \
    catch (const std::exception& ex) {                                            \
        return fail(OD_EINVAL, std::string("internal error: ") + ex.what());      \
    }                                                                             \
    catch (...) {                                                                 \
        return fail(OD_EINVAL, "internal error");                                 \
    }

}  // namespace

extern "C" {

void od_config_default(od_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n[0] = cfg->n[1] = cfg->n[2] = 64;
    cfg->odf = 8;
    cfg->dtype = OD_F64;
    cfg->bc[0] = 1.0;
    cfg->seed = 12734;
    cfg->exec = OD_GRAPH;
}

const char* od_last_error(void) { return od::g_last_error.c_str(); }

const char* od_version(void) { return "od 0.1 (gfx950)"; }

od_status od_workspace_bytes(const od_config* cfg, size_t* bytes) {
    OD_GUARD_BEGIN
    if (bytes == nullptr) return fail(OD_EINVAL, "bytes is NULL");
    Grid G;
    od_status s = plan_only(cfg, G);
    if (s != OD_OK) return s;
    *bytes = G.L.total;
    return OD_OK;
    OD_GUARD_END
}

od_status od_create(const od_config* cfg, void* hip_stream, void* dev_workspace, size_t workspace_bytes,
                    od_grid** out) {
    OD_GUARD_BEGIN
    if (out == nullptr) return fail(OD_EINVAL, "out is NULL");
    *out = nullptr;
    std::unique_ptr<od_grid> h(new od_grid);
    Grid& G = h->g;
    od_status s = plan_only(cfg, G);
    if (s != OD_OK) return s;
    if (dev_workspace == nullptr) return fail(OD_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % od::kAlign != 0)
        return fail(OD_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < G.L.total)
        return fail(OD_ENOMEM, "workspace of " + std::to_string(workspace_bytes) + " bytes, need " +
                                   std::to_string(G.L.total));
    G.st = static_cast<hipStream_t>(hip_stream);
    G.base = static_cast<char*>(dev_workspace);
    G.ws_bytes = workspace_bytes;
    s = G.upload();
    if (s != OD_OK) return s;
    s = G.reset_state();
    if (s != OD_OK) return s;
    s = G.init_field();
    if (s != OD_OK) return s;
    s = G.setup_cooperative();
    if (s != OD_OK) return s;
    hipError_t e = hipStreamSynchronize(G.st);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("create sync: ") + hipGetErrorString(e));
    *out = h.release();
    return OD_OK;
    OD_GUARD_END
}

od_status od_create_static(const od_config* cfg, void* hip_stream, void* dev_fields, size_t field_bytes,
                           od_grid** out) {
    OD_GUARD_BEGIN
    if (out == nullptr) return fail(OD_EINVAL, "out is NULL");
    *out = nullptr;
    if (cfg == nullptr) return fail(OD_EINVAL, "cfg is NULL");
    if (cfg->exec != OD_FUSED && cfg->exec != OD_PERSISTENT && cfg->exec != OD_MSGDRIVEN)
        return fail(OD_EINVAL, "od_create_static supports OD_FUSED, OD_PERSISTENT and OD_MSGDRIVEN (the graph "
                               "and per-chare forms create graphs and streams when they first iterate)");
    std::unique_ptr<od_grid> h(new od_grid);
    Grid& G = h->g;
    G.tune_room = false;   // descriptor room for the planned tiles only
    od_status s = plan_only(cfg, G);
    if (s != OD_OK) return s;
    const size_t ctrl_bytes = G.L.total - G.L.ctrl_begin;
    if (ctrl_bytes > kStaticControlBytes)
        return fail(OD_ENOMEM, "grid needs " + std::to_string(ctrl_bytes) +
                                   " bytes of control state; the static array holds " +
                                   std::to_string(kStaticControlBytes));
    if (dev_fields == nullptr) return fail(OD_EINVAL, "field buffer is NULL");
    if (reinterpret_cast<uintptr_t>(dev_fields) % od::kAlign != 0)
        return fail(OD_EINVAL, "field buffer must be 256-byte aligned");
    if (field_bytes < G.L.ctrl_begin)
        return fail(OD_ENOMEM, "field buffer of " + std::to_string(field_bytes) + " bytes, need " +
                                   std::to_string(G.L.ctrl_begin));
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
    char* ctrl = nullptr;
    s = static_control(dev, &ctrl);
    if (s != OD_OK) return s;
    G.st = static_cast<hipStream_t>(hip_stream);
    G.base = static_cast<char*>(dev_fields);
    G.ctrl = ctrl;
    G.ws_bytes = field_bytes;
    G.static_dev = dev;
    G.static_gen = g_static_gen[dev].fetch_add(1, std::memory_order_acq_rel) + 1;
    // upload writes every descriptor; reset_state clears the residual
    // slots, barrier words, error flag and step counters the previous user
    // of the array left behind
    s = G.upload();
    if (s != OD_OK) return s;
    s = G.reset_state();
    if (s != OD_OK) return s;
    s = G.init_field();
    if (s != OD_OK) return s;
    s = G.setup_cooperative();
    if (s != OD_OK) return s;
    he = hipStreamSynchronize(G.st);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("create sync: ") + hipGetErrorString(he));
    *out = h.release();
    return OD_OK;
    OD_GUARD_END
}

od_status od_plan_create(const od_config* cfg, od_grid** out) {
    OD_GUARD_BEGIN
    if (out == nullptr) return fail(OD_EINVAL, "out is NULL");
    *out = nullptr;
    std::unique_ptr<od_grid> h(new od_grid);
    od_status s = plan_only(cfg, h->g);
    if (s != OD_OK) return s;
    *out = h.release();
    return OD_OK;
    OD_GUARD_END
}

#define OD_NEED_DEVICE(g)                                                                  \
    do {                                                                                   \
        if (!(g)) return fail(OD_EINVAL, "grid is NULL");                                  \
        if ((g)->g.base == nullptr) return fail(OD_EINVAL, "host-only plan handle");       \
        if (static_superseded((g)->g))                                                     \
            return fail(OD_EINVAL, "grid superseded by a later od_create_static on its device"); \
    } while (0)

od_status od_iterate(od_grid* g, int64_t n) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    return g->g.iterate(n);
    OD_GUARD_END
}

od_status od_residual(od_grid* g, double* r) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    if (!r) return fail(OD_EINVAL, "NULL argument");
    return g->g.residual(r);
    OD_GUARD_END
}

od_status od_iterations(od_grid* g, int64_t* iters) {
    if (!g || !iters) return fail(OD_EINVAL, "NULL argument");
    *iters = g->g.iters;
    return OD_OK;
}

#define OD_NEED_UNIFORM(g)                                                                           \
    do {                                                                                             \
        if ((g)->g.plan.multires)                                                                    \
            return fail(OD_EINVAL, "multi-resolution grid: use od_read_block / od_write_block");     \
    } while (0)

od_status od_read(od_grid* g, void* host_dst, size_t bytes) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    OD_NEED_UNIFORM(g);
    if (!host_dst) return fail(OD_EINVAL, "NULL argument");
    return g->g.io(host_dst, bytes, true);
    OD_GUARD_END
}

od_status od_write(od_grid* g, const void* host_src, size_t bytes) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    OD_NEED_UNIFORM(g);
    if (!host_src) return fail(OD_EINVAL, "NULL argument");
    return g->g.io(const_cast<void*>(host_src), bytes, false);
    OD_GUARD_END
}

od_status od_read_points(od_grid* g, const int64_t* idx, int64_t count, void* host_dst) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    OD_NEED_UNIFORM(g);
    if (count > 0 && (!idx || !host_dst)) return fail(OD_EINVAL, "NULL argument");
    return g->g.read_points(idx, count, host_dst);
    OD_GUARD_END
}

od_status od_block_cells(od_grid* g, int32_t b, int32_t cells[3]) {
    if (!g || !cells) return fail(OD_EINVAL, "NULL argument");
    const Grid& G = g->g;
    if (b < 0 || b >= (int32_t)G.plan.chares.size()) return fail(OD_EINVAL, "block index out of range");
    for (int d = 0; d < 3; ++d) cells[d] = G.plan.chares[(size_t)b].e[d];
    return OD_OK;
}

od_status od_read_block(od_grid* g, int32_t b, void* host_dst, size_t bytes) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    if (!host_dst) return fail(OD_EINVAL, "NULL argument");
    return g->g.block_io(b, host_dst, bytes, true);
    OD_GUARD_END
}

od_status od_write_block(od_grid* g, int32_t b, const void* host_src, size_t bytes) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    if (!host_src) return fail(OD_EINVAL, "NULL argument");
    return g->g.block_io(b, const_cast<void*>(host_src), bytes, false);
    OD_GUARD_END
}

od_status od_plan(od_grid* g, od_plan_info* info) {
    if (!g || !info) return fail(OD_EINVAL, "NULL argument");
    const Grid& G = g->g;
    info->nchares = (int32_t)G.plan.chares.size();
    info->ntiles = (int32_t)G.tiles_h.size();
    info->npseudo = (int32_t)(G.blocks_h.size() - G.plan.chares.size());
    info->interior = G.plan.interior;
    info->halo_cells = G.plan.halo_cells;
    info->bytes_per_iter = (int64_t)G.s * (2 * G.plan.interior + G.plan.halo_cells);
    for (int d = 0; d < 3; ++d) info->tile[d] = G.plan.tile[d];
    info->grid_wgs = G.grid_wgs;
    info->schedule = G.cfg.exec == OD_PERSISTENT ? G.sched() : (G.cfg.exec == OD_MSGDRIVEN ? G.msg_sched_bits() : 0);
    info->coop_waves = G.persist_waves;
    info->field_bytes = (int64_t)G.L.ctrl_begin;
    info->control_bytes = (int64_t)(G.L.total - G.L.ctrl_begin);
    info->steps_per_pass = G.two_step ? 2 : 1;
    info->bytes_per_pass = G.bytes_per_pass();
    return OD_OK;
}

od_status od_tile_info_get(od_grid* g, int32_t t, od_tile_info* out) {
    if (!g || !out) return fail(OD_EINVAL, "NULL argument");
    const Grid& G = g->g;
    if (t < 0 || t >= (int32_t)G.plan.tiles.size()) return fail(OD_EINVAL, "tile index out of range");
    const od::TileHost& th = G.plan.tiles[(size_t)t];
    out->chare = th.chare;
    for (int d = 0; d < 3; ++d) {
        out->origin[d] = th.o[d];
        out->extent[d] = th.e[d];
    }
    for (int f = 0; f < 6; ++f) {
        out->src_kind[f] = th.kind[f] == 1 ? 1 : (th.kind[f] == 3 ? 2 : 0);
        out->src[f] = th.kind[f] == 2 ? th.chare : th.src[f];
        for (int d = 0; d < 3; ++d) out->src_origin[f][d] = th.g[f][d];
    }
    return OD_OK;
}

od_status od_tile_deps(od_grid* g, int32_t t, int32_t* out, int32_t cap, int32_t* count) {
    if (!g || !count || (cap > 0 && !out)) return fail(OD_EINVAL, "NULL argument");
    const Grid& G = g->g;
    if (G.cfg.exec != OD_MSGDRIVEN) return fail(OD_EINVAL, "dependency lists exist for OD_MSGDRIVEN grids only");
    if (t < 0 || t >= (int32_t)G.plan.tiles.size() || (size_t)t + 1 >= G.dep_ptr.size())
        return fail(OD_EINVAL, "tile index out of range");
    const int32_t lo = G.dep_ptr[(size_t)t], hi = G.dep_ptr[(size_t)t + 1];
    *count = hi - lo;
    for (int32_t i = 0; i < hi - lo && i < cap; ++i) out[i] = G.dep_idx[(size_t)(lo + i)];
    return OD_OK;
}

od_status od_chare_get(od_grid* g, int32_t c, od_block* out) {
    if (!g || !out) return fail(OD_EINVAL, "NULL argument");
    const Grid& G = g->g;
    if (c < 0 || c >= (int32_t)G.plan.chares.size()) return fail(OD_EINVAL, "chare index out of range");
    const od::Chare& ch = G.plan.chares[(size_t)c];
    for (int d = 0; d < 3; ++d) {
        out->origin[d] = ch.u[d];
        out->extent[d] = ch.e[d] * ch.h;
    }
    return OD_OK;
}

od_status od_timeline(od_grid* g, double* out, int32_t max_iters, int32_t* n_iters) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    if (!out || !n_iters || max_iters < 0) return fail(OD_EINVAL, "NULL argument or negative max_iters");
    Grid& G = g->g;
    if (G.cfg.exec != OD_PERSISTENT || !(G.cfg.hints & od::kHintTimeline))
        return fail(OD_EINVAL, "the timeline is recorded by OD_PERSISTENT grids created with hints bit 3");
    od_status s = G.device_error();
    if (s != OD_OK) return s;
    const int32_t n = std::min(G.stamp_iters, max_iters);
    std::vector<unsigned long long> v((size_t)4 * n);
    if (n > 0) {
        hipError_t e = hipMemcpy(v.data(), G.cp(G.L.stamps), v.size() * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("read timeline: ") + hipGetErrorString(e));
    }
    const double us_per_tick = 1e6 / (double)od::device_wait_ticks(1.0);
    for (size_t i = 0; i < v.size(); ++i) out[i] = ((double)v[i] - (double)v[0]) * us_per_tick;
    *n_iters = n;
    return OD_OK;
    OD_GUARD_END
}

od_status od_extra_sweeps(od_grid* g, int64_t step, int32_t* out, int32_t n) {
    if (!g || !out) return fail(OD_EINVAL, "NULL argument");
    const Grid& G = g->g;
    if (n != (int32_t)G.plan.chares.size()) return fail(OD_EINVAL, "n must equal the number of chares");
    if (step < 0) return fail(OD_EINVAL, "step must be >= 0");
    for (int32_t c = 0; c < n; ++c) out[c] = od::imb_extra(G.imb, step, c);
    return OD_OK;
}

od_status od_destroy(od_grid* g) {
    if (!g) return OD_OK;
    hipError_t e = g->g.base ? hipStreamSynchronize(g->g.st) : hipSuccess;
    delete g;
    if (e != hipSuccess) return fail(OD_EHIP, std::string("destroy sync: ") + hipGetErrorString(e));
    return OD_OK;
}

od_status od_stream_bench(void* hip_stream, void* dst, const void* src, size_t bytes, int32_t iters, int32_t kind,
                          double* seconds, int32_t* variant) {
    if (!dst || !src || !seconds || iters < 1 || bytes % 16 != 0 || bytes == 0 || kind < 0 || kind > 2)
        return fail(OD_EINVAL, "need non-NULL buffers, bytes a positive multiple of 16, iters >= 1, kind 0..2");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    uint32_t* sink = static_cast<uint32_t*>(dst);
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    double best = 1e30;
    int32_t best_v = -1;
    for (int v = 0; v < od::copy_variant_count() && e == hipSuccess; ++v) {
        e = od::launch_stream(st, dst, src, bytes, v, kind, sink);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(a, st);
        for (int32_t i = 0; i < iters && e == hipSuccess; ++i) e = od::launch_stream(st, dst, src, bytes, v, kind, sink);
        if (e == hipSuccess) e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && ms * 1e-3 < best) {
            best = ms * 1e-3;
            best_v = v;
        }
    }
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("stream bench: ") + hipGetErrorString(e));
    *seconds = best;
    if (variant) *variant = best_v;
    return OD_OK;
}

od_status od_stream_copy(void* hip_stream, void* dst, const void* src, size_t bytes, int32_t iters, double* seconds) {
    return od_stream_bench(hip_stream, dst, src, bytes, iters, 0, seconds, nullptr);
}

od_status od_time_iterate(od_grid* g, int64_t n, double* seconds) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    if (!seconds) return fail(OD_EINVAL, "NULL argument");
    Grid& G = g->g;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("event: ") + hipGetErrorString(e));
    od_status s = OD_OK;
    e = hipEventRecord(a, G.st);
    if (e == hipSuccess) s = G.iterate(n);
    if (e == hipSuccess && s == OD_OK) e = hipEventRecord(b, G.st);
    if (e == hipSuccess && s == OD_OK) e = hipEventSynchronize(b);
    float ms = 0;
    if (e == hipSuccess && s == OD_OK) e = hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (s != OD_OK) return s;
    if (e != hipSuccess) return fail(OD_EHIP, std::string("timing: ") + hipGetErrorString(e));
    *seconds = ms * 1e-3;
    return OD_OK;
    OD_GUARD_END
}

od_status od_autotune(od_grid* g, int32_t iters, int32_t out_tile[3]) {
    OD_GUARD_BEGIN
    OD_NEED_DEVICE(g);
    if (iters < 1) return fail(OD_EINVAL, "iters must be >= 1");
    return od::autotune(g->g, iters, out_tile);
    OD_GUARD_END
}

}  // extern "C"
