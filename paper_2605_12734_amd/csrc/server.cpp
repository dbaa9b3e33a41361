// Serving: independent Jacobi solves of different sizes and precisions,
// admitted as they arrive under a device-memory budget and run together by
// the message-driven device scheduler (continuous batching).
//
// A worker thread owns the device.  Each round it admits queued requests
// (FIFO) while a slot and arena space are free, then launches one
// scheduling epoch: a cooperative kernel over the tiles of every resident
// solve, in which any tile runs as soon as the tiles it reads halos from
// have finished the previous step.  A solve stops at the first decision
// step (a multiple of its check_every) whose residual is below its
// tolerance, or at its cap; the last tile to finish that step writes the
// completion record (final step, residual) to host-coherent memory, where
// the worker stamps the completion time while the epoch keeps running.  To
// admit new arrivals or retire finished solves the worker raises a yield
// flag; every workgroup then stops taking new tasks and the epoch ends.  All
// scheduler state (per-tile step counters, gates, residual slots) lives in
// HBM, so the next epoch resumes exactly where this one stopped.  A
// finished solve leaves the next epoch's tile list; a second host thread
// copies its field to host memory with the copy engine while the worker
// goes on launching and polling, then frees its slot and arena space.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "od_runtime.hpp"

namespace od {

namespace {

constexpr int32_t kMaxTiles = 8192;                 // tiles per solve
constexpr int32_t kTileStride = kMaxTiles + 1;      // per-slot stride of per-tile arrays
constexpr int32_t kMaxBlocks = 256;                 // chares + Dirichlet faces per solve
constexpr int32_t kMaxDeps = 8 * kMaxTiles;         // dependency entries per solve
constexpr size_t kMaxQueue = 1 << 16;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

od_config request_config(const od_request& r) {
    od_config c;
    od_config_default(&c);
    c.n[0] = c.n[1] = c.n[2] = r.n;
    c.odf = r.odf;
    c.dtype = r.dtype;
    for (int i = 0; i < 6; ++i) c.bc[i] = r.bc[i];
    c.seed = r.seed;
    c.exec = OD_MSGDRIVEN;
    // the serving kernel runs tasks of one step (a solve may stop at any
    // step): its dependency lists reach one cell
    c.hints = 4096;
    if (r.dtype == OD_F64) {
        c.tile[0] = kServeTx8;
        c.tile[1] = kServeTy8;
    } else {
        c.tile[0] = kServeTx4;
        c.tile[1] = kServeTy4;
    }
    c.tile[2] = 32;
    return c;
}

}  // namespace

struct Request {
    uint64_t ticket = 0;
    od_request req{};
    size_t bytes = 0;
    int32_t state = OD_REQ_QUEUED;
    int32_t slot = -1;
    double t_arrival = 0, t_submit = 0, t_admit = 0, t_done = 0;
    int64_t iters = 0;
    double residual = 0;
    std::unique_ptr<Grid> grid;
    size_t off = 0;
    bool finished = false;           // final step reached; waiting to be copied out
    std::vector<char> result;
};

struct Server {
    hipStream_t st = nullptr;
    hipStream_t cst = nullptr;        // result copies (copy engine), overlapping the next epoch
    char* arena = nullptr;
    size_t arena_bytes = 0;
    int32_t max_slots = 0;
    // control region (byte offsets from arena)
    size_t c_blocks = 0, c_tiles = 0, c_done = 0, c_dep_ptr = 0, c_dep_idx = 0, c_tile_solve = 0;
    size_t c_target = 0, c_final = 0, c_gate = 0, c_count = 0, c_res = 0, c_ce = 0, c_tol = 0, c_ntiles = 0;
    size_t c_dtype = 0, c_list = 0, c_err = 0, c_yield = 0, c_xpub = 0, c_tpos = 0, c_bar = 0;
    size_t c_sbase = 0, c_pend = 0, c_qslots = 0, c_qctl = 0;
    size_t data_begin = 0;
    // host-coherent completion records and the yield flag
    int32_t* h_done = nullptr;
    unsigned long long* h_res = nullptr;
    int32_t* h_yield = nullptr;
    void* staging = nullptr;          // pinned host staging for result copies
    size_t staging_bytes = 0;
    // arena allocator over [data_begin, arena_bytes): offset -> size
    std::map<size_t, size_t> free_list;

    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    // finished solves waiting to be copied out, and the thread that does it
    std::deque<Request*> retire_q;
    std::condition_variable rcv;
    std::thread retirer;
    bool retire_stop = false;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<uint64_t> slot_ticket;
    uint64_t next_ticket = 1;
    int32_t grid_cap = 0;
    // od_server_set_hints: kernel hints of later epochs (bit 2: schedule
    // check) and the seed of the schedule perturbation
    std::atomic<int32_t> hints{0};
    std::atomic<uint64_t> check_seed{12734};
    std::string fatal;
    od_server_stats stats{};          // guarded by mu

    size_t alloc(size_t bytes) {
        bytes = align_up(bytes, kAlign);
        for (auto it = free_list.begin(); it != free_list.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rest = it->second - bytes;
                free_list.erase(it);
                if (rest) free_list[off + bytes] = rest;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes, kAlign);
        auto it = free_list.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_list.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_list.erase(nx);
        }
        if (it != free_list.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_list.erase(it);
            }
        }
    }
    bool fits_somewhere(size_t bytes) const {
        bytes = align_up(bytes, kAlign);
        for (const auto& kv : free_list)
            if (kv.second >= bytes) return true;
        return false;
    }
    int32_t free_slot() const {
        for (int32_t s = 0; s < max_slots; ++s)
            if (slot_ticket[(size_t)s] == 0) return s;
        return -1;
    }

    // the worker has something to do: a running solve, or a queued request
    // that a free slot and free arena space can take (caller holds mu)
    bool worker_has_work() const {
        for (uint64_t t : slot_ticket) {
            if (!t) continue;
            const auto it = reqs.find(t);
            if (it != reqs.end() && it->second->state == OD_REQ_RUNNING && !it->second->finished) return true;
        }
        if (queue.empty()) return false;
        const auto it = reqs.find(queue.front());
        return it == reqs.end() || (free_slot() >= 0 && fits_somewhere(it->second->bytes));
    }

    od_status setup_slot(Request& R, int32_t slot);
    void run();
    void retire(Request& R);
    void retire_run();
    void cancel_unfinished();
};

// ---- admission: plan the solve, initialise it, fill its slot's tables ------

od_status Server::setup_slot(Request& R, int32_t slot) {
    Grid& G = *R.grid;
    G.st = st;
    G.base = arena + R.off;
    G.ws_bytes = R.bytes;
    od_status s = G.upload();
    if (s == OD_OK) s = G.reset_state();
    if (s == OD_OK) s = G.init_field();
    if (s != OD_OK) return s;
    const int32_t ntiles = (int32_t)G.tiles_h.size();
    const int sb = G.s;
    std::vector<BlockDev> blocks(G.blocks_h);
    for (BlockDev& b : blocks) {
        b.off[0] += (int64_t)(R.off / (size_t)sb);
        b.off[1] += (int64_t)(R.off / (size_t)sb);
    }
    std::vector<TileDev> tiles(G.tiles_h);
    for (TileDev& t : tiles) {
        t.blk += slot * kMaxBlocks;
        for (int f = 0; f < 6; ++f) t.f[f].src += slot * kMaxBlocks;
        t.rslot = slot;
    }
    const int32_t tbase = slot * kTileStride;
    std::vector<int32_t> dep_ptr((size_t)ntiles + 1), dep_idx(G.dep_idx.size());
    for (int32_t i = 0; i <= ntiles; ++i) dep_ptr[(size_t)i] = slot * kMaxDeps + G.dep_ptr[(size_t)i];
    for (size_t q = 0; q < G.dep_idx.size(); ++q) dep_idx[q] = tbase + G.dep_idx[q];
    std::vector<int32_t> zeros((size_t)ntiles, 0), owner((size_t)ntiles, slot);
    const int32_t tgt = (int32_t)R.req.max_iters, zero = 0, ce = R.req.check_every, dt = (int32_t)R.req.dtype;
    const unsigned long long zr = 0;
    const double tol = R.req.tol;
    auto put = [&](size_t off, const void* src, size_t n) -> hipError_t {
        return n ? hipMemcpyAsync(arena + off, src, n, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    hipError_t e = put(c_blocks + (size_t)slot * kMaxBlocks * sizeof(BlockDev), blocks.data(),
                       blocks.size() * sizeof(BlockDev));
    if (e == hipSuccess) e = put(c_tiles + (size_t)tbase * sizeof(TileDev), tiles.data(), tiles.size() * sizeof(TileDev));
    if (e == hipSuccess) e = put(c_done + (size_t)tbase * 4, zeros.data(), zeros.size() * 4);
    if (e == hipSuccess) e = put(c_tile_solve + (size_t)tbase * 4, owner.data(), owner.size() * 4);
    if (e == hipSuccess) e = put(c_dep_ptr + (size_t)tbase * 4, dep_ptr.data(), dep_ptr.size() * 4);
    if (e == hipSuccess) e = put(c_dep_idx + (size_t)slot * kMaxDeps * 4, dep_idx.data(), dep_idx.size() * 4);
    if (e == hipSuccess) e = put(c_target + (size_t)slot * 4, &tgt, 4);
    if (e == hipSuccess) e = put(c_final + (size_t)slot * 4, &zero, 4);
    if (e == hipSuccess) e = put(c_gate + (size_t)slot * 4, &zero, 4);
    if (e == hipSuccess) e = put(c_count + (size_t)slot * 4, &zero, 4);
    if (e == hipSuccess) e = put(c_res + (size_t)slot * 8, &zr, 8);
    if (e == hipSuccess) e = put(c_ce + (size_t)slot * 4, &ce, 4);
    if (e == hipSuccess) e = put(c_tol + (size_t)slot * 8, &tol, 8);
    if (e == hipSuccess) e = put(c_ntiles + (size_t)slot * 4, &ntiles, 4);
    if (e == hipSuccess) e = put(c_dtype + (size_t)slot * 4, &dt, 4);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("serving admission: ") + hipGetErrorString(e));
    h_done[slot] = 0;
    h_res[slot] = 0;
    return OD_OK;
}

void Server::retire(Request& R) {
    // The solve's field is final and no kernel touches it any more: copy
    // each chare's storage (final parity) to host memory with the copy
    // engine while the next epoch runs, lay it out as the padded global
    // field (Dirichlet shell from the request), free the arena space.
    Grid& G = *R.grid;
    const int32_t fs = __atomic_load_n(&h_done[R.slot], __ATOMIC_ACQUIRE);
    unsigned long long rb = __atomic_load_n(&h_res[R.slot], __ATOMIC_ACQUIRE);
    double r;
    std::memcpy(&r, &rb, 8);
    const int par = fs & 1;
    const int64_t n = R.req.n, P = n + 2;
    const size_t s = (size_t)G.s;
    std::vector<char> host((size_t)P * P * P * s, 0);
    auto put = [&](int64_t i, int64_t j, int64_t k, double v) {
        char* d = host.data() + (size_t)((k * P + j) * P + i) * s;
        if (s == 8) std::memcpy(d, &v, 8);
        else {
            const float f = (float)v;
            std::memcpy(d, &f, 4);
        }
    };
    for (int64_t a = 1; a <= n; ++a)
        for (int64_t b = 1; b <= n; ++b) {
            put(0, a, b, R.req.bc[0]);
            put(P - 1, a, b, R.req.bc[1]);
            put(a, 0, b, R.req.bc[2]);
            put(a, P - 1, b, R.req.bc[3]);
            put(a, b, 0, R.req.bc[4]);
            put(a, b, P - 1, R.req.bc[5]);
        }
    hipError_t e = hipSuccess;
    char* stage = static_cast<char*>(staging);
    for (size_t c = 0; c < G.plan.chares.size() && e == hipSuccess; ++c) {
        const Chare& ch = G.plan.chares[c];
        const BlockDev& B = G.blocks_h[c];
        const char* src = G.base + (size_t)(par ? B.off[1] : B.off[0]) * s;
        const size_t plane = (size_t)B.pz * s, row = (size_t)B.ex * s;
        const int32_t per = (int32_t)std::max<size_t>(1, staging_bytes / plane);
        for (int32_t z0 = 0; z0 < B.ez && e == hipSuccess; z0 += per) {
            const int32_t nz = std::min<int32_t>(per, B.ez - z0);
            e = hipMemcpyAsync(stage, src + (size_t)z0 * plane, (size_t)nz * plane, hipMemcpyDeviceToHost, cst);
            if (e == hipSuccess) e = hipStreamSynchronize(cst);
            if (e != hipSuccess) break;
            for (int32_t z = 0; z < nz; ++z)
                for (int32_t y = 0; y < B.ey; ++y) {
                    const int64_t k = ch.o[2] + z0 + z + 1, j = ch.o[1] + y + 1, i = ch.o[0] + 1;
                    std::memcpy(host.data() + (size_t)((k * P + j) * P + i) * s,
                                stage + (size_t)z * plane + (size_t)y * B.py * s, row);
                }
        }
    }
    std::lock_guard<std::mutex> lk(mu);
    R.iters = fs;
    R.residual = r;
    if (e == hipSuccess) {
        R.result.swap(host);
        R.state = OD_REQ_DONE;
    } else {
        R.state = OD_REQ_CANCELED;
        if (fatal.empty()) fatal = std::string("result copy: ") + hipGetErrorString(e);
    }
    slot_ticket[(size_t)R.slot] = 0;
    release(R.off, R.bytes);
    R.grid.reset();
}

void Server::run() {
    const int64_t wait_ticks = device_wait_ticks(20.0);
    const int64_t yield_poll_ticks = device_wait_ticks(20e-6);   // host flag polled every 20 us
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = "event creation failed";
        return;
    }
    std::vector<int32_t> list;
    for (;;) {
        std::vector<Request*> admitted;
        const double t_wait = now_s();
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || worker_has_work(); });
            if (stop) break;
            stats.idle_s += now_s() - t_wait;
            // FIFO admission while a slot and arena space are free
            while (!queue.empty()) {
                Request& R = *reqs[queue.front()];
                const int32_t slot = free_slot();
                if (slot < 0) break;
                const size_t off = alloc(R.bytes);
                if (off == SIZE_MAX) break;
                queue.pop_front();
                R.off = off;
                R.slot = slot;
                slot_ticket[(size_t)slot] = R.ticket;
                admitted.push_back(&R);
            }
        }
        const double t_admit0 = now_s();
        for (Request* R : admitted) {
            od_status s = setup_slot(*R, R->slot);
            std::lock_guard<std::mutex> lk(mu);
            if (s == OD_OK) {
                R->state = OD_REQ_RUNNING;
                R->t_admit = now_s();
            } else {
                R->state = OD_REQ_CANCELED;
                slot_ticket[(size_t)R->slot] = 0;
                release(R->off, R->bytes);
                R->grid.reset();
            }
        }
        // one scheduling epoch over every resident, unfinished solve
        std::vector<Request*> active;
        list.clear();
        {
            std::lock_guard<std::mutex> lk(mu);
            stats.admit_s += now_s() - t_admit0;
            for (int32_t s2 = 0; s2 < max_slots; ++s2) {
                const uint64_t t = slot_ticket[(size_t)s2];
                if (!t) continue;
                Request& R = *reqs[t];
                if (R.state != OD_REQ_RUNNING || R.finished) continue;
                active.push_back(&R);
                const int32_t nt = (int32_t)R.grid->tiles_h.size();
                for (int32_t i = 0; i < nt; ++i) list.push_back(s2 * kTileStride + i);
                // keep every solve's XCD groups aligned to launch positions mod 8
                while (list.size() % kNumXcd) list.push_back(-1);
            }
        }
        hipError_t e = hipSuccess;
        bool launched = false;
        double t_epoch = now_s();
        std::vector<char> seen(active.size(), 0);
        if (!active.empty()) {
        // tile list: solves back to back, each padded (-1) to a multiple of
        // 8 entries; each solve's tiles keep their own XCD-interleaved order,
        // so a solve's XCD groups stay together
        e = hipMemcpyAsync(arena + c_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, st);
        // launch position of every listed tile and of every listed solve's
        // first tile, filled on the device (the kernel reads them only for
        // the tiles of the list)
        if (e == hipSuccess)
            e = launch_serve_positions(st, reinterpret_cast<const int32_t*>(arena + c_list), (int32_t)list.size(),
                                       kTileStride, reinterpret_cast<int32_t*>(arena + c_tpos),
                                       reinterpret_cast<int32_t*>(arena + c_sbase));
        __atomic_store_n(h_yield, 0, __ATOMIC_RELEASE);
        if (e == hipSuccess) e = hipMemsetAsync(arena + c_yield, 0, 4, st);
        MsgArgs a{};
        a.tile_list = reinterpret_cast<const int32_t*>(arena + c_list);
        a.solve_dtype = reinterpret_cast<const int32_t*>(arena + c_dtype);
        a.arena = arena;
        a.blocks = reinterpret_cast<const BlockDev*>(arena + c_blocks);
        a.tiles = reinterpret_cast<const TileDev*>(arena + c_tiles);
        a.ntiles = (int32_t)list.size();
        a.dep_ptr = reinterpret_cast<const int32_t*>(arena + c_dep_ptr);
        a.dep_idx = reinterpret_cast<const int32_t*>(arena + c_dep_idx);
        a.done = reinterpret_cast<int32_t*>(arena + c_done);
        a.target = reinterpret_cast<const int32_t*>(arena + c_target);
        a.tile_solve = reinterpret_cast<const int32_t*>(arena + c_tile_solve);
        a.res = reinterpret_cast<unsigned long long*>(arena + c_res);
        a.err = reinterpret_cast<unsigned int*>(arena + c_err);
        a.wait_ticks = wait_ticks;
        a.solve_count = reinterpret_cast<int32_t*>(arena + c_count);
        a.gate = reinterpret_cast<int32_t*>(arena + c_gate);
        a.solve_ntiles = reinterpret_cast<const int32_t*>(arena + c_ntiles);
        a.check_every = reinterpret_cast<const int32_t*>(arena + c_ce);
        a.tol = reinterpret_cast<const double*>(arena + c_tol);
        a.final_step = reinterpret_cast<int32_t*>(arena + c_final);
        a.host_done = h_done;
        a.host_res = h_res;
        a.yield_flag = h_yield;
        a.yield_dev = reinterpret_cast<int32_t*>(arena + c_yield);
        a.yield_poll_ticks = yield_poll_ticks;
        a.xpub = reinterpret_cast<uint8_t*>(arena + c_xpub);
        a.tile_pos = reinterpret_cast<const int32_t*>(arena + c_tpos);
        a.solve_base = reinterpret_cast<const int32_t*>(arena + c_sbase);
        a.nlive = (int32_t)active.size();
        a.bar = reinterpret_cast<unsigned int*>(arena + c_bar);
        a.pend = reinterpret_cast<int32_t*>(arena + c_pend);
        a.qslots = reinterpret_cast<unsigned long long*>(arena + c_qslots);
        a.pslots = a.qslots + (2 * list.size() + 8);
        a.ready = reinterpret_cast<int32_t*>(a.qslots);   // cursor mode: ready words in the ready-queue region
        a.qhead = reinterpret_cast<unsigned int*>(arena + c_qctl);
        a.hints = hints.load() & kHintCheck;
        a.seed = check_seed.load();
        a.pert_ticks = (a.hints & kHintCheck) ? device_wait_ticks(20e-6) : 0;
        int grid = std::min<int>(grid_cap, (int)list.size());
        if (grid >= kNumXcd) grid -= grid % kNumXcd;
        if (e == hipSuccess) e = launch_queue_init(st, a);
        t_epoch = now_s();
        if (e == hipSuccess) e = launch_serve(st, grid, a);
        if (e == hipSuccess) e = hipEventRecord(ev, st);
        launched = e == hipSuccess;
        }
        if (!launched && e == hipSuccess) continue;
        while (e == hipSuccess) {
            const hipError_t q = hipEventQuery(ev);
            const double t = now_s();
            bool finished_any = false;
            {
                std::lock_guard<std::mutex> lk(mu);
                for (size_t i = 0; i < active.size(); ++i) {
                    if (!seen[i] && __atomic_load_n(&h_done[active[i]->slot], __ATOMIC_ACQUIRE) > 0) {
                        seen[i] = 1;
                        active[i]->t_done = t;
                    }
                    finished_any |= seen[i] != 0;
                }
                bool want_admit = false;
                if (!queue.empty()) {
                    const Request& H = *reqs[queue.front()];
                    want_admit = free_slot() >= 0 && fits_somewhere(H.bytes);
                }
                const double age = t - t_epoch;
                // a launch also ends every few seconds, which bounds its
                // queue tickets and finish counters (rebuilt at the next start)
                if ((want_admit && age > 1e-3) || (finished_any && age > 2e-3) || age > 4.0 || stop)
                    __atomic_store_n(h_yield, 1, __ATOMIC_RELEASE);
            }
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) {
                e = q;
                break;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            stats.epochs += 1;
            stats.epoch_s += now_s() - t_epoch;
        }
        unsigned int derr = 0;
        if (e == hipSuccess) e = hipMemcpy(&derr, arena + c_err, 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess || derr != 0) {
            std::lock_guard<std::mutex> lk(mu);
            fatal = e != hipSuccess ? std::string("serving epoch: ") + hipGetErrorString(e)
                    : (derr & kErrSchedule) ? "serving epoch: schedule check failed (a tile's step counter did not "
                                              "advance by one, or a tile ran while a neighbour was not within one step)"
                                            : "serving epoch: a device-side wait exceeded its bound";
            for (Request* R : active) {
                R->state = OD_REQ_CANCELED;
                slot_ticket[(size_t)R->slot] = 0;
                release(R->off, R->bytes);
                R->grid.reset();
            }
            break;
        }
        // finished solves go to the retire thread (their chares are in no
        // later tile list)
        for (size_t i = 0; i < active.size(); ++i)
            if (__atomic_load_n(&h_done[active[i]->slot], __ATOMIC_ACQUIRE) > 0) {
                std::lock_guard<std::mutex> lk(mu);
                if (!seen[i]) active[i]->t_done = now_s();
                active[i]->finished = true;
                retire_q.push_back(active[i]);
                rcv.notify_one();
            }
    }
    hipEventDestroy(ev);
    cancel_unfinished();
}

// Retire thread: copy out finished solves in completion order; each freed
// slot and arena range may let the worker admit the next request.
void Server::retire_run() {
    for (;;) {
        Request* R = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            rcv.wait(lk, [&] { return retire_stop || !retire_q.empty(); });
            if (retire_q.empty()) return;   // asked to stop, nothing left
            R = retire_q.front();
            retire_q.pop_front();
        }
        const double t0 = now_s();
        retire(*R);
        std::lock_guard<std::mutex> lk(mu);
        stats.retire_s += now_s() - t0;
        cv.notify_all();
    }
}

// Cancel every request that is queued or still running (finished solves
// belong to the retire thread, which completes or cancels them itself).
void Server::cancel_unfinished() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : reqs) {
        Request& R = *kv.second;
        if (R.finished) continue;
        if (R.state == OD_REQ_QUEUED || R.state == OD_REQ_RUNNING) R.state = OD_REQ_CANCELED;
        if (R.grid) {
            R.grid.reset();
            if (R.slot >= 0) slot_ticket[(size_t)R.slot] = 0;
        }
    }
    queue.clear();
}

// Byte layout of the control region for max_slots slots; returns its size.
size_t control_layout(Server& S, int32_t max_slots) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = align_up(o, kAlign);
        o = r + std::max<size_t>(bytes, 1);
        return r;
    };
    const size_t ms = (size_t)max_slots;
    S.c_blocks = take(ms * kMaxBlocks * sizeof(BlockDev));
    S.c_tiles = take(ms * kTileStride * sizeof(TileDev));
    S.c_done = take(ms * kTileStride * 4);
    S.c_tile_solve = take(ms * kTileStride * 4);
    S.c_dep_ptr = take(ms * kTileStride * 4);
    S.c_dep_idx = take(ms * kMaxDeps * 4);
    S.c_target = take(ms * 4);
    S.c_final = take(ms * 4);
    S.c_gate = take(ms * 4);
    S.c_count = take(ms * 4);
    S.c_res = take(ms * 8);
    S.c_ce = take(ms * 4);
    S.c_tol = take(ms * 8);
    S.c_ntiles = take(ms * 4);
    S.c_dtype = take(ms * 4);
    S.c_list = take(ms * (kTileStride + kNumXcd) * 4);
    S.c_err = take(16);
    S.c_yield = take(16);
    S.c_xpub = take(ms * (kTileStride + kNumXcd));
    S.c_sbase = take(ms * 4);
    S.c_pend = take(ms * kTileStride * 2 * 4);
    // ready queues, then cross lists: 2 * positions + 8 slots each
    S.c_qslots = take(2 * (2 * ms * (kTileStride + kNumXcd) + 8) * 8);
    S.c_qctl = take(64 * 4);
    S.c_tpos = take(ms * kTileStride * 4);
    S.c_bar = take(16);
    S.data_begin = align_up(o, kAlign);
    return S.data_begin;
}

}  // namespace od

struct od_server {
    od::Server s;
};

using od::fail;

namespace {

od_status validate_request(const od_request* r) {
    if (!r) return fail(OD_EINVAL, "request is NULL");
    if (r->n < 1 || r->n > 1024) return fail(OD_EINVAL, "request n must be in [1, 1024]");
    if (r->dtype != OD_F32 && r->dtype != OD_F64) return fail(OD_EINVAL, "request dtype must be OD_F32 or OD_F64");
    if (r->odf < 1) return fail(OD_EINVAL, "request odf must be >= 1");
    if (r->max_iters < 1 || r->max_iters > INT32_MAX) return fail(OD_EINVAL, "request max_iters must be in [1, 2^31)");
    if (r->check_every < 0) return fail(OD_EINVAL, "request check_every must be >= 0");
    if (!(r->t_arrival >= 0.0)) return fail(OD_EINVAL, "request t_arrival must be >= 0 (0 = submit time)");
    return OD_OK;
}

// Plan of a request: its grid (host side) and the arena bytes it needs.
od_status plan_request(const od_request* r, std::unique_ptr<od::Grid>& G) {
    od_status s = validate_request(r);
    if (s != OD_OK) return s;
    G.reset(new od::Grid);
    const od_config cfg = od::request_config(*r);
    std::string err = od::build_layout(cfg, *G);
    if (!err.empty()) return fail(OD_EINVAL, err);
    if (G->tiles_h.size() > (size_t)od::kMaxTiles || G->blocks_h.size() > (size_t)od::kMaxBlocks ||
        G->dep_idx.size() > (size_t)od::kMaxDeps)
        return fail(OD_EINVAL, "request too large for a serving slot (tiles/blocks/dependencies)");
    return OD_OK;
}

}  // namespace

extern "C" {

od_status od_server_control_bytes(int32_t max_slots, size_t* bytes) {
    if (!bytes || max_slots < 1 || max_slots > 4096) return fail(OD_EINVAL, "need bytes and max_slots in [1, 4096]");
    od::Server S;
    *bytes = od::control_layout(S, max_slots);
    return OD_OK;
}

od_status od_request_bytes(const od_request* req, size_t* bytes) {
    try {
        if (!bytes) return fail(OD_EINVAL, "bytes is NULL");
        std::unique_ptr<od::Grid> G;
        od_status s = plan_request(req, G);
        if (s != OD_OK) return s;
        *bytes = od::align_up(G->L.total, od::kAlign);
        return OD_OK;
    } catch (...) {
        return fail(OD_EINVAL, "internal error");
    }
}

od_status od_server_create(void* hip_stream, void* dev_arena, size_t arena_bytes, int32_t max_slots,
                           od_server** out) {
    try {
        if (!out) return fail(OD_EINVAL, "out is NULL");
        *out = nullptr;
        if (!dev_arena || reinterpret_cast<uintptr_t>(dev_arena) % od::kAlign != 0)
            return fail(OD_EINVAL, "arena must be non-NULL and 256-byte aligned");
        if (max_slots < 1 || max_slots > 4096) return fail(OD_EINVAL, "max_slots must be in [1, 4096]");
        std::unique_ptr<od_server> h(new od_server);
        od::Server& S = h->s;
        S.st = static_cast<hipStream_t>(hip_stream);
        S.arena = static_cast<char*>(dev_arena);
        S.arena_bytes = arena_bytes;
        S.max_slots = max_slots;
        const size_t ms = (size_t)max_slots;
        od::control_layout(S, max_slots);
        if (S.data_begin >= arena_bytes)
            return fail(OD_ENOMEM, "arena of " + std::to_string(arena_bytes) + " bytes cannot hold the " +
                                       std::to_string(S.data_begin) + "-byte control region for " +
                                       std::to_string(max_slots) + " slots");
        S.free_list[S.data_begin] = arena_bytes - S.data_begin;
        S.slot_ticket.assign(ms, 0);
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&S.h_done), ms * 4, hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S.h_res), ms * 8, hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S.h_yield), 64, hipHostMallocCoherent);
        // staging for result copies: the largest plane chunk od_read uses
        S.staging_bytes = (size_t)64 << 20;
        if (e == hipSuccess) e = hipHostMalloc(&S.staging, S.staging_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.cst, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMemsetAsync(S.arena + S.c_err, 0, 16, S.st);
        if (e == hipSuccess) e = hipMemsetAsync(S.arena + S.c_bar, 0, 16, S.st);
        if (e == hipSuccess) e = hipStreamSynchronize(S.st);
        if (e != hipSuccess) {
            if (S.h_done) hipHostFree(S.h_done);
            if (S.h_res) hipHostFree(S.h_res);
            if (S.h_yield) hipHostFree(S.h_yield);
            if (S.staging) hipHostFree(S.staging);
            if (S.cst) hipStreamDestroy(S.cst);
            return fail(OD_EHIP, std::string("server setup: ") + hipGetErrorString(e));
        }
        std::memset(S.h_done, 0, ms * 4);
        std::memset(S.h_res, 0, ms * 8);
        *S.h_yield = 0;
        S.grid_cap = od::serve_max_grid();
        if (S.grid_cap <= 0) {
            hipHostFree(S.h_done);
            hipHostFree(S.h_res);
            hipHostFree(S.h_yield);
            hipHostFree(S.staging);
            hipStreamDestroy(S.cst);
            return fail(OD_EHIP, "no co-resident workgroups for the serving kernel");
        }
        S.retirer = std::thread([&S] { S.retire_run(); });
        S.worker = std::thread([&S] { S.run(); });
        *out = h.release();
        return OD_OK;
    } catch (const std::exception& ex) {
        return fail(OD_EINVAL, std::string("internal error: ") + ex.what());
    }
}

od_status od_submit(od_server* sv, const od_request* req, uint64_t* ticket) {
    try {
        if (!sv || !ticket) return fail(OD_EINVAL, "NULL argument");
        std::unique_ptr<od::Grid> G;
        od_status s = plan_request(req, G);
        if (s != OD_OK) return s;
        od::Server& S = sv->s;
        const size_t bytes = od::align_up(G->L.total, od::kAlign);
        std::unique_ptr<od::Request> R(new od::Request);
        R->req = *req;
        R->bytes = bytes;
        R->grid = std::move(G);
        R->t_submit = od::now_s();
        R->t_arrival = req->t_arrival > 0.0 ? req->t_arrival : R->t_submit;
        if (R->t_arrival > R->t_submit)
            return fail(OD_EINVAL, "request t_arrival lies in the future of the monotonic clock");
        std::lock_guard<std::mutex> lk(S.mu);
        if (!S.fatal.empty()) return fail(OD_ECANCELED, S.fatal);
        if (bytes > S.arena_bytes - S.data_begin)
            return fail(OD_ENOMEM, "request needs " + std::to_string(bytes) + " bytes; the arena holds " +
                                       std::to_string(S.arena_bytes - S.data_begin));
        if (S.queue.size() >= od::kMaxQueue) return fail(OD_EAGAIN, "submission queue full");
        R->ticket = S.next_ticket++;
        *ticket = R->ticket;
        S.queue.push_back(R->ticket);
        S.reqs[R->ticket] = std::move(R);
        S.cv.notify_all();
        return OD_OK;
    } catch (const std::bad_alloc&) {
        return fail(OD_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(OD_EINVAL, "internal error");
    }
}

od_status od_server_set_hints(od_server* sv, int32_t hints, uint64_t seed) {
    if (!sv) return fail(OD_EINVAL, "server is NULL");
    if (hints & ~od::kHintCheck) return fail(OD_EINVAL, "serving hints: only bit 2 (schedule check) is defined");
    sv->s.check_seed.store(seed);
    sv->s.hints.store(hints);
    return OD_OK;
}

od_status od_server_step(od_server* sv, int32_t* active, int32_t* queued) {
    if (!sv) return fail(OD_EINVAL, "server is NULL");
    od::Server& S = sv->s;
    std::lock_guard<std::mutex> lk(S.mu);
    int32_t a = 0;
    for (uint64_t t : S.slot_ticket) a += t ? 1 : 0;
    if (active) *active = a;
    if (queued) *queued = (int32_t)S.queue.size();
    if (!S.fatal.empty()) return fail(OD_ECANCELED, S.fatal);
    return OD_OK;
}

od_status od_server_stats_get(od_server* sv, od_server_stats* out) {
    if (!sv || !out) return fail(OD_EINVAL, "NULL argument");
    od::Server& S = sv->s;
    std::lock_guard<std::mutex> lk(S.mu);
    *out = S.stats;
    return OD_OK;
}

od_status od_poll(od_server* sv, uint64_t ticket, od_info* out) {
    if (!sv || !out) return fail(OD_EINVAL, "NULL argument");
    od::Server& S = sv->s;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(OD_EINVAL, "unknown ticket " + std::to_string(ticket));
    const od::Request& R = *it->second;
    out->state = R.state;
    out->iters = R.iters;
    out->residual = R.residual;
    out->t_submit = R.t_submit;
    out->t_admit = R.t_admit;
    out->t_done = R.t_done;
    out->t_arrival = R.t_arrival;
    if (R.state == OD_REQ_DONE) return OD_OK;
    if (R.state == OD_REQ_CANCELED) return fail(OD_ECANCELED, S.fatal.empty() ? "request cancelled" : S.fatal);
    return OD_ENOTREADY;
}

od_status od_fetch(od_server* sv, uint64_t ticket, void* host_dst, size_t bytes) {
    if (!sv || !host_dst) return fail(OD_EINVAL, "NULL argument");
    od::Server& S = sv->s;
    std::unique_ptr<od::Request> R;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        auto it = S.reqs.find(ticket);
        if (it == S.reqs.end()) return fail(OD_EINVAL, "unknown ticket " + std::to_string(ticket));
        const od::Request& Q = *it->second;
        if (Q.state == OD_REQ_CANCELED) return fail(OD_ECANCELED, "request cancelled");
        if (Q.state != OD_REQ_DONE) return fail(OD_ENOTREADY, "request not finished");
        if (bytes < Q.result.size())
            return fail(OD_EINVAL, "buffer of " + std::to_string(bytes) + " bytes, need " + std::to_string(Q.result.size()));
        R = std::move(it->second);
        S.reqs.erase(it);
    }
    // the (possibly large) copy runs without the server lock held
    std::memcpy(host_dst, R->result.data(), R->result.size());
    return OD_OK;
}

od_status od_server_destroy(od_server* sv) {
    if (!sv) return OD_OK;
    od::Server& S = sv->s;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
        if (S.h_yield) __atomic_store_n(S.h_yield, 1, __ATOMIC_RELEASE);
        S.cv.notify_all();
    }
    if (S.worker.joinable()) S.worker.join();
    // the retire thread finishes the solves already handed to it, then stops
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.retire_stop = true;
        S.rcv.notify_all();
    }
    if (S.retirer.joinable()) S.retirer.join();
    hipError_t e = hipStreamSynchronize(S.st);
    if (S.cst) {
        const hipError_t e2 = hipStreamSynchronize(S.cst);
        if (e == hipSuccess) e = e2;
        hipStreamDestroy(S.cst);
    }
    if (S.h_done) hipHostFree(S.h_done);
    if (S.h_res) hipHostFree(S.h_res);
    if (S.h_yield) hipHostFree(S.h_yield);
    if (S.staging) hipHostFree(S.staging);
    delete sv;
    if (e != hipSuccess) return fail(OD_EHIP, std::string("server destroy: ") + hipGetErrorString(e));
    return OD_OK;
}

}  // extern "C"
