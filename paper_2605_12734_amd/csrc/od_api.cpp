// libod runtime: the C ABI of include/od.h for one grid.
//
// od_create decomposes the grid into chares (regular split or explicit
// uneven blocks), cuts chares into sweep tiles, builds every tile face's
// halo source (the pre-filled location table of Section IV: each ghost slab
// knows which chare, or which Dirichlet face, it is read from), carves the
// caller's workspace, uploads the descriptors once and initialises the
// field on the device.  od_iterate then only enqueues device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "od_runtime.hpp"

namespace od {

thread_local std::string g_last_error;

od_status fail(od_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

uint64_t host_sm64(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

namespace {

constexpr int kStreamPool = 16;          // per-chare baseline: non-blocking streams
constexpr int64_t kMaxGraphLen = 1024;   // iterations per captured graph

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = align_up(off, kAlign);
        off = o + std::max<size_t>(bytes, 1);
        return o;
    }
};

int32_t pitch_of(int32_t ex, int s) {
    const int32_t q = 64 / s;   // 64-byte rows
    return (int32_t)align_up((size_t)ex, (size_t)q);
}

// Face f of chare c: pseudo-block extents, pitches, element count.
void face_shape(const Chare& c, int32_t cpy, int f, int32_t e[3], int32_t* py, int64_t* pz, int64_t* cnt) {
    const int d = f / 2;
    e[0] = c.e[0];
    e[1] = c.e[1];
    e[2] = c.e[2];
    e[d] = 1;
    if (d == 0) {
        *py = 1;
        *pz = c.e[1];
        *cnt = (int64_t)c.e[1] * c.e[2];
    } else if (d == 1) {
        // rows of the y faces keep the chare's (aligned) row pitch so the
        // sweep can load them as 16-byte vectors
        *py = cpy;
        *pz = cpy;
        *cnt = (int64_t)cpy * c.e[2];
    } else {
        *py = cpy;
        *pz = (int64_t)cpy * c.e[1];
        *cnt = (int64_t)cpy * c.e[1];
    }
}

bool on_domain_face(const Plan& p, const Chare& c, int f) {
    const int d = f / 2;
    return (f % 2 == 0) ? c.u[d] == 0 : (int64_t)c.u[d] + (int64_t)c.e[d] * c.h == p.n[d];
}

int32_t log2i(int32_t v) {
    int32_t l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Ghost-fill rectangles of every resolution-change face: one per (face,
// neighbour chare), found by walking the face's unit slab at the owner
// grid's granularity.  Returns the number of neighbour cells the fill reads,
// or -1 if a face has a neighbour more than 16 times finer (the largest
// ratio the fill is built and tested for: 256 source values per ghost cell).
int64_t build_fill_segments(Grid& G) {
    const Plan& p = G.plan;
    G.segs_h.clear();
    G.fill_total = 0;
    int64_t reads = 0;
    const int64_t g = p.gran;
    for (int32_t ci = 0; ci < (int32_t)p.chares.size(); ++ci) {
        const Chare& c = p.chares[(size_t)ci];
        for (int f = 0; f < 6; ++f) {
            const int32_t pb = G.amr_pb[(size_t)ci * 6 + f];
            if (pb < 0) continue;
            const int d = f / 2, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            const int64_t nrm = (f % 2) ? (int64_t)c.u[d] + (int64_t)c.e[d] * c.h : (int64_t)c.u[d] - 1;
            int64_t lo[3], hi[3];
            for (int q = 0; q < 3; ++q) {
                lo[q] = c.u[q];
                hi[q] = (int64_t)c.u[q] + (int64_t)c.e[q] * c.h;
            }
            lo[d] = nrm;
            hi[d] = nrm + 1;
            std::vector<int32_t> seen;
            for (int64_t z = lo[2] / g * g; z < hi[2]; z += g)
                for (int64_t y = lo[1] / g * g; y < hi[1]; y += g)
                    for (int64_t x = lo[0] / g * g; x < hi[0]; x += g) {
                        const int32_t nb = plan_owner(p, std::max(x, lo[0]), std::max(y, lo[1]), std::max(z, lo[2]));
                        if (std::find(seen.begin(), seen.end(), nb) != seen.end()) continue;
                        seen.push_back(nb);
                        const Chare& N = p.chares[(size_t)nb];
                        int64_t a[3], b[3];
                        for (int q = 0; q < 3; ++q) {
                            a[q] = std::max<int64_t>(lo[q], N.u[q]);
                            b[q] = std::min<int64_t>(hi[q], (int64_t)N.u[q] + (int64_t)N.e[q] * N.h);
                        }
                        FillSeg S{};
                        S.dst = pb;
                        S.src = nb;
                        S.d = d;
                        S.lay = (int32_t)((nrm - N.u[d]) / N.h);
                        S.a1 = (int32_t)((a[t1] - c.u[t1]) / c.h);
                        S.a2 = (int32_t)((a[t2] - c.u[t2]) / c.h);
                        S.n1 = (int32_t)((b[t1] - a[t1]) / c.h);
                        S.n2 = (int32_t)((b[t2] - a[t2]) / c.h);
                        S.r1 = (int32_t)(a[t1] - N.u[t1]);
                        S.r2 = (int32_t)(a[t2] - N.u[t2]);
                        S.hc = c.h;
                        S.lhn = log2i(N.h);
                        S.first = G.fill_total;
                        S.eoff[0] = S.eoff[1] = -1;   // no export (set by build_layout)
                        const int64_t cells = (int64_t)S.n1 * S.n2;
                        G.fill_total += cells;
                        const int64_t r = N.h < c.h ? c.h / N.h : 1;
                        if (r > 16) return -1;
                        reads += cells * r * r;
                        G.segs_h.push_back(S);
                    }
        }
    }
    return reads;
}

}  // namespace

// ---- two steps per pass ------------------------------------------------------

namespace {

// Pairs of iterations in one pass need blocks at one resolution (every
// line of cells around a tile in one block: so in a regular decomposition;
// explicit blocks have their tiles split until it holds) and a tile shape
// with a two-step variant (3D tiles, or the 2D stencil's row tiles); the
// persistent form also the 3D stencil, the fixed-stride or counter
// schedule (with or without the guided tail) and no timeline; the
// message-driven form the 3D stencil.  Under load imbalance a heavy
// chare's extra runs are one-step sweeps before its pass (3D stencil only).
bool two_step_possible(const Grid& G) {
    const od_config& cfg = G.cfg;
    const Plan& p = G.plan;
    const bool form = cfg.exec == OD_FUSED || cfg.exec == OD_GRAPH ||
                      (cfg.exec == OD_PERSISTENT && cfg.stencil != 5 && G.sched() >= 1 && G.sched() <= 3 &&
                       !(cfg.hints & kHintTimeline)) ||
                      (cfg.exec == OD_MSGDRIVEN && cfg.stencil != 5);
    return form && !(cfg.hints & 4096) && !p.multires && (G.imb.heavy == 0 || cfg.stencil != 5);
}

// Room for two-step descriptors: the forms that can pair steps under any
// schedule the autotuner may choose.
bool two_step_room(const Grid& G) {
    const od_config& cfg = G.cfg;
    const Plan& p = G.plan;
    const bool form = cfg.exec == OD_FUSED || cfg.exec == OD_GRAPH ||
                      (cfg.exec == OD_PERSISTENT && cfg.stencil != 5 && !(cfg.hints & (kHintTimeline | 2048))) ||
                      (cfg.exec == OD_MSGDRIVEN && cfg.stencil != 5);
    const bool imbalance = cfg.imbalance_pct > 0 && cfg.imbalance_max_extra > 0;
    return form && !(cfg.hints & 4096) && !p.multires && (!imbalance || cfg.stencil != 5);
}

// Block and local coordinates of global cell (x, y, z) as a FaceDev: its
// chare, or for a cell of the domain's ghost shell the Dirichlet
// pseudo-block of that face (normal coordinate 0; every cell of it holds
// the face's value); `other` for a cell outside the domain along two or
// more axes (never read).
FaceDev cell_src(const Grid& G, int64_t x, int64_t y, int64_t z, const FaceDev& other) {
    const Plan& p = G.plan;
    int64_t v[3] = {x, y, z};
    int outs = 0, f = -1;
    for (int d = 0; d < 3; ++d) {
        if (v[d] < 0) {
            ++outs;
            f = 2 * d;
            v[d] = 0;
        } else if (v[d] >= p.n[d]) {
            ++outs;
            f = 2 * d + 1;
            v[d] = p.n[d] - 1;
        }
    }
    if (outs >= 2) return other;
    const int32_t c = plan_owner(p, v[0], v[1], v[2]);
    const Chare& ch = p.chares[(size_t)c];
    int32_t l[3];
    for (int d = 0; d < 3; ++d) l[d] = (int32_t)(v[d] - ch.u[d]);
    FaceDev out{};
    out.src = c;
    if (outs == 1) {
        out.src = G.dir_pb[(size_t)c * 6 + f];
        if (out.src < 0) return other;   // a face without a boundary buffer (the 2D grid's y faces): never read
        l[f / 2] = 0;
    }
    out.sx = l[0];
    out.sy = l[1];
    out.sz = l[2];
    return out;
}

void fill_tile2(const Grid& G, const TileHost& th, Tile2Dev& t2) {
    const Chare& ch = G.plan.chares[(size_t)th.chare];
    const int64_t X0 = (int64_t)ch.u[0] + th.o[0], Y0 = (int64_t)ch.u[1] + th.o[1], Z0 = (int64_t)ch.u[2] + th.o[2];
    const int64_t nx = th.e[0], ny = th.e[1], nz = th.e[2];
    const FaceDev own{th.chare, th.o[0], th.o[1], th.o[2]};
    t2 = Tile2Dev{};
    for (int f = 0; f < 6; ++f)
        if (th.kind[f] == 1) t2.dir |= 1 << f;
    const int64_t xs[2] = {X0 - 1, X0 + nx}, ys[2] = {Y0 - 1, Y0 + ny}, zs[2] = {Z0 - 1, Z0 + nz};
    for (int k = 0; k < 4; ++k) {
        t2.e[k] = cell_src(G, xs[k & 1], ys[k >> 1], Z0, own);
        t2.e[4 + k] = cell_src(G, xs[k & 1], Y0, zs[k >> 1], own);
        t2.e[8 + k] = cell_src(G, X0, ys[k & 1], zs[k >> 1], own);
    }
    t2.r2[0] = cell_src(G, X0 - 2, Y0, Z0, own);
    t2.r2[1] = cell_src(G, X0 + nx + 1, Y0, Z0, own);
    t2.r2[2] = cell_src(G, X0, Y0 - 2, Z0, own);
    t2.r2[3] = cell_src(G, X0, Y0 + ny + 1, Z0, own);
    t2.r2[4] = cell_src(G, X0, Y0, Z0 - 2, own);
    t2.r2[5] = cell_src(G, X0, Y0, Z0 + nz + 1, own);
}

// Cells of other chares within two stencil steps of each chare (L1
// distance <= 2, inside the domain): each face's two layers and the cells
// diagonal to each edge, summed over the chares.
int64_t halo2_count(const Plan& p) {
    int64_t g = 0;
    for (const Chare& c : p.chares) {
        auto inside = [&](int d, int64_t v) { return v >= 0 && v < p.n[d]; };
        int64_t r1[6];
        for (int f = 0; f < 6; ++f) {
            const int d = f / 2;
            const int64_t area = (int64_t)c.e[(d + 1) % 3] * c.e[(d + 2) % 3];
            r1[f] = (f % 2) ? (int64_t)c.u[d] + c.e[d] : (int64_t)c.u[d] - 1;
            const int64_t r2 = (f % 2) ? r1[f] + 1 : r1[f] - 1;
            if (inside(d, r1[f])) g += area;
            if (inside(d, r2)) g += area;
        }
        for (int d1 = 0; d1 < 3; ++d1)
            for (int d2 = d1 + 1; d2 < 3; ++d2)
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        if (inside(d1, r1[2 * d1 + a]) && inside(d2, r1[2 * d2 + b])) g += c.e[3 - d1 - d2];
    }
    return g;
}

}  // namespace

int64_t Grid::bytes_per_pass() const {
    return two_step ? (int64_t)s * (2 * plan.interior + halo2_cells) : (int64_t)s * (2 * plan.interior + plan.halo_cells);
}

// Device descriptors of every tile: owning chare, box, and for each face
// the block (chare or face pseudo-block) its ghost slab is read from.
std::string fill_tile_descs(Grid& G) {
    const Plan& p = G.plan;
    const od_config& cfg = G.cfg;
    const size_t ntiles = p.tiles.size();
    G.tiles_h.resize(ntiles);
    for (size_t i = 0; i < ntiles; ++i) {
        const TileHost& th = p.tiles[i];
        TileDev& td = G.tiles_h[i];
        const Chare& ch = p.chares[(size_t)th.chare];
        td.blk = th.chare;
        td.x0 = th.o[0];
        td.y0 = th.o[1];
        td.z0 = th.o[2];
        td.nx = th.e[0];
        td.ny = th.e[1];
        td.nz = th.e[2];
        td.rslot = cfg.exec == OD_PER_CHARE ? th.chare : 0;
        for (int f = 0; f < 6; ++f) {
            FaceDev& fd = td.f[f];
            if (cfg.stencil == 5 && f / 2 == 1) {
                // 2D stencil: the y ghost "slab" is the tile's own row (never used)
                fd.src = th.chare;
                fd.sx = th.o[0];
                fd.sy = th.o[1];
                fd.sz = th.o[2];
                continue;
            }
            int32_t src_chare = -1, pb = -1;
            if (th.kind[f] == 2) src_chare = th.chare;
            else if (th.kind[f] == 0) {
                if (cfg.exec == OD_PER_CHARE) pb = G.ghost_pb[(size_t)th.chare * 6 + f];
                else src_chare = th.src[f];
            } else if (th.kind[f] == 3) {
                pb = G.amr_pb[(size_t)th.chare * 6 + f];
            } else {
                pb = G.dir_pb[(size_t)th.chare * 6 + f];
            }
            if (src_chare >= 0) {
                const Chare& sc = p.chares[(size_t)src_chare];
                fd.src = src_chare;
                fd.sx = th.g[f][0] - sc.o[0];
                fd.sy = th.g[f][1] - sc.o[1];
                fd.sz = th.g[f][2] - sc.o[2];
            } else {
                if (pb < 0) return "internal error: missing face pseudo-block";
                fd.src = pb;
                int32_t sxyz[3];
                for (int q = 0; q < 3; ++q) sxyz[q] = th.g[f][q] - ch.o[q];
                sxyz[f / 2] = 0;
                fd.sx = sxyz[0];
                fd.sy = sxyz[1];
                fd.sz = sxyz[2];
            }
        }
    }
    decide_two_step(G);
    return "";
}

// Pair steps where the grid's form, schedule and tile allow it; the tiles'
// line descriptors follow the tile list.
void decide_two_step(Grid& G) {
    const Plan& p = G.plan;
    G.two_step = two_step_possible(G) && sweep2_variant_ok(G.s, p.tile[0], p.tile[1], G.cfg.stencil == 5) &&
                 p.tiles.size() <= G.tile2_cap;
    G.tiles2_h.clear();
    if (G.two_step) {
        G.tiles2_h.resize(p.tiles.size());
        for (size_t i = 0; i < p.tiles.size(); ++i) fill_tile2(G, p.tiles[i], G.tiles2_h[i]);
    }
}

// ---------------------------------------------------------------------------
// layout: everything od_create needs, computed identically by
// od_workspace_bytes.

std::string build_layout(const od_config& cfg, Grid& G) {
    G.cfg = cfg;
    G.cfg.blocks = nullptr;   // the caller's array is not kept
    G.s = (int)cfg.dtype;
    Plan& p = G.plan;
    std::string err = plan_decompose(cfg, p);
    if (!err.empty()) return err;
    if (cfg.exec < OD_PER_CHARE || cfg.exec > OD_MSGDRIVEN) return "unknown exec mode";
    if (cfg.exec == OD_PER_CHARE && !p.regular) return "OD_PER_CHARE needs a regular decomposition";
    if (cfg.imbalance_pct < 0 || cfg.imbalance_pct > 100 || cfg.imbalance_max_extra < 0 ||
        cfg.imbalance_max_extra > 255)
        return "imbalance_pct must be in [0,100] and imbalance_max_extra in [0,255]";
    if (!(cfg.wait_s >= 0.0) || cfg.wait_s > 3600.0) return "wait_s must be in [0, 3600] seconds";
    if (cfg.imbalance_pct > 0 && cfg.exec == OD_GRAPH) return "imbalance is not supported with OD_GRAPH";
    if (p.multires && cfg.exec != OD_FUSED && cfg.exec != OD_GRAPH && cfg.exec != OD_PERSISTENT)
        return "multi-resolution blocks are supported with OD_FUSED, OD_GRAPH and OD_PERSISTENT";
    if (p.multires && cfg.exec == OD_PERSISTENT &&
        ((cfg.hints & (kHintTimeline | 32 | 2048 | 8192)) || (cfg.imbalance_pct > 0 && cfg.imbalance_max_extra > 0)))
        return "persistent multi-resolution grids take tiles from counters: no timeline, forced schedule or "
               "imbalance";
    if (p.multires && cfg.stencil == 5) return "multi-resolution blocks need the 3D 7-point stencil";
    if (!p.regular) {
        // tile rows are loaded as 16-byte vectors: explicit blocks start on a
        // vector boundary along x
        const int32_t vx = 16 / (int32_t)cfg.dtype;
        for (const Chare& c : p.chares)
            if (c.o[0] % vx != 0)
                return "explicit block x-origins must be multiples of " + std::to_string(vx) + " for this dtype";
    }
    plan_default_tile(cfg, p);
    p.xcd_order = (cfg.hints & 2) == 0;
    // message-driven tiles publish to other XCDs only across group
    // boundaries: compact boxes keep that boundary small
    p.xcd_boxes = cfg.exec == OD_MSGDRIVEN;
    // with per-chare load imbalance and few chares, compact boxes would give
    // each XCD whole chares and the heavy chare's XCD its extra sweeps
    // alone; below 512 chares (measured gains at ODF 8 and 64) every chare
    // is cut into 8 boxes instead, one per XCD group
#ifndef OD_SPLIT_CHARES_BELOW
#define OD_SPLIT_CHARES_BELOW 512
#endif
    p.xcd_split_chares = p.xcd_boxes && cfg.imbalance_pct > 0 && p.chares.size() < (size_t)OD_SPLIT_CHARES_BELOW;
    if (!sweep_variant_ok(G.s, p.tile[0], p.tile[1]))
        return "tile (" + std::to_string(p.tile[0]) + "," + std::to_string(p.tile[1]) + ") is not a compiled variant";
    p.two_step_lines = !p.regular && two_step_room(G);
    err = plan_tiles(p);
    if (!err.empty()) return err;
    if (cfg.exec == OD_PER_CHARE) {
        // chare-major tile order: one launch per chare covers a contiguous range
        std::stable_sort(p.tiles.begin(), p.tiles.end(),
                         [](const TileHost& a, const TileHost& b) { return a.chare < b.chare; });
    }
    const int32_t C = (int32_t)p.chares.size();
    const int s = G.s;

    // ---- block table: chares, then pseudo-blocks
    Carver cv;
    G.blocks_h.assign((size_t)C, BlockDev{});
    G.cpy.assign((size_t)C, 0);
    std::vector<size_t> field_off(2 * (size_t)C);
    G.dir_pb.assign((size_t)C * 6, -1);
    G.ghost_pb.assign((size_t)C * 6, -1);
    G.pb_face.clear();
    G.pb_block.clear();

    // field storage first (chares, face pseudo-blocks, per-chare messages),
    // then the control regions (descriptors and state), so the control part
    // can be placed apart from the field storage.
    // The 2D stencil never reads y neighbours: no y-face buffers (each would
    // be as large as the chare), y ghost slabs point at the tile itself
    const bool flat = cfg.stencil == 5;
    int32_t npb = 0;
    for (int32_t c = 0; c < C; ++c)
        for (int f = 0; f < 6; ++f) {
            if (flat && f / 2 == 1) continue;
            if (on_domain_face(p, p.chares[(size_t)c], f)) ++npb;
            else if (cfg.exec == OD_PER_CHARE) ++npb;
            else if (p.multires && p.mr[(size_t)c * 6 + f]) ++npb;
        }
    // load imbalance: drawn per step on the device (ImbDev)
    G.imb = ImbDev{};
    if (cfg.imbalance_pct > 0 && cfg.imbalance_max_extra > 0) {
        G.imb.seed = cfg.seed;
        G.imb.nchares = C;
        G.imb.heavy = (int32_t)std::llround(cfg.imbalance_pct / 100.0 * C);
        G.imb.maxe = cfg.imbalance_max_extra;
    }

    // ---- field storage (two parities per chare)
    for (int32_t c = 0; c < C; ++c) {
        const Chare& ch = p.chares[(size_t)c];
        const int32_t cpy = pitch_of(ch.e[0], s);
        G.cpy[(size_t)c] = cpy;
        const size_t bytes = (size_t)cpy * ch.e[1] * ch.e[2] * s;
        field_off[2 * (size_t)c] = cv.take(bytes);
        field_off[2 * (size_t)c + 1] = cv.take(bytes);
        BlockDev& B = G.blocks_h[(size_t)c];
        B.off[0] = (int64_t)(field_off[2 * (size_t)c] / s);
        B.off[1] = (int64_t)(field_off[2 * (size_t)c + 1] / s);
        B.py = cpy;
        B.pz = (int64_t)cpy * ch.e[1];
        B.ex = ch.e[0];
        B.ey = ch.e[1];
        B.ez = ch.e[2];
    }
    // ---- pseudo-blocks
    G.amr_pb.assign((size_t)C * 6, -1);
    for (int32_t c = 0; c < C; ++c) {
        const Chare& ch = p.chares[(size_t)c];
        for (int f = 0; f < 6; ++f) {
            if (flat && f / 2 == 1) continue;
            const bool dom = on_domain_face(p, ch, f);
            const bool res = !dom && p.multires && p.mr[(size_t)c * 6 + f];
            if (!dom && !res && cfg.exec != OD_PER_CHARE) continue;
            int32_t e[3], py;
            int64_t pz, cnt;
            face_shape(ch, G.cpy[(size_t)c], f, e, &py, &pz, &cnt);
            BlockDev B{};
            const size_t o = cv.take((size_t)cnt * s);
            B.off[0] = B.off[1] = (int64_t)(o / s);
            B.py = py;
            B.pz = pz;
            B.ex = e[0];
            B.ey = e[1];
            B.ez = e[2];
            const int32_t id = (int32_t)G.blocks_h.size();
            G.blocks_h.push_back(B);
            if (dom) {
                G.dir_pb[(size_t)c * 6 + f] = id;
                G.pb_face.push_back(f);
                G.pb_block.push_back(id);
            } else if (res) {
                G.amr_pb[(size_t)c * 6 + f] = id;
            } else {
                G.ghost_pb[(size_t)c * 6 + f] = id;
            }
        }
    }
    // ---- per-chare baseline messages: outbox (2 parities) and inbox per face
    G.msg.clear();
    if (cfg.exec == OD_PER_CHARE) {
        G.msg.resize((size_t)C);
        for (int32_t c = 0; c < C; ++c) {
            const Chare& ch = p.chares[(size_t)c];
            for (int f = 0; f < 6; ++f) {
                if (ch.nb[f] < 0) continue;
                int32_t e[3], py;
                int64_t pz, cnt;
                face_shape(ch, G.cpy[(size_t)c], f, e, &py, &pz, &cnt);
                G.msg[(size_t)c].cnt[f] = cnt;
                G.msg[(size_t)c].out[0][f] = cv.take((size_t)cnt * s);
                G.msg[(size_t)c].out[1][f] = cv.take((size_t)cnt * s);
                G.msg[(size_t)c].in[f] = cv.take((size_t)cnt * s);
            }
        }
    }
    // ---- multi-resolution ghost fill rectangles
    G.segs_h.clear();
    G.fill_total = 0;
    if (p.multires) {
        const int64_t reads = build_fill_segments(G);
        if (reads < 0) return "a block face borders cells more than 16 times finer (cell ratio across a face is limited to 16)";
        // by decreasing cost (ghost cells times the source values each
        // averages, plus its store): the persistent form deals rectangles to
        // its waves with a fixed stride, so each gets a similar share
        auto cost = [](const FillSeg& S) {
            const int32_t rr = S.hc >> S.lhn, r = rr > 1 ? rr : 1;
            return (int64_t)S.n1 * S.n2 * (r * r + 1);
        };
        std::stable_sort(G.segs_h.begin(), G.segs_h.end(),
                         [&](const FillSeg& a, const FillSeg& b) { return cost(a) > cost(b); });
        // algorithmic ghost traffic: same-size faces read their neighbour
        // cells, resolution-change faces the neighbour cells their fill reads
        int64_t direct = 0;
        for (const TileHost& t : p.tiles)
            for (int f = 0; f < 6; ++f)
                if (t.kind[f] == 0) direct += (int64_t)t.e[0] * t.e[1] * t.e[2] / t.e[f / 2];
        p.halo_cells = direct + reads;
    }
    // ---- x-column exports of the chares a resolution-change x face reads:
    // per (chare, side) one (y, z) array per parity, written by the sweep
    G.xexp_h.clear();
    if (!G.segs_h.empty()) {
        G.xexp_h.assign((size_t)C, XExpDev{{{-1, -1}, {-1, -1}}});
        for (FillSeg& S : G.segs_h) {
            if (S.d != 0) continue;
            const Chare& N = p.chares[(size_t)S.src];
            const int side = S.lay == 0 ? 0 : (S.lay == N.e[0] - 1 ? 1 : -1);
            if (side < 0) continue;
            XExpDev& X = G.xexp_h[(size_t)S.src];
            if (X.off[side][0] < 0)
                for (int q = 0; q < 2; ++q) X.off[side][q] = (int64_t)(cv.take((size_t)N.e[1] * N.e[2] * s) / s);
            S.eoff[0] = X.off[side][0];
            S.eoff[1] = X.off[side][1];
            S.ey = N.e[1];
        }
    }
    // ---- control regions: descriptors and device state
    G.L.field_end = align_up(cv.off, kAlign);
    cv.off = G.L.field_end;
    G.L.ctrl_begin = G.L.field_end;
    const size_t nblocks = (size_t)C + (size_t)npb;
    const size_t ntiles = p.tiles.size();
    G.L.blocks = cv.take(nblocks * sizeof(BlockDev));
    // room for the tiles of any autotune candidate (smallest candidate tile,
    // plus splits down to the block granularity for explicit blocks)
    G.tile_cap = ntiles;
    if (G.tune_room && (cfg.exec == OD_FUSED || cfg.exec == OD_GRAPH || cfg.exec == OD_PERSISTENT)) {
        int32_t m[3], eymax = 1;
        for (const Chare& c : p.chares) eymax = std::max(eymax, c.e[1]);
        tune_min_tile(G.s, eymax, m);
        size_t cap = 0;
        for (const Chare& c : p.chares) {
            size_t k = 1;
            for (int d = 0; d < 3; ++d) {
                int32_t md = m[d];
                if (!p.regular) md = std::min(md, std::max<int32_t>(1, p.gcell));
                k *= (size_t)ceil_div(c.e[d], md);
            }
            cap += k;
        }
        G.tile_cap = std::max(ntiles, cap);
    }
    // the persistent form's guided tail adds up to three entries per
    // workgroup plus padding (guided_tail); cooperative grids stay below 8192
    // two-step line descriptors: room for the planned tiles and for
    // autotune candidates down to (32, 8, 16) tiles (finer candidates run
    // one step per pass), plus the persistent guided tail's entries
    G.tile2_cap = 0;
    if (two_step_room(G)) {
        size_t cap2 = 0;
        for (const Chare& c : p.chares)
            cap2 += (size_t)ceil_div(c.e[0], 32) * (size_t)ceil_div(c.e[1], 8) * (size_t)ceil_div(c.e[2], 16);
        G.tile2_cap = std::min(G.tile_cap, std::max(ntiles, G.tune_room ? cap2 * (p.regular ? 1 : 2) : ntiles));
        if (cfg.exec == OD_PERSISTENT) G.tile2_cap += 3 * 8192 + kNumXcd;
    }
    if (cfg.exec == OD_PERSISTENT) G.tile_cap += 3 * 8192 + kNumXcd;
    G.L.tiles = cv.take(G.tile_cap * sizeof(TileDev));
    G.halo2_cells = two_step_room(G) ? halo2_count(p) : 0;
    G.L.tiles2 = cv.take(std::max<size_t>(G.tile2_cap, 1) * sizeof(Tile2Dev));
    for (int d = 0; d < 3; ++d) G.L.cidx[d] = cv.take((size_t)(p.regular ? p.n[d] : 1) * 4);
    G.L.owner = cv.take((p.regular ? 1 : p.owner.size()) * 4);
    G.L.corigin = cv.take((size_t)C * 3 * 4);
    G.L.ccell = cv.take((size_t)C * 4);
    G.L.dir_pb = cv.take((size_t)C * 6 * 4);
    G.L.pb_face = cv.take((size_t)std::max(npb, 1) * 4);
    G.L.pb_block = cv.take((size_t)std::max(npb, 1) * 4);
    G.L.bc = cv.take(6 * 8);
    G.nres = cfg.exec == OD_PER_CHARE ? C : 1;
    G.L.res = cv.take((size_t)(2 * G.nres + 2) * 8);
    G.L.bar = cv.take(kBarWords * 4);
    G.L.err = cv.take(4);
    G.L.done = cv.take(ntiles * 4);
    G.L.target = cv.take(4 * 4);
    // message-driven dependencies
    G.dep_ptr.clear();
    G.dep_idx.clear();
    if (cfg.exec == OD_MSGDRIVEN) {
        // two-step tasks (decided with the tile list, as decide_two_step
        // will) read tiles up to two cells away
        const bool reach2 = two_step_possible(G) && sweep2_variant_ok(G.s, p.tile[0], p.tile[1]) &&
                            p.tiles.size() <= G.tile2_cap;
        std::string e2 = build_tile_deps(p, G.dep_ptr, G.dep_idx, reach2);
        if (!e2.empty()) return e2;
    }
    G.L.xpub = cv.take(cfg.exec == OD_MSGDRIVEN ? ntiles : 1);
    if (cfg.exec == OD_MSGDRIVEN) {
        // a queue entry holds a tile index in 24 bits
        if (ntiles >= ((size_t)1 << 23)) return "message-driven grids are limited to 2^23 - 1 tiles";
        // dependency counters; per present XCD a ready ring and a cross
        // list of the next power of two >= its tile count
        G.L.pend = cv.take(ntiles * 2 * 4);
        G.L.qslots = cv.take(2 * (2 * ntiles + 8) * 8);   // ready queues, then cross lists
        G.L.qctl = cv.take(64 * 4);
    }
    G.L.stamps = cv.take(cfg.exec == OD_PERSISTENT ? (size_t)4 * kStampIters * 8 : 8);
    G.L.dep_ptr = cv.take((G.dep_ptr.size() + 1) * 4);
    G.L.dep_idx = cv.take((G.dep_idx.size() + 1) * 4);
    G.L.segs = cv.take(std::max<size_t>(G.segs_h.size(), 1) * sizeof(FillSeg));
    G.L.xexp = cv.take(std::max<size_t>(G.xexp_h.size(), 1) * sizeof(XExpDev));
    G.L.total = align_up(cv.off, kAlign) + kAlign;
    return fill_tile_descs(G);
}

// Tiles whose box intersects a ghost slab of tile t (face neighbours through
// which halos are read), as CSR lists.
std::string build_tile_deps(const Plan& p, std::vector<int32_t>& ptr, std::vector<int32_t>& idx, bool reach2) {
    const size_t T = p.tiles.size();
    // per chare: regular cut index -> tile ids
    struct Key {
        int32_t c, ix, iy, iz;
        bool operator<(const Key& o) const {
            if (c != o.c) return c < o.c;
            if (iz != o.iz) return iz < o.iz;
            if (iy != o.iy) return iy < o.iy;
            return ix < o.ix;
        }
    };
    std::map<Key, std::vector<int32_t>> cut;
    for (size_t i = 0; i < T; ++i) {
        const TileHost& t = p.tiles[i];
        cut[Key{t.chare, t.o[0] / p.tile[0], t.o[1] / p.tile[1], t.o[2] / p.tile[2]}].push_back((int32_t)i);
    }
    ptr.assign(T + 1, 0);
    idx.clear();
    for (size_t i = 0; i < T; ++i) {
        const TileHost& t = p.tiles[i];
        std::vector<int32_t> deps;
        // tiles of chare sc overlapping the box [lo, hi) (chare-local)
        auto add_box = [&](int32_t sc, const int64_t lo[3], const int64_t hi[3]) {
            for (int64_t iz = lo[2] / p.tile[2]; iz <= (hi[2] - 1) / p.tile[2]; ++iz)
                for (int64_t iy = lo[1] / p.tile[1]; iy <= (hi[1] - 1) / p.tile[1]; ++iy)
                    for (int64_t ix = lo[0] / p.tile[0]; ix <= (hi[0] - 1) / p.tile[0]; ++ix) {
                        auto it = cut.find(Key{sc, (int32_t)ix, (int32_t)iy, (int32_t)iz});
                        if (it == cut.end()) continue;
                        for (int32_t o : it->second) {
                            const TileHost& u = p.tiles[(size_t)o];
                            bool hit = true;
                            for (int d = 0; d < 3 && hit; ++d)
                                hit = u.o[d] < hi[d] && lo[d] < (int64_t)u.o[d] + u.e[d];
                            if (hit && o != (int32_t)i) deps.push_back(o);
                        }
                    }
        };
        for (int f = 0; f < 6; ++f) {
            if (t.kind[f] == 1) continue;
            const int32_t sc = t.kind[f] == 2 ? t.chare : t.src[f];
            const Chare& c = p.chares[(size_t)sc];
            int64_t lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = t.g[f][d] - c.o[d];
                hi[d] = lo[d] + (d == f / 2 ? 1 : t.e[d]);
            }
            add_box(sc, lo, hi);
        }
        if (reach2) {
            // a pass of two steps also reads the slabs two out and the
            // cells diagonal to each edge (every such box lies in one
            // chare: the two-step lines' condition); boxes outside the
            // domain are boundary values
            const Chare& own = p.chares[(size_t)t.chare];
            int64_t g0[3], g1[3];
            for (int d = 0; d < 3; ++d) {
                g0[d] = (int64_t)own.u[d] + t.o[d];
                g1[d] = g0[d] + t.e[d];
            }
            std::vector<std::array<int64_t, 6>> boxes;   // global lo[3], hi[3]
            for (int f = 0; f < 6; ++f) {
                const int d = f / 2;
                std::array<int64_t, 6> b{g0[0], g0[1], g0[2], g1[0], g1[1], g1[2]};
                b[(size_t)d] = (f & 1) ? g1[d] + 1 : g0[d] - 2;
                b[(size_t)d + 3] = b[(size_t)d] + 1;
                boxes.push_back(b);
            }
            for (int d1 = 0; d1 < 3; ++d1)
                for (int d2 = d1 + 1; d2 < 3; ++d2)
                    for (int s1 = 0; s1 < 2; ++s1)
                        for (int s2 = 0; s2 < 2; ++s2) {
                            std::array<int64_t, 6> b{g0[0], g0[1], g0[2], g1[0], g1[1], g1[2]};
                            b[(size_t)d1] = s1 ? g1[d1] : g0[d1] - 1;
                            b[(size_t)d1 + 3] = b[(size_t)d1] + 1;
                            b[(size_t)d2] = s2 ? g1[d2] : g0[d2] - 1;
                            b[(size_t)d2 + 3] = b[(size_t)d2] + 1;
                            boxes.push_back(b);
                        }
            for (const auto& b : boxes) {
                bool inside = true;
                for (int d = 0; d < 3; ++d) inside = inside && b[(size_t)d] >= 0 && b[(size_t)d + 3] <= p.n[d];
                if (!inside) continue;
                const int32_t sc = plan_owner(p, b[0], b[1], b[2]);
                if (sc != plan_owner(p, b[3] - 1, b[4] - 1, b[5] - 1))
                    return std::string("internal error: a two-step box spans chares");
                const Chare& c = p.chares[(size_t)sc];
                int64_t lo[3], hi[3];
                for (int d = 0; d < 3; ++d) {
                    lo[d] = b[(size_t)d] - c.u[d];
                    hi[d] = b[(size_t)d + 3] - c.u[d];
                }
                add_box(sc, lo, hi);
            }
        }
        std::sort(deps.begin(), deps.end());
        deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
        idx.insert(idx.end(), deps.begin(), deps.end());
        ptr[i + 1] = (int32_t)idx.size();
    }
    // The schedulers need the relation symmetric (a tile waits for the
    // tiles that read it before overwriting a parity, and counts its finish
    // for them): add any missing reverse edge.
    std::vector<std::vector<int32_t>> adj(T);
    bool sym = true;
    for (size_t i = 0; i < T; ++i)
        for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) {
            const int32_t j = idx[(size_t)q];
            adj[i].push_back(j);
            if (!std::binary_search(idx.begin() + ptr[(size_t)j], idx.begin() + ptr[(size_t)j + 1], (int32_t)i)) {
                adj[(size_t)j].push_back((int32_t)i);
                sym = false;
            }
        }
    if (!sym) {
        idx.clear();
        for (size_t i = 0; i < T; ++i) {
            std::sort(adj[i].begin(), adj[i].end());
            adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
            idx.insert(idx.end(), adj[i].begin(), adj[i].end());
            ptr[i + 1] = (int32_t)idx.size();
        }
    }
    return "";
}

// Persistent form with tile counters: the workgroups of XCD group g claim
// list positions g, g + 8, g + 16, ... in order.  The last claims of an
// iteration leave workgroups idle until the slowest tile ends, so the last
// `tail` tiles of each group are cut into `pieces` z-ranges (sub-tiles: the
// same box cut along z, a cut face reading the tile's own plane) and
// claimed last, shortening that wait to about one piece.  Groups are padded
// to one length with empty entries (nz = 0).  Sub-tiles compute the same
// expression at every point, so results are unchanged.
std::vector<TileHost> guided_tail(const Plan& p, const std::vector<TileHost>& tiles, int32_t tail, int32_t pieces) {
    if (tiles.size() < (size_t)kNumXcd || tail <= 0 || pieces <= 1) return tiles;
    auto sub = [&](const TileHost& t, int32_t za, int32_t zb) {
        const Chare& c = p.chares[(size_t)t.chare];
        TileHost u = t;
        u.o[2] = t.o[2] + za;
        u.e[2] = zb - za;
        for (int f = 0; f < 4; ++f) u.g[f][2] = t.g[f][2] + za;
        if (za > 0) {   // z- slab: the tile's own plane below
            u.kind[4] = 2;
            u.src[4] = t.chare;
            u.g[4][0] = c.o[0] + t.o[0];
            u.g[4][1] = c.o[1] + t.o[1];
            u.g[4][2] = c.o[2] + u.o[2] - 1;
        }
        if (zb < t.e[2]) {   // z+ slab: the tile's own plane above
            u.kind[5] = 2;
            u.src[5] = t.chare;
            u.g[5][0] = c.o[0] + t.o[0];
            u.g[5][1] = c.o[1] + t.o[1];
            u.g[5][2] = c.o[2] + u.o[2] + u.e[2];
        }
        return u;
    };
    std::vector<std::vector<TileHost>> seq((size_t)kNumXcd);
    size_t len = 0;
    for (int g = 0; g < kNumXcd; ++g) {
        std::vector<TileHost>& q = seq[(size_t)g];
        for (size_t i = (size_t)g; i < tiles.size(); i += kNumXcd) q.push_back(tiles[i]);
        const size_t keep = q.size() > (size_t)tail ? q.size() - (size_t)tail : 0;
        std::vector<TileHost> cut(q.begin(), q.begin() + (std::ptrdiff_t)keep);
        for (size_t i = keep; i < q.size(); ++i) {
            const TileHost& t = q[i];
            const int32_t np = std::max<int32_t>(1, std::min<int32_t>(pieces, t.e[2] / 4));
            for (int32_t k = 0; k < np; ++k) {
                const int32_t za = (int32_t)((int64_t)t.e[2] * k / np), zb = (int32_t)((int64_t)t.e[2] * (k + 1) / np);
                cut.push_back(sub(t, za, zb));
            }
        }
        q.swap(cut);
        len = std::max(len, q.size());
    }
    std::vector<TileHost> out(len * kNumXcd);
    for (size_t k = 0; k < len; ++k)
        for (int g = 0; g < kNumXcd; ++g) {
            const std::vector<TileHost>& q = seq[(size_t)g];
            if (k < q.size()) {
                out[k * kNumXcd + (size_t)g] = q[k];
            } else {
                TileHost e = q.empty() ? tiles[0] : q.back();
                e.e[2] = 0;
                out[k * kNumXcd + (size_t)g] = e;
            }
        }
    return out;
}

od_status Grid::setup_cooperative(bool fresh_plan) {
    grid_wgs = 0;
    if (cfg.exec != OD_PERSISTENT && cfg.exec != OD_MSGDRIVEN) return OD_OK;
    if (fresh_plan || base_tiles.empty()) base_tiles = plan.tiles;
    // the schedule may have changed since the tile list was built: the
    // kernel (and with it the co-resident grid) follows it
    if (cfg.exec == OD_PERSISTENT)
        two_step = two_step_possible(*this) && sweep2_variant_ok(s, plan.tile[0], plan.tile[1]) &&
                   base_tiles.size() <= tile2_cap;
    int cap = persistent_max_grid(s, plan.tile[0], plan.tile[1], coop_kind(), persist_waves);
    // a message-driven grid with two-step tasks runs an odd last iteration
    // with the one-step kernel on the same grid
    if (cfg.exec == OD_MSGDRIVEN && two_step)
        cap = std::min(cap, persistent_max_grid(s, plan.tile[0], plan.tile[1], 1, persist_waves));
    int grid = std::min<int>(cap, (int)base_tiles.size());
    if (grid >= kNumXcd) grid -= grid % kNumXcd;
    grid_wgs = grid;
    if (grid <= 0) return fail(OD_EHIP, "no co-resident workgroups for the cooperative kernel");
    if (cfg.exec == OD_PERSISTENT) {
        std::vector<TileHost> list = base_tiles;
        if (sched() == 3 && two_step) {
            // uniform passes: only the partial last round of each XCD group
            // is cut, into enough z-ranges to occupy the group's workgroups
            const int32_t W = grid / kNumXcd, per = (int32_t)(base_tiles.size() / kNumXcd);
            const int32_t rem = W > 0 ? per % W : 0;
            if (rem > 0) list = guided_tail(plan, base_tiles, rem, std::min<int32_t>(4, (W + rem - 1) / rem));
        } else if (sched() == 3) {
            list = guided_tail(plan, base_tiles, grid / kNumXcd, 4);
        }
        if (list.size() > tile_cap || (two_step && list.size() > tile2_cap))
            return fail(OD_EINVAL, "cut tile list exceeds the tile capacity");
        if (list.size() != plan.tiles.size() || !fresh_plan || two_step) {
            plan.tiles.swap(list);
            std::string e = fill_tile_descs(*this);   // also the two-step lines of the final list
            if (!e.empty()) return fail(OD_EINVAL, e);
            od_status us = upload_tiles();
            if (us != OD_OK) return us;
        }
    }
    return OD_OK;
}

// ---------------------------------------------------------------------------

od_status Grid::upload() {
    if (!ctrl) ctrl = base + L.ctrl_begin;   // control regions follow the fields in the workspace
    auto put = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(cp(off), src, bytes, hipMemcpyHostToDevice, st);
    };
    const Plan& p = plan;
    const int32_t C = (int32_t)p.chares.size();
    std::vector<int32_t> corigin((size_t)C * 3);
    std::vector<int32_t> ccell((size_t)C);
    for (int32_t c = 0; c < C; ++c) {
        for (int d = 0; d < 3; ++d) corigin[(size_t)c * 3 + d] = p.chares[(size_t)c].u[d];
        ccell[(size_t)c] = p.chares[(size_t)c].h;
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = put(L.blocks, blocks_h.data(), blocks_h.size() * sizeof(BlockDev));
    if (e == hipSuccess) e = put(L.tiles, tiles_h.data(), tiles_h.size() * sizeof(TileDev));
    if (e == hipSuccess) e = put(L.tiles2, tiles2_h.data(), tiles2_h.size() * sizeof(Tile2Dev));
    std::vector<int32_t> cidx[3];
    if (p.regular) {
        for (int d = 0; d < 3; ++d) {
            cidx[d].resize((size_t)p.n[d]);
            for (int32_t i = 0; i < p.k[d]; ++i)
                for (int32_t v = p.split[d][(size_t)i]; v < p.split[d][(size_t)i + 1]; ++v) cidx[d][(size_t)v] = i;
            if (e == hipSuccess) e = put(L.cidx[d], cidx[d].data(), cidx[d].size() * 4);
        }
    } else if (e == hipSuccess) {
        e = put(L.owner, p.owner.data(), p.owner.size() * 4);
    }
    if (e == hipSuccess) e = put(L.corigin, corigin.data(), corigin.size() * 4);
    if (e == hipSuccess) e = put(L.ccell, ccell.data(), ccell.size() * 4);
    if (e == hipSuccess) e = put(L.segs, segs_h.data(), segs_h.size() * sizeof(FillSeg));
    if (e == hipSuccess) e = put(L.xexp, xexp_h.data(), xexp_h.size() * sizeof(XExpDev));
    if (e == hipSuccess) e = put(L.dir_pb, dir_pb.data(), dir_pb.size() * 4);
    if (e == hipSuccess) e = put(L.pb_face, pb_face.data(), pb_face.size() * 4);
    if (e == hipSuccess) e = put(L.pb_block, pb_block.data(), pb_block.size() * 4);
    if (e == hipSuccess) e = put(L.bc, cfg.bc, 6 * 8);
    if (e == hipSuccess) e = put(L.dep_ptr, dep_ptr.data(), dep_ptr.size() * 4);
    if (e == hipSuccess) e = put(L.dep_idx, dep_idx.data(), dep_idx.size() * 4);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("descriptor upload: ") + hipGetErrorString(e));

    gdev.arena = base;
    gdev.blocks = reinterpret_cast<const BlockDev*>(cp(L.blocks));
    gdev.lk.regular = p.regular ? 1 : 0;
    for (int d = 0; d < 3; ++d) {
        gdev.lk.k[d] = p.k[d];
        gdev.lk.cidx[d] = reinterpret_cast<const int32_t*>(cp(L.cidx[d]));
        gdev.lk.og[d] = (int32_t)p.og[d];
        gdev.n[d] = p.n[d];
    }
    gdev.lk.owner = reinterpret_cast<const int32_t*>(cp(L.owner));
    gdev.lk.gran = p.gran;
    gdev.lk.corigin = reinterpret_cast<const int32_t*>(cp(L.corigin));
    gdev.lk.dir_pb = reinterpret_cast<const int32_t*>(cp(L.dir_pb));
    return OD_OK;
}

od_status Grid::reset_state() {
    // zero residual slots, barrier, error flag and step counters with a
    // plain fill (not captured into any graph)
    hipError_t e = hipMemsetAsync(cp(L.res), 0, (size_t)(2 * nres + 2) * 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(cp(L.bar), 0, kBarWords * 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(cp(L.err), 0, 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(cp(L.done), 0, std::max<size_t>(tiles_h.size(), 1) * 4, st);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("state reset: ") + hipGetErrorString(e));
    parity = 0;
    iters = 0;
    flips = 0;
    faces_packed = false;
    return OD_OK;
}

od_status Grid::init_field() {
    hipError_t e = launch_init(s, st, gdev, (int32_t)plan.chares.size(), cfg.seed, (int32_t)pb_face.size(),
                               reinterpret_cast<const int32_t*>(cp(L.pb_face)),
                               reinterpret_cast<const int32_t*>(cp(L.pb_block)),
                               reinterpret_cast<const double*>(cp(L.bc)), !plan.multires);
    if (e == hipSuccess && plan.multires)
        e = launch_init_cells(s, st, gdev, reinterpret_cast<const int32_t*>(cp(L.ccell)),
                              (int32_t)plan.chares.size(), cfg.seed);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("init: ") + hipGetErrorString(e));
    return refresh_xexp(0);
}

const XExpDev* Grid::xexp_dev() {
    return xexp_h.empty() ? nullptr : reinterpret_cast<const XExpDev*>(cp(L.xexp));
}

// Copy the exported x-columns of field `par` from the chares (after the
// field was written other than by a sweep: initialisation, block writes).
od_status Grid::refresh_xexp(int par) {
    if (xexp_h.empty()) return OD_OK;
    hipError_t e = launch_xexp_refresh(s, st, base, reinterpret_cast<const BlockDev*>(cp(L.blocks)), xexp_dev(),
                                       (int32_t)plan.chares.size(), par);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("x-column export refresh: ") + hipGetErrorString(e));
    return OD_OK;
}

Grid::~Grid() {
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    for (hipEvent_t ev : packed) hipEventDestroy(ev);
    for (hipStream_t s2 : pool) hipStreamDestroy(s2);
    if (cap_st) hipStreamDestroy(cap_st);
    if (pinned && !pinned_borrowed) hipHostFree(pinned);
}

od_status Grid::ensure_pinned(size_t bytes) {
    if (pinned_bytes >= bytes) return OD_OK;
    if (pinned_borrowed) return fail(OD_EINVAL, "borrowed staging buffer too small");
    if (pinned) hipHostFree(pinned);
    pinned = nullptr;
    pinned_bytes = 0;
    hipError_t e = hipHostMalloc(&pinned, bytes, hipHostMallocDefault);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("hipHostMalloc staging: ") + hipGetErrorString(e));
    pinned_bytes = bytes;
    return OD_OK;
}

// ---- sweeps ------------------------------------------------------------------

unsigned long long* Grid::res_ptr() { return reinterpret_cast<unsigned long long*>(cp(L.res)); }

od_status Grid::fused_one(hipStream_t s2, int par, int64_t step) {
    if (!segs_h.empty()) {
        hipError_t e0 = launch_amr_fill(s, s2, base, reinterpret_cast<const BlockDev*>(cp(L.blocks)),
                                        reinterpret_cast<const FillSeg*>(cp(L.segs)), (int32_t)segs_h.size(),
                                        fill_total, par);
        if (e0 != hipSuccess) return fail(OD_EHIP, std::string("ghost fill launch: ") + hipGetErrorString(e0));
    }
    hipError_t e = launch_sweep(s, plan.tile[0], plan.tile[1], s2, base,
                                reinterpret_cast<const BlockDev*>(cp(L.blocks)),
                                reinterpret_cast<const TileDev*>(cp(L.tiles)), (int32_t)tiles_h.size(), par,
                                res_ptr(), 0, 1, imb, step, mode(), xexp_dev());
    if (e != hipSuccess) return fail(OD_EHIP, std::string("sweep launch: ") + hipGetErrorString(e));
    return OD_OK;
}

od_status Grid::fused_two(hipStream_t s2, int par, int64_t step) {
    hipError_t e = launch_sweep2(s, plan.tile[0], plan.tile[1], s2, base, reinterpret_cast<const BlockDev*>(cp(L.blocks)),
                                 reinterpret_cast<const TileDev*>(cp(L.tiles)),
                                 reinterpret_cast<const Tile2Dev*>(cp(L.tiles2)), (int32_t)tiles_h.size(), par,
                                 res_ptr(), 0, 1, mode(), imb, step);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("two-step sweep launch: ") + hipGetErrorString(e));
    return OD_OK;
}

od_status Grid::upload_tiles() {
    hipError_t he = hipMemcpyAsync(cp(L.tiles), tiles_h.data(), tiles_h.size() * sizeof(TileDev),
                                   hipMemcpyHostToDevice, st);
    if (he == hipSuccess && !tiles2_h.empty())
        he = hipMemcpyAsync(cp(L.tiles2), tiles2_h.data(), tiles2_h.size() * sizeof(Tile2Dev), hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return fail(OD_EHIP, std::string("tile upload: ") + hipGetErrorString(he));
    return OD_OK;
}

od_status Grid::graph_run(int64_t n) {
    while (n > 0) {
        const int64_t m = std::min(n, kMaxGraphLen);
        auto key = std::make_pair(parity, m);
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            if (!cap_st) {
                hipError_t e = hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking);
                if (e != hipSuccess) return fail(OD_EHIP, std::string("capture stream: ") + hipGetErrorString(e));
            }
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(cap_st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return fail(OD_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
            od_status os = OD_OK;
            int par = parity;
            for (int64_t i = 0; i < m && os == OD_OK; par ^= 1) {
                if (two_step && m - i >= 2) {
                    os = fused_two(cap_st, par, iters + i);
                    i += 2;
                } else {
                    os = fused_one(cap_st, par, iters + i);
                    i += 1;
                }
            }
            e = hipStreamEndCapture(cap_st, &graph);
            if (os != OD_OK) {
                if (graph) hipGraphDestroy(graph);
                return os;
            }
            if (e != hipSuccess) return fail(OD_EHIP, std::string("end capture: ") + hipGetErrorString(e));
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(OD_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            it = graphs.emplace(key, exec).first;
        }
        hipError_t e = hipGraphLaunch(it->second, st);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
        parity ^= (int)((two_step ? m / 2 + m % 2 : m) & 1);   // one flip per pass
        iters += m;
        n -= m;
    }
    return OD_OK;
}

od_status Grid::persistent_run(int64_t n) {
    if (grid_wgs <= 0) return fail(OD_EHIP, "persistent kernel: no co-resident workgroups");
    if (plan.multires) {
        hipError_t e = launch_persistent_mr(s, plan.tile[0], plan.tile[1], st, grid_wgs, base,
                                            reinterpret_cast<const BlockDev*>(cp(L.blocks)),
                                            reinterpret_cast<const TileDev*>(cp(L.tiles)), (int32_t)tiles_h.size(),
                                            parity, n, res_ptr(), 1, reinterpret_cast<unsigned int*>(cp(L.bar)),
                                            reinterpret_cast<unsigned int*>(cp(L.err)),
                                            device_wait_ticks(cfg.wait_s > 0 ? cfg.wait_s : 10.0), mode(),
                                            reinterpret_cast<const FillSeg*>(cp(L.segs)), (int32_t)segs_h.size(),
                                            xexp_dev());
        if (e != hipSuccess) return fail(OD_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
        parity ^= (int)(n & 1);
        iters += n;
        return OD_OK;
    }
    if (two_step) {
        // n / 2 two-step passes in one launch, an odd last step as a single sweep
        const int64_t passes = n / 2;
        hipError_t e = launch_persistent2(s, plan.tile[0], plan.tile[1], st, grid_wgs, base,
                                          reinterpret_cast<const BlockDev*>(cp(L.blocks)),
                                          reinterpret_cast<const TileDev*>(cp(L.tiles)),
                                          reinterpret_cast<const Tile2Dev*>(cp(L.tiles2)), (int32_t)tiles_h.size(),
                                          parity, passes, res_ptr(), 1, reinterpret_cast<unsigned int*>(cp(L.bar)),
                                          reinterpret_cast<unsigned int*>(cp(L.err)), mode(),
                                          device_wait_ticks(cfg.wait_s > 0 ? cfg.wait_s : 10.0),
                                          persistent_dyn() ? 1 : 0, imb, iters);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
        parity ^= (int)(passes & 1);
        iters += 2 * passes;
        if (n & 1) {
            od_status os = fused_one(st, parity, iters);
            if (os != OD_OK) return os;
            parity ^= 1;
            iters += 1;
        }
        return OD_OK;
    }
    unsigned long long* stamps = nullptr;
    if (cfg.hints & kHintTimeline) {
        stamps = reinterpret_cast<unsigned long long*>(cp(L.stamps));
        stamp_iters = (int32_t)std::min<int64_t>(n, kStampIters);
        hipError_t e0 = launch_stamp_init(st, stamps, stamp_iters);
        if (e0 != hipSuccess) return fail(OD_EHIP, std::string("timeline init: ") + hipGetErrorString(e0));
    }
    hipError_t e = launch_persistent(s, plan.tile[0], plan.tile[1], st, grid_wgs, base,
                                     reinterpret_cast<const BlockDev*>(cp(L.blocks)),
                                     reinterpret_cast<const TileDev*>(cp(L.tiles)), (int32_t)tiles_h.size(),
                                     parity, n, res_ptr(), 1, reinterpret_cast<unsigned int*>(cp(L.bar)),
                                     reinterpret_cast<unsigned int*>(cp(L.err)),
                                     imb, iters, mode(),
                                     persistent_dyn() ? 1 : 0,
                                     device_wait_ticks(cfg.wait_s > 0 ? cfg.wait_s : 10.0), stamps,
                                     sched() == 4 ? 1 : 0);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("persistent launch: ") + hipGetErrorString(e));
    parity ^= (int)(n & 1);
    iters += n;
    return OD_OK;
}

od_status Grid::msgdriven_run(int64_t n) {
    if (grid_wgs <= 0) return fail(OD_EHIP, "message-driven kernel: no co-resident workgroups");
    if (iters + n > INT32_MAX) return fail(OD_EINVAL, "step counters limited to 2^31 iterations");
    // One launch runs fewer than 2^16 steps (a task carries its step
    // relative to the launch's first) and at most 2^23 tasks, so a queue's
    // 24-bit slot sequences never alias and finish counters never wrap.
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(((int64_t)1 << 16) - 1,
                                                               ((int64_t)1 << 23) / std::max<size_t>(tiles_h.size(), 1)));
    // two-step tasks: n / 2 passes, an odd last iteration as a one-step launch
    int64_t m = two_step ? n / 2 : n;
    while (m > 0) {
        const int64_t k = std::min(m, per);
        od_status st2 = msgdriven_launch(k, two_step);
        if (st2 != OD_OK) return st2;
        m -= k;
    }
    if (two_step && (n & 1)) return msgdriven_launch(1, false);
    return OD_OK;
}

od_status Grid::msgdriven_launch(int64_t n, bool pairs) {
    // target = flips + n scheduler steps; the final-step residual slots
    // (2, 3) are cleared
    const int32_t tgt = (int32_t)(flips + n);
    MsgArgs a{};
    a.arena = base;
    a.blocks = reinterpret_cast<const BlockDev*>(cp(L.blocks));
    a.tiles = reinterpret_cast<const TileDev*>(cp(L.tiles));
    a.tiles2 = pairs ? reinterpret_cast<const Tile2Dev*>(cp(L.tiles2)) : nullptr;
    a.ntiles = (int32_t)tiles_h.size();
    a.dep_ptr = reinterpret_cast<const int32_t*>(cp(L.dep_ptr));
    a.dep_idx = reinterpret_cast<const int32_t*>(cp(L.dep_idx));
    a.done = reinterpret_cast<int32_t*>(cp(L.done));
    a.target = reinterpret_cast<const int32_t*>(cp(L.target));
    a.tile_solve = nullptr;
    a.res = res_ptr() + 2;   // slot (final step & 1) of this 2-slot pair
    a.err = reinterpret_cast<unsigned int*>(cp(L.err));
    a.imb = imb;
    // scheduler step k of this launch is iteration iters + (k - flips) per
    // step of a one-step task, two per two-step task
    a.imb_base = pairs ? iters - 2 * flips : iters - flips;
    a.wait_ticks = device_wait_ticks(cfg.wait_s > 0 ? cfg.wait_s : 10.0);
    a.hints = mode();
    a.seed = cfg.seed;
    a.pert_ticks = (cfg.hints & kHintCheck) ? device_wait_ticks(20e-6) : 0;
    a.sched = msg_sched_bits();
    a.xpub = reinterpret_cast<uint8_t*>(cp(L.xpub));
    a.tile_pos = nullptr;
    a.bar = reinterpret_cast<unsigned int*>(cp(L.bar));
    a.pend = reinterpret_cast<int32_t*>(cp(L.pend));
    a.qslots = reinterpret_cast<unsigned long long*>(cp(L.qslots));
    a.pslots = a.qslots + (2 * tiles_h.size() + 8);
    a.ready = reinterpret_cast<int32_t*>(a.qslots);   // the cursor scheduler uses the ready-queue region
    a.qhead = reinterpret_cast<unsigned int*>(cp(L.qctl));
    a.qsteps = (int32_t)n;
    // the init kernel stores the target step and clears the final-step
    // residual pair (kernel arguments: nothing on the host outlives this call)
    hipError_t e = launch_queue_init(st, a, tgt, reinterpret_cast<int32_t*>(cp(L.target)), res_ptr() + 2);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("queue init: ") + hipGetErrorString(e));
    e = pairs ? launch_msgdriven2(s, plan.tile[0], plan.tile[1], st, grid_wgs, a)
              : launch_msgdriven(s, plan.tile[0], plan.tile[1], st, grid_wgs, a);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("msg-driven launch: ") + hipGetErrorString(e));
    parity = tgt & 1;
    flips = tgt;
    iters += pairs ? 2 * n : n;
    msg_final = true;
    return OD_OK;
}

od_status Grid::per_chare_run(int64_t n) {
    const Plan& p = plan;
    const int32_t C = (int32_t)p.chares.size();
    if (pool.empty()) {
        pool.resize((size_t)std::min(C, kStreamPool));
        for (auto& s2 : pool) {
            hipError_t e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
            if (e != hipSuccess) return fail(OD_EHIP, std::string("stream pool: ") + hipGetErrorString(e));
        }
        packed.resize((size_t)C);
        for (auto& ev : packed) {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return fail(OD_EHIP, std::string("event: ") + hipGetErrorString(e));
        }
        // per-chare tile ranges (tiles are chare-major in this mode)
        tile_lo.assign((size_t)C + 1, 0);
        for (const TileHost& t : p.tiles) tile_lo[(size_t)t.chare + 1]++;
        for (int32_t c = 0; c < C; ++c) tile_lo[(size_t)c + 1] += tile_lo[(size_t)c];
        if (!join_ev) {
            hipError_t e = hipEventCreateWithFlags(&join_ev, hipEventDisableTiming);
            if (e != hipSuccess) return fail(OD_EHIP, std::string("event: ") + hipGetErrorString(e));
        }
    }
    auto sp = [&](int32_t c) { return pool[(size_t)c % pool.size()]; };
    auto face_out = [&](int32_t c, int par) {
        FaceSet fs{};
        for (int f = 0; f < 6; ++f) {
            const MsgBufs& mb = msg[(size_t)c];
            if (mb.cnt[f] > 0) {
                fs.p[f] = base + mb.out[par][f];
                fs.cnt[f] = mb.cnt[f];
            }
        }
        return fs;
    };
    // the pool streams start after all work already queued on the grid stream
    hipError_t e = hipEventRecord(join_ev, st);
    for (auto& s2 : pool)
        if (e == hipSuccess) e = hipStreamWaitEvent(s2, join_ev, 0);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("per-chare join: ") + hipGetErrorString(e));
    if (!faces_packed) {
        for (int32_t c = 0; c < C && e == hipSuccess; ++c) {
            e = launch_pack_b(s, sp(c), base, blocks_h[(size_t)c], parity, face_out(c, parity));
            if (e == hipSuccess) e = hipEventRecord(packed[(size_t)c], sp(c));
        }
        if (e != hipSuccess) return fail(OD_EHIP, std::string("initial pack: ") + hipGetErrorString(e));
        faces_packed = true;
    }
    for (int64_t it = 0; it < n; ++it) {
        const int par = parity;
        // pass 1: receive — wait for the neighbours' messages, D2D copies, unpack
        for (int32_t c = 0; c < C && e == hipSuccess; ++c) {
            const Chare& ch = p.chares[(size_t)c];
            hipStream_t s2 = sp(c);
            FaceSet in{}, gh{};
            for (int f = 0; f < 6 && e == hipSuccess; ++f) {
                const int32_t nb = ch.nb[f];
                if (nb < 0) continue;
                const MsgBufs& mine = msg[(size_t)c];
                const MsgBufs& theirs = msg[(size_t)nb];
                e = hipStreamWaitEvent(s2, packed[(size_t)nb], 0);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(base + mine.in[f], base + theirs.out[par][f ^ 1], (size_t)mine.cnt[f] * s,
                                       hipMemcpyDeviceToDevice, s2);
                in.p[f] = base + mine.in[f];
                in.cnt[f] = mine.cnt[f];
                gh.p[f] = base + (size_t)blocks_h[(size_t)ghost_pb[(size_t)c * 6 + f]].off[0] * s;
                gh.cnt[f] = mine.cnt[f];
            }
            if (e == hipSuccess) e = launch_unpack(s, s2, in, gh);
        }
        // pass 2: compute — sweep, pack the new faces, announce them
        for (int32_t c = 0; c < C && e == hipSuccess; ++c) {
            hipStream_t s2 = sp(c);
            const int32_t t0 = tile_lo[(size_t)c], t1 = tile_lo[(size_t)c + 1];
            e = launch_sweep(s, plan.tile[0], plan.tile[1], s2, base, reinterpret_cast<const BlockDev*>(cp(L.blocks)),
                             reinterpret_cast<const TileDev*>(cp(L.tiles)) + t0, t1 - t0, par, res_ptr(), c, c + 1,
                             imb, iters, mode());
            if (e == hipSuccess) e = launch_pack_b(s, s2, base, blocks_h[(size_t)c], par ^ 1, face_out(c, par ^ 1));
            if (e == hipSuccess) e = hipEventRecord(packed[(size_t)c], s2);
        }
        if (e != hipSuccess) return fail(OD_EHIP, std::string("per-chare iteration: ") + hipGetErrorString(e));
        parity ^= 1;
        ++iters;
    }
    // the grid stream waits for every pool stream
    for (auto& s2 : pool) {
        if (e == hipSuccess) e = hipEventRecord(join_ev, s2);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, join_ev, 0);
    }
    if (e != hipSuccess) return fail(OD_EHIP, std::string("per-chare join: ") + hipGetErrorString(e));
    return OD_OK;
}

od_status Grid::iterate(int64_t n) {
    if (n < 0) return fail(OD_EINVAL, "n must be >= 0");
    if (n == 0) return OD_OK;
    switch (cfg.exec) {
        case OD_FUSED: {
            msg_final = false;
            for (int64_t i = 0; i < n;) {
                const int k = two_step && n - i >= 2 ? 2 : 1;
                od_status os = k == 2 ? fused_two(st, parity, iters) : fused_one(st, parity, iters);
                if (os != OD_OK) return os;
                parity ^= 1;
                iters += k;
                i += k;
            }
            return OD_OK;
        }
        case OD_GRAPH:
            msg_final = false;
            return graph_run(n);
        case OD_PERSISTENT:
            msg_final = false;
            return persistent_run(n);
        case OD_MSGDRIVEN:
            return msgdriven_run(n);
        case OD_PER_CHARE:
            msg_final = false;
            return per_chare_run(n);
    }
    return fail(OD_EINVAL, "unknown exec mode");
}

od_status Grid::device_error() {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("sync: ") + hipGetErrorString(e));
    unsigned int err = 0;
    e = hipMemcpy(&err, cp(L.err), 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("read error flag: ") + hipGetErrorString(e));
    if (err & kErrSchedule)
        return fail(OD_ESCHED, "message-driven schedule check failed: a tile's step counter did not advance by one, "
                               "or a tile ran while a neighbour was not within one step (flag " +
                                   std::to_string(err) + ")");
    if (err != 0) return fail(OD_ETIMEDOUT, "a device-side wait exceeded its bound (flag " + std::to_string(err) + ")");
    return OD_OK;
}

od_status Grid::residual(double* r) {
    od_status es = device_error();
    if (es != OD_OK) return es;
    hipError_t e = hipSuccess;
    if (iters == 0) {
        *r = 0.0;
        return OD_OK;
    }
    std::vector<unsigned long long> v((size_t)(2 * nres + 2));
    e = hipMemcpy(v.data(), cp(L.res), v.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("read residual: ") + hipGetErrorString(e));
    unsigned long long m = 0;
    if (msg_final) {
        m = v[(size_t)(2 + (parity & 1))];
    } else {
        for (int32_t s2 = 0; s2 < nres; ++s2) m = std::max(m, v[(size_t)(2 * s2 + parity)]);
    }
    double d;
    std::memcpy(&d, &m, 8);
    *r = d;
    return OD_OK;
}

// ---- global-layout I/O -------------------------------------------------------

od_status Grid::io(void* host, size_t bytes, bool to_host) {
    const int64_t PX = plan.n[0] + 2, PY = plan.n[1] + 2, PZ = plan.n[2] + 2;
    const size_t need = (size_t)PX * PY * PZ * s;
    if (bytes < need) return fail(OD_EINVAL, "buffer of " + std::to_string(bytes) + " bytes, need " + std::to_string(need));
    hipError_t e = hipSuccess;
    if (to_host) {
        // a result of a run whose device-side wait gave up is not returned
        od_status es = device_error();
        if (es != OD_OK) return es;
    } else {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("sync: ") + hipGetErrorString(e));
    }
    const size_t plane = (size_t)PX * PY * s;
    const size_t chunk_planes = std::max<size_t>(1, ((size_t)64 << 20) / plane);
    od_status os = ensure_pinned(chunk_planes * plane);
    if (os != OD_OK) return os;
    if (!to_host) {
        // a write replaces the field: parity 0 becomes current
        os = reset_state();
        if (os != OD_OK) return os;
    }
    for (int64_t k0 = 0; k0 < PZ; k0 += (int64_t)chunk_planes) {
        const int64_t k1 = std::min<int64_t>(PZ, k0 + (int64_t)chunk_planes);
        char* h = static_cast<char*>(host) + (size_t)k0 * plane;
        const size_t nb = (size_t)(k1 - k0) * plane;
        if (to_host) {
            e = launch_gather(s, st, gdev, parity, k0, k1, pinned);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return fail(OD_EHIP, std::string("gather: ") + hipGetErrorString(e));
            std::memcpy(h, pinned, nb);
        } else {
            std::memcpy(pinned, h, nb);
            e = launch_scatter(s, st, gdev, 0, k0, k1, pinned);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return fail(OD_EHIP, std::string("scatter: ") + hipGetErrorString(e));
        }
    }
    return OD_OK;
}

od_status Grid::block_io(int32_t b, void* host, size_t bytes, bool to_host) {
    if (b < 0 || b >= (int32_t)plan.chares.size()) return fail(OD_EINVAL, "block index out of range");
    const BlockDev& B = blocks_h[(size_t)b];
    const size_t row = (size_t)B.ex * s, need = row * B.ey * B.ez;
    if (bytes < need) return fail(OD_EINVAL, "buffer of " + std::to_string(bytes) + " bytes, need " + std::to_string(need));
    hipError_t e = hipSuccess;
    if (to_host) {
        od_status es = device_error();
        if (es != OD_OK) return es;
    } else {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("sync: ") + hipGetErrorString(e));
    }
    const size_t pitch = (size_t)B.py * s, store = (size_t)B.pz * B.ez * s;
    od_status os = ensure_pinned(store);
    if (os != OD_OK) return os;
    char* dev = base + (size_t)(parity ? B.off[1] : B.off[0]) * s;
    char* h = static_cast<char*>(host);
    char* pin = static_cast<char*>(pinned);
    if (to_host) {
        e = hipMemcpyAsync(pin, dev, store, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("read block: ") + hipGetErrorString(e));
        for (int32_t z = 0; z < B.ez; ++z)
            for (int32_t y = 0; y < B.ey; ++y)
                std::memcpy(h + ((size_t)z * B.ey + y) * row, pin + (size_t)z * B.pz * s + (size_t)y * pitch, row);
    } else {
        e = hipMemcpyAsync(pin, dev, store, hipMemcpyDeviceToHost, st);   // keep the row padding
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("write block: ") + hipGetErrorString(e));
        for (int32_t z = 0; z < B.ez; ++z)
            for (int32_t y = 0; y < B.ey; ++y)
                std::memcpy(pin + (size_t)z * B.pz * s + (size_t)y * pitch, h + ((size_t)z * B.ey + y) * row, row);
        e = hipMemcpyAsync(dev, pin, store, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(OD_EHIP, std::string("write block: ") + hipGetErrorString(e));
        faces_packed = false;
        od_status rs = refresh_xexp(parity);
        if (rs != OD_OK) return rs;
    }
    return OD_OK;
}

od_status Grid::read_points(const int64_t* idx, int64_t count, void* host_dst) {
    if (count < 0) return fail(OD_EINVAL, "count must be >= 0");
    if (count == 0) return OD_OK;
    const int64_t total = plan.interior;
    for (int64_t i = 0; i < count; ++i)
        if (idx[i] < 0 || idx[i] >= total) return fail(OD_EINVAL, "point index out of range");
    od_status es = device_error();
    if (es != OD_OK) return es;
    hipError_t e = hipSuccess;
    const size_t need = (size_t)count * (8 + (size_t)s);
    od_status os = ensure_pinned(need);
    if (os != OD_OK) return os;
    std::memcpy(pinned, idx, (size_t)count * 8);
    char* out = static_cast<char*>(pinned) + (size_t)count * 8;
    e = launch_points(s, st, gdev, parity, static_cast<const int64_t*>(pinned), count, out);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(OD_EHIP, std::string("read points: ") + hipGetErrorString(e));
    std::memcpy(host_dst, out, (size_t)count * s);
    return OD_OK;
}

}  // namespace od
