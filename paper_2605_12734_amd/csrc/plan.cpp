// Host planner: decomposition of the global grid into chares, the chare
// "location table" (which chare owns a cell; Section IV pre-fills it so a
// sender knows its destination), cutting chares into sweep tiles, the halo
// map of every tile face, and an XCD-aware launch order.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <numeric>

#include "od_internal.hpp"

namespace od {

namespace {

std::string fmt(const char* f, long long a = 0, long long b = 0, long long c = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, f, a, b, c);
    return buf;
}

// Balanced split of odf into three factors, largest on z, smallest on x.
std::array<int32_t, 3> factor3(int32_t odf) {
    int32_t k = (int32_t)std::llround(std::cbrt((double)odf));
    for (int32_t c = std::max(1, k - 1); c <= k + 1; ++c)
        if ((int64_t)c * c * c == odf) return {c, c, c};
    std::array<int32_t, 3> best = {1, 1, odf};
    double best_score = 1e300;
    for (int32_t a = 1; (int64_t)a * a * a <= odf; ++a) {
        if (odf % a) continue;
        int32_t rest = odf / a;
        for (int32_t b = a; (int64_t)b * b <= rest; ++b) {
            if (rest % b) continue;
            int32_t c = rest / b;
            double score = (double)c / (double)a;
            if (score < best_score) {
                best_score = score;
                best = {a, b, c};
            }
        }
    }
    return best;
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a < 0 ? -a : a;
}

}  // namespace

// Every chare face of a multi-resolution plan that borders a block of
// another cell size is marked in p.mr; across such a face a finer
// neighbour must align to the chare's cells (each averaged patch lies in one
// block).  Uses the owner grid, so it runs after it is built.
std::string plan_resolution_faces(Plan& p) {
    const int32_t C = (int32_t)p.chares.size();
    p.mr.assign((size_t)C * 6, 0);
    const int64_t g = p.gran;
    for (int32_t ci = 0; ci < C; ++ci) {
        const Chare& c = p.chares[(size_t)ci];
        for (int f = 0; f < 6; ++f) {
            const int d = f / 2;
            const int64_t nrm = (f % 2) ? (int64_t)c.u[d] + (int64_t)c.e[d] * c.h : (int64_t)c.u[d] - 1;
            if (nrm < 0 || nrm >= p.n[d]) continue;
            int64_t lo[3], hi[3];
            for (int q = 0; q < 3; ++q) {
                lo[q] = c.u[q];
                hi[q] = (int64_t)c.u[q] + (int64_t)c.e[q] * c.h;
            }
            lo[d] = nrm;
            hi[d] = nrm + 1;
            bool differs = false;
            for (int64_t z = lo[2] / g * g; z < hi[2]; z += g)
                for (int64_t y = lo[1] / g * g; y < hi[1]; y += g)
                    for (int64_t x = lo[0] / g * g; x < hi[0]; x += g) {
                        const int32_t nb = plan_owner(p, std::max(x, lo[0]), std::max(y, lo[1]), std::max(z, lo[2]));
                        const Chare& N = p.chares[(size_t)nb];
                        if (N.h == c.h) continue;
                        differs = true;
                        if (N.h > c.h) continue;
                        for (int q = 0; q < 3; ++q) {
                            if (q == d) continue;
                            const int64_t a = N.u[q], b = (int64_t)N.u[q] + (int64_t)N.e[q] * N.h;
                            if ((a > lo[q] && a % c.h != 0) || (b < hi[q] && b % c.h != 0))
                                return fmt("block %lld: a finer neighbour across face %lld does not align to its cells",
                                           ci, f);
                        }
                    }
            if (differs) p.mr[(size_t)ci * 6 + f] = 1;
        }
    }
    return "";
}

std::string plan_decompose(const od_config& cfg, Plan& p) {
    for (int d = 0; d < 3; ++d) {
        if (cfg.n[d] < 1 || cfg.n[d] > (1 << 20)) return fmt("n[%lld] = %lld out of range [1, 2^20]", d, cfg.n[d]);
        p.n[d] = cfg.n[d];
    }
    if (cfg.dtype != OD_F32 && cfg.dtype != OD_F64) return fmt("dtype %lld is neither OD_F32 nor OD_F64", (long long)cfg.dtype);
    if (cfg.stencil != 0 && cfg.stencil != 7 && cfg.stencil != 5) return fmt("stencil %lld must be 7 or 5", cfg.stencil);
    if (cfg.stencil == 5 && cfg.n[1] != 1) return "the 5-point (2D) stencil needs n[1] == 1";
    p.interior = p.n[0] * p.n[1] * p.n[2];
    p.chares.clear();
    p.owner.clear();

    p.multires = false;
    p.mr.clear();
    if (cfg.block_cell != nullptr && cfg.blocks == nullptr) return "block_cell needs explicit blocks";
    if (cfg.blocks != nullptr || cfg.nblocks > 0) {
        if (cfg.blocks == nullptr || cfg.nblocks < 1) return "blocks/nblocks inconsistent";
        p.regular = false;
        int64_t g = 0;
        for (int d = 0; d < 3; ++d) g = gcd64(g, p.n[d]);
        int64_t vol = 0;
        for (int32_t b = 0; b < cfg.nblocks; ++b) {
            const od_block& B = cfg.blocks[b];
            for (int d = 0; d < 3; ++d) {
                if (B.extent[d] < 1 || B.origin[d] < 0 || (int64_t)B.origin[d] + B.extent[d] > p.n[d])
                    return fmt("block %lld lies outside the domain along dim %lld", b, d);
                g = gcd64(g, B.origin[d]);
                g = gcd64(g, B.extent[d]);
            }
            vol += (int64_t)B.extent[0] * B.extent[1] * B.extent[2];
            const int32_t h = cfg.block_cell ? cfg.block_cell[b] : 1;
            if (h < 1 || h > 1024 || (h & (h - 1)) != 0)
                return fmt("block %lld: cell edge %lld is not a power of two in [1, 1024]", b, h);
            for (int d = 0; d < 3; ++d)
                if (B.origin[d] % h != 0 || B.extent[d] % h != 0)
                    return fmt("block %lld: origin and extent must be multiples of its cell edge %lld", b, h);
            if (h != 1) p.multires = true;
        }
        if (vol != p.interior) return fmt("blocks cover %lld cells, the domain has %lld", vol, p.interior);
        p.gran = (int32_t)g;
        for (int d = 0; d < 3; ++d) p.og[d] = p.n[d] / g;
        int64_t cells = p.og[0] * p.og[1] * p.og[2];
        if (cells > (int64_t(1) << 26)) return fmt("block granularity %lld too fine (owner grid %lld cells)", g, cells);
        p.owner.assign((size_t)cells, -1);
        p.interior = 0;
        for (int32_t b = 0; b < cfg.nblocks; ++b) {
            const od_block& B = cfg.blocks[b];
            Chare c{};
            c.h = cfg.block_cell ? cfg.block_cell[b] : 1;
            for (int d = 0; d < 3; ++d) {
                c.u[d] = B.origin[d];
                c.o[d] = B.origin[d] / c.h;
                c.e[d] = B.extent[d] / c.h;
            }
            p.interior += (int64_t)c.e[0] * c.e[1] * c.e[2];
            for (int f = 0; f < 6; ++f) c.nb[f] = -2;   // not a regular neighbour table
            p.chares.push_back(c);
            for (int64_t z = B.origin[2] / g; z < (B.origin[2] + B.extent[2]) / g; ++z)
                for (int64_t y = B.origin[1] / g; y < (B.origin[1] + B.extent[1]) / g; ++y)
                    for (int64_t x = B.origin[0] / g; x < (B.origin[0] + B.extent[0]) / g; ++x) {
                        int32_t& o = p.owner[(size_t)((z * p.og[1] + y) * p.og[0] + x)];
                        if (o != -1) return fmt("blocks %lld and %lld overlap", o, b);
                        o = b;
                    }
        }
        p.gcell = 0;
        for (const Chare& c : p.chares)
            for (int d = 0; d < 3; ++d) p.gcell = (int32_t)gcd64(gcd64(p.gcell, c.o[d]), c.e[d]);
        if (p.multires) {
            std::string err = plan_resolution_faces(p);
            if (!err.empty()) return err;
        }
        return "";
    }

    p.regular = true;
    int32_t k[3];
    bool have_block = cfg.block[0] > 0 || cfg.block[1] > 0 || cfg.block[2] > 0;
    if (have_block) {
        for (int d = 0; d < 3; ++d) {
            if (cfg.block[d] < 1) return "block extents must all be >= 1 when given";
            k[d] = (int32_t)ceil_div(p.n[d], std::min<int64_t>(cfg.block[d], p.n[d]));
        }
    } else {
        if (cfg.odf < 1) return fmt("odf %lld must be >= 1", cfg.odf);
        // split over the dimensions that have more than one cell
        int act[3], na = 0;
        for (int d = 0; d < 3; ++d)
            if (p.n[d] > 1) act[na++] = d;
        for (int d = 0; d < 3; ++d) k[d] = 1;
        if (na == 3) {
            auto f = factor3(cfg.odf);
            for (int d = 0; d < 3; ++d) k[d] = f[d];
        } else if (na == 2) {
            int32_t a = (int32_t)std::llround(std::sqrt((double)cfg.odf));
            while (a > 1 && cfg.odf % a) --a;
            k[act[0]] = a;
            k[act[1]] = cfg.odf / a;
        } else if (na == 1) {
            k[act[0]] = cfg.odf;
        } else if (cfg.odf != 1) {
            return "a 1x1x1 grid has one chare";
        }
    }
    for (int d = 0; d < 3; ++d) {
        if (k[d] > p.n[d]) return fmt("%lld chares along dim %lld exceed the %lld cells", k[d], d, p.n[d]);
        p.k[d] = k[d];
        int64_t q = p.n[d] / k[d], r = p.n[d] % k[d];
        p.split[d].resize(k[d] + 1);
        for (int32_t i = 0; i <= k[d]; ++i) p.split[d][i] = (int32_t)(i * q + std::min<int64_t>(i, r));
    }
    int64_t nch = (int64_t)k[0] * k[1] * k[2];
    if (nch > (1 << 22)) return fmt("%lld chares exceed the 2^22 limit", nch);
    p.chares.resize((size_t)nch);
    for (int32_t cz = 0; cz < k[2]; ++cz)
        for (int32_t cy = 0; cy < k[1]; ++cy)
            for (int32_t cx = 0; cx < k[0]; ++cx) {
                Chare& c = p.chares[(size_t)((cz * k[1] + cy) * k[0] + cx)];
                int32_t ci[3] = {cx, cy, cz};
                c.h = 1;
                for (int d = 0; d < 3; ++d) {
                    c.o[d] = p.split[d][ci[d]];
                    c.e[d] = p.split[d][ci[d] + 1] - c.o[d];
                    c.u[d] = c.o[d];
                }
                for (int f = 0; f < 6; ++f) {
                    int d = f / 2, s = (f % 2) ? 1 : -1;
                    int32_t cj[3] = {cx, cy, cz};
                    cj[d] += s;
                    c.nb[f] = (cj[d] < 0 || cj[d] >= k[d]) ? -1 : (cj[2] * k[1] + cj[1]) * k[0] + cj[0];
                }
            }
    return "";
}

int32_t plan_owner(const Plan& p, int64_t x, int64_t y, int64_t z) {
    if (x < 0 || y < 0 || z < 0 || x >= p.n[0] || y >= p.n[1] || z >= p.n[2]) return -1;
    if (p.regular) {
        int64_t c[3], v[3] = {x, y, z};
        for (int d = 0; d < 3; ++d) {
            const auto& s = p.split[d];
            c[d] = (int64_t)(std::upper_bound(s.begin(), s.end(), (int32_t)v[d]) - s.begin()) - 1;
        }
        return (int32_t)((c[2] * p.k[1] + c[1]) * p.k[0] + c[0]);
    }
    int64_t g = p.gran;
    return p.owner[(size_t)(((z / g) * p.og[1] + (y / g)) * p.og[0] + (x / g))];
}

void plan_default_tile(const od_config& cfg, Plan& p) {
    if (cfg.tile[0] > 0 && cfg.tile[1] > 0 && cfg.tile[2] > 0) {
        for (int d = 0; d < 3; ++d) p.tile[d] = cfg.tile[d];
        return;
    }
    int32_t emin[3] = {1 << 30, 1 << 30, 1 << 30};
    for (const auto& c : p.chares)
        for (int d = 0; d < 3; ++d) emin[d] = std::min(emin[d], c.e[d]);
    int32_t emax1 = 1;
    for (const auto& c : p.chares) emax1 = std::max(emax1, c.e[1]);
    if (emax1 == 1) {
        // one cell thick in y (2D): long single-row tiles marching z
        p.tile[0] = cfg.dtype == OD_F64 ? 256 : 512;
        p.tile[1] = 1;
        p.tile[2] = std::min<int32_t>(64, std::max<int32_t>(1, emin[2]));
        return;
    }
    // rows of 32 cells (one 16-lane row of 16-byte vectors for f64), 16 rows
    // (f64) / 32 rows (f32), z-columns of up to 32 cells
    p.tile[0] = 32;
    p.tile[1] = cfg.dtype == OD_F64 ? 16 : 32;
    p.tile[2] = std::min<int32_t>(32, std::max<int32_t>(1, emin[2]));
}

namespace {

// Face of a box: ghost slab (global coords, inclusive-exclusive).
struct Box {
    int64_t lo[3], hi[3];
};

// Ghost slab of a tile face in grid units: the tile's tangential extent,
// one unit layer across the face.
Box ghost_slab(const Chare& c, const int32_t o[3], const int32_t e[3], int f) {
    Box b;
    for (int d = 0; d < 3; ++d) {
        b.lo[d] = (int64_t)c.u[d] + (int64_t)o[d] * c.h;
        b.hi[d] = b.lo[d] + (int64_t)e[d] * c.h;
    }
    int d = f / 2;
    if (f % 2 == 0) {
        b.lo[d] -= 1;
        b.hi[d] = b.lo[d] + 1;
    } else {
        b.lo[d] = b.hi[d];
        b.hi[d] = b.lo[d] + 1;
    }
    return b;
}

// Owner of every cell of the slab if unique (>= 0); -1 outside domain;
// -2 if several owners, in which case (*split_dim, *split_at) gives a
// tangential coordinate (global) where the owner changes.
int32_t slab_owner(const Plan& p, const Box& b, int* split_dim, int64_t* split_at) {
    int32_t first = plan_owner(p, b.lo[0], b.lo[1], b.lo[2]);
    if (first < 0) return -1;
    if (p.regular) {
        // Regular chares: owner is separable; check each tangential range.
        for (int d = 0; d < 3; ++d) {
            const auto& s = p.split[d];
            int64_t ci = (std::upper_bound(s.begin(), s.end(), (int32_t)b.lo[d]) - s.begin()) - 1;
            if (b.hi[d] > s[(size_t)ci + 1]) {
                *split_dim = d;
                *split_at = s[(size_t)ci + 1];
                return -2;
            }
        }
        return first;
    }
    int64_t g = p.gran;
    // any coarse cell in the slab interior
    for (int64_t z = b.lo[2] / g * g; z < b.hi[2]; z += g)
        for (int64_t y = b.lo[1] / g * g; y < b.hi[1]; y += g)
            for (int64_t x = b.lo[0] / g * g; x < b.hi[0]; x += g) {
                int64_t q[3] = {std::max(x, b.lo[0]), std::max(y, b.lo[1]), std::max(z, b.lo[2])};
                if (plan_owner(p, q[0], q[1], q[2]) != first) {
                    // owner changes somewhere: split on the first coarse boundary
                    for (int d = 0; d < 3; ++d)
                        if (b.hi[d] - b.lo[d] > 1 && q[d] > b.lo[d]) {
                            *split_dim = d;
                            *split_at = q[d];
                            return -2;
                        }
                }
            }
    return first;
}

}  // namespace

// Two steps per pass read, beyond a tile's face slabs, the slabs two cells
// out, the four (x, y) corner columns and the one-cell ring's rows just
// below and above the tile.  Each must lie in one block (a box in the
// domain's ghost shell along one axis: in the face buffer of one block,
// i.e. its projection onto the boundary layer in one block; along two axes
// it is never read).  Returns true with a cut (*split_dim, *split_at, a
// global coordinate along one of the tile's extents) if one does not.
static bool two_step_straddle(const Plan& p, const Chare& c, const TileHost& t, int* split_dim, int64_t* split_at) {
    Box tb;
    for (int d = 0; d < 3; ++d) {
        tb.lo[d] = (int64_t)c.u[d] + (int64_t)t.o[d] * c.h;
        tb.hi[d] = tb.lo[d] + (int64_t)t.e[d] * c.h;
    }
    std::vector<Box> boxes;
    for (int f = 0; f < 6; ++f) {   // slabs two cells out
        Box b = tb;
        const int d = f / 2;
        b.lo[d] = (f % 2) ? tb.hi[d] + 1 : tb.lo[d] - 2;
        b.hi[d] = b.lo[d] + 1;
        boxes.push_back(b);
    }
    const int64_t xs[2] = {tb.lo[0] - 1, tb.hi[0]}, ys[2] = {tb.lo[1] - 1, tb.hi[1]}, zs[2] = {tb.lo[2] - 1, tb.hi[2]};
    for (int k = 0; k < 4; ++k) {
        Box cz = tb, ax = tb, ay = tb;   // corner column along z; x-arm row along y; y-arm row along x
        cz.lo[0] = xs[k & 1];
        cz.lo[1] = ys[k >> 1];
        ax.lo[0] = xs[k & 1];
        ax.lo[2] = zs[k >> 1];
        ay.lo[1] = ys[k & 1];
        ay.lo[2] = zs[k >> 1];
        cz.hi[0] = cz.lo[0] + 1;
        cz.hi[1] = cz.lo[1] + 1;
        ax.hi[0] = ax.lo[0] + 1;
        ax.hi[2] = ax.lo[2] + 1;
        ay.hi[1] = ay.lo[1] + 1;
        ay.hi[2] = ay.lo[2] + 1;
        boxes.push_back(cz);
        boxes.push_back(ax);
        boxes.push_back(ay);
    }
    for (Box b : boxes) {
        int outs = 0;
        for (int d = 0; d < 3; ++d) {
            if (b.hi[d] <= 0 || b.lo[d] >= p.n[d]) {
                ++outs;
                b.lo[d] = b.lo[d] < 0 ? 0 : p.n[d] - 1;
                b.hi[d] = b.lo[d] + 1;
            }
        }
        if (outs >= 2) continue;
        if (slab_owner(p, b, split_dim, split_at) == -2) return true;
    }
    return false;
}

std::string plan_tiles(Plan& p) {
    for (int d = 0; d < 3; ++d)
        if (p.tile[d] < 1) return "tile extents must be >= 1";
    std::vector<TileHost> out;
    std::vector<TileHost> work;
    p.halo_cells = 0;
    for (int32_t ci = 0; ci < (int32_t)p.chares.size(); ++ci) {
        const Chare& c = p.chares[(size_t)ci];
        for (int32_t z = 0; z < c.e[2]; z += p.tile[2])
            for (int32_t y = 0; y < c.e[1]; y += p.tile[1])
                for (int32_t x = 0; x < c.e[0]; x += p.tile[0]) {
                    TileHost t{};
                    t.chare = ci;
                    t.o[0] = x;
                    t.o[1] = y;
                    t.o[2] = z;
                    t.e[0] = std::min(p.tile[0], c.e[0] - x);
                    t.e[1] = std::min(p.tile[1], c.e[1] - y);
                    t.e[2] = std::min(p.tile[2], c.e[2] - z);
                    work.push_back(t);
                }
        while (!work.empty()) {
            TileHost t = work.back();
            work.pop_back();
            bool split = false;
            for (int f = 0; f < 6 && !split; ++f) {
                Box b = ghost_slab(c, t.o, t.e, f);
                int d = f / 2;
                int64_t lo_local = (f % 2) ? (int64_t)t.o[d] + t.e[d] : (int64_t)t.o[d] - 1;
                if (lo_local >= 0 && lo_local < c.e[d]) {
                    t.kind[f] = 2;
                    t.src[f] = ci;
                } else if (p.multires && p.mr[(size_t)ci * 6 + f]) {
                    t.kind[f] = 3;
                    t.src[f] = f;
                } else {
                    int sd = -1;
                    int64_t sat = 0;
                    int32_t ow = slab_owner(p, b, &sd, &sat);
                    if (ow == -1) {
                        t.kind[f] = 1;
                        t.src[f] = f;
                    } else if (ow >= 0) {
                        t.kind[f] = 0;
                        t.src[f] = ow;
                    } else {
                        // split the tile at grid coordinate sat along sd
                        int64_t cut = (sat - c.u[sd]) / c.h - t.o[sd];
                        if (cut <= 0 || cut >= t.e[sd]) return "internal error: bad tile split";
                        TileHost a = t, bb = t;
                        a.e[sd] = (int32_t)cut;
                        bb.o[sd] = t.o[sd] + (int32_t)cut;
                        bb.e[sd] = t.e[sd] - (int32_t)cut;
                        work.push_back(bb);
                        work.push_back(a);
                        split = true;
                    }
                }
                for (int q = 0; q < 3; ++q) t.g[f][q] = (int32_t)(b.lo[q] >= 0 ? b.lo[q] / c.h : -1);
            }
            if (!split && p.two_step_lines) {
                int sd = -1;
                int64_t sat = 0;
                if (two_step_straddle(p, c, t, &sd, &sat)) {
                    int64_t cut = (sat - c.u[sd]) / c.h - t.o[sd];
                    if (cut <= 0 || cut >= t.e[sd]) return "internal error: bad two-step tile split";
                    TileHost a = t, bb = t;
                    a.e[sd] = (int32_t)cut;
                    bb.o[sd] = t.o[sd] + (int32_t)cut;
                    bb.e[sd] = t.e[sd] - (int32_t)cut;
                    work.push_back(bb);
                    work.push_back(a);
                    split = true;
                }
            }
            if (split) continue;
            for (int f = 0; f < 6; ++f)
                if (t.kind[f] == 0 || t.kind[f] == 3) p.halo_cells += (int64_t)t.e[0] * t.e[1] * t.e[2] / t.e[f / 2];
            out.push_back(t);
        }
    }
    // XCD-aware order: z-major spatial sort, 8 contiguous groups, interleave so
    // that launch index w (dispatched to XCD w % 8) takes group w % 8.
    std::vector<size_t> idx(out.size());
    std::iota(idx.begin(), idx.end(), 0);
    auto gkey = [&](const TileHost& t, int d) {
        const Chare& c = p.chares[(size_t)t.chare];
        return (int64_t)c.u[d] + (int64_t)t.o[d] * c.h;
    };
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        const TileHost& A = out[a];
        const TileHost& B = out[b];
        for (int d = 2; d >= 0; --d) {
            int64_t ka = gkey(A, d), kb = gkey(B, d);
            if (ka != kb) return ka < kb;
        }
        return false;
    });
    size_t T = out.size();
    if (p.xcd_order && p.xcd_boxes && T >= (size_t)kNumXcd) {
        // three rounds of bisection by tile count, each along the longest
        // extent of the part: 8 compact boxes (fewer tiles on a group
        // boundary than 8 thin slabs); z-major order inside each box
        auto bisect8 = [&](size_t lo0, size_t hi0) {
            std::vector<std::pair<size_t, size_t>> parts{{lo0, hi0}};
            for (int round = 0; round < 3; ++round) {
                std::vector<std::pair<size_t, size_t>> next;
                for (auto [lo, hi] : parts) {
                    int64_t mn[3], mx[3];
                    for (int d = 0; d < 3; ++d) {
                        mn[d] = INT64_MAX;
                        mx[d] = INT64_MIN;
                    }
                    for (size_t q = lo; q < hi; ++q)
                        for (int d = 0; d < 3; ++d) {
                            mn[d] = std::min(mn[d], gkey(out[idx[q]], d));
                            mx[d] = std::max(mx[d], gkey(out[idx[q]], d));
                        }
                    int dim = 2;
                    for (int d = 1; d >= 0; --d)
                        if (mx[d] - mn[d] > mx[dim] - mn[dim]) dim = d;
                    std::stable_sort(idx.begin() + (std::ptrdiff_t)lo, idx.begin() + (std::ptrdiff_t)hi,
                                     [&](size_t x, size_t y) { return gkey(out[x], dim) < gkey(out[y], dim); });
                    const size_t mid = lo + (hi - lo) / 2;
                    next.push_back({lo, mid});
                    next.push_back({mid, hi});
                }
                parts.swap(next);
            }
            for (auto [lo, hi] : parts)
                std::stable_sort(idx.begin() + (std::ptrdiff_t)lo, idx.begin() + (std::ptrdiff_t)hi,
                                 [&](size_t x, size_t y) {
                                     for (int d = 2; d >= 0; --d) {
                                         int64_t kx = gkey(out[x], d), ky = gkey(out[y], d);
                                         if (kx != ky) return kx < ky;
                                     }
                                     return false;
                                 });
            return parts;
        };
        // group g: box g of the whole grid, or (xcd_split_chares) box g of
        // every chare, so each chare's work is spread over all groups
        std::vector<std::vector<size_t>> groups((size_t)kNumXcd);
        if (p.xcd_split_chares) {
            std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return out[x].chare < out[y].chare; });
            size_t lo = 0;
            while (lo < T) {
                size_t hi = lo;
                while (hi < T && out[idx[hi]].chare == out[idx[lo]].chare) ++hi;
                const auto parts = bisect8(lo, hi);
                for (int g = 0; g < kNumXcd; ++g)
                    for (size_t q = parts[(size_t)g].first; q < parts[(size_t)g].second; ++q) groups[(size_t)g].push_back(idx[q]);
                lo = hi;
            }
        } else {
            const auto parts = bisect8(0, T);
            for (int g = 0; g < kNumXcd; ++g)
                for (size_t q = parts[(size_t)g].first; q < parts[(size_t)g].second; ++q) groups[(size_t)g].push_back(idx[q]);
        }
        // while every group has a j-th tile it goes to launch position
        // 8j + g; when group sizes differ (by at most one tile per box), the
        // tiles of the last rounds fill the remaining positions in group
        // order and so may run in another group (placement only: a launch
        // takes each tile's group from its position)
        std::vector<TileHost> seq;
        seq.reserve(T);
        size_t maxc = 0;
        for (const auto& gr : groups) maxc = std::max(maxc, gr.size());
        for (size_t j = 0; j < maxc; ++j)
            for (int g = 0; g < kNumXcd; ++g)
                if (j < groups[(size_t)g].size()) seq.push_back(out[groups[(size_t)g][j]]);
        p.tiles.swap(seq);
        return "";
    }
    size_t m = (T + kNumXcd - 1) / kNumXcd;
    std::vector<TileHost> ordered;
    ordered.reserve(T);
    if (!p.xcd_order) {
        for (size_t s = 0; s < T; ++s) ordered.push_back(out[idx[s]]);
    } else {
        for (size_t j = 0; j < m; ++j)
            for (int g = 0; g < kNumXcd; ++g) {
                size_t s = (size_t)g * m + j;
                if (s < T) ordered.push_back(out[idx[s]]);
            }
    }
    p.tiles.swap(ordered);
    return "";
}

}  // namespace od
