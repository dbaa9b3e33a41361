// Internal types shared by the host planner, the runtime and the HIP
// kernels of libod.  Nothing here is part of the public ABI (include/od.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/od.h"

namespace od {

constexpr int kNumXcd = 8;          // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr size_t kAlign = 256;      // byte alignment of every carved region

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Storage of a block: a chare (two parities) or a pseudo-block holding a
// face's ghost values (Dirichlet values of the domain, or the per-chare
// ghost layer of the per-chare baseline), single-buffered (off[0]==off[1]).
// Element (x, y, z) of the block lives at arena[off[p] + x + y*py + z*pz].
struct BlockDev {
    int64_t off[2];
    int64_t pz;
    int32_t py;
    int32_t ex, ey, ez;
    int32_t pad_;
};
static_assert(sizeof(BlockDev) == 48, "BlockDev layout");

// Where a tile reads the ghost slab of one face: block `src`, whose local
// coordinates (sx, sy, sz) correspond to the slab cell next to the tile's
// local (0,0,0) (the slab's normal coordinate is fixed, the tangential
// ones advance with the tile's local coordinates).
struct FaceDev {
    int32_t src;
    int32_t sx, sy, sz;
};

// One unit of sweep work: a box of one chare.
struct TileDev {
    int32_t blk;            // owning chare (index into the block table)
    int32_t x0, y0, z0;     // origin inside the chare
    int32_t nx, ny, nz;     // extent (nx <= TX, ny <= TY of the kernel variant)
    int32_t rslot;          // residual slot (solve index; 0 for a single grid)
    FaceDev f[6];           // x-, x+, y-, y+, z-, z+
};
static_assert(sizeof(TileDev) == 128, "TileDev layout");

// ---------------------------------------------------------------------------
// Host-side plan of one grid.

struct Chare {
    int32_t o[3];           // origin in cells of the chare's own size (= grid units when h == 1)
    int32_t e[3];           // extent in cells
    int32_t nb[6];          // regular decompositions: neighbour chare per face, -1 = domain boundary
    int32_t h = 1;          // cell edge in grid units (multi-resolution blocks)
    int32_t u[3];           // origin in grid units (= o * h)
};

struct TileHost {
    int32_t chare;
    int32_t o[3];           // origin within chare
    int32_t e[3];           // extent
    // per face: kind 0 = chare (src = chare id), 1 = Dirichlet face of the
    // domain (src = face id), 2 = own chare, 3 = resolution-change ghost
    // buffer of the chare's face (src = face id); g = slab start in cells of
    // the chare's size
    int32_t kind[6], src[6], g[6][3];
};

struct Plan {
    int64_t n[3] = {0, 0, 0};
    int32_t k[3] = {0, 0, 0};            // regular split counts (0 if explicit blocks)
    bool regular = true;
    std::vector<int32_t> split[3];       // regular: split points per dimension (k+1 entries)
    std::vector<Chare> chares;
    // explicit blocks: owner grid at granularity gran
    int32_t gran = 0;
    int64_t og[3] = {0, 0, 0};
    std::vector<int32_t> owner;          // (og z, og y, og x) -> chare
    std::vector<TileHost> tiles;         // in launch order (XCD-interleaved)
    int32_t tile[3] = {0, 0, 0};
    bool xcd_order = true;               // group tiles per XCD (else plain spatial order)
    bool xcd_boxes = false;              // XCD groups are 8 compact boxes (else 8 z-slabs)
    bool xcd_split_chares = false;       // with xcd_boxes: 8 boxes per chare, box g of each in group g
    int64_t interior = 0;
    int64_t halo_cells = 0;              // ghost cells read from other chares per sweep
    // multi-resolution blocks
    bool multires = false;               // some chare has h != 1
    std::vector<uint8_t> mr;             // per (chare, face): the face borders another cell size
    int32_t gcell = 0;                   // gcd of chare origins / extents in own cells (tile splits)
    // explicit blocks at one resolution that may run two steps per pass:
    // tiles are also split until every line of cells the pair reads beyond
    // the face slabs lies in one block
    bool two_step_lines = false;
};

// Build the decomposition (chares + owner lookup).  Returns "" or an error.
std::string plan_decompose(const od_config& cfg, Plan& plan);
// Choose a default tile shape for the plan's block shapes and dtype.
void plan_default_tile(const od_config& cfg, Plan& plan);
// Cut chares into tiles of plan.tile, split tiles whose ghost slabs would
// straddle several source chares, fill face sources and order the tiles
// for XCD locality.  Returns "" or an error.
std::string plan_tiles(Plan& plan);
// Owner chare of a global interior cell (-1 outside the domain).
int32_t plan_owner(const Plan& plan, int64_t x, int64_t y, int64_t z);

}  // namespace od
