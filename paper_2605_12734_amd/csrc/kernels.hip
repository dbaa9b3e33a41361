// HIP kernels of libod for gfx950 (CDNA4, wave64).
//
// The hot kernel is the fused 7-point sweep: one workgroup owns a tile of a
// chare (TX x TY cells in the xy-plane, nz planes along z) and marches z
// with a register-resident column (plane below / current / above) while the
// current plane, plus its x/y halo, is staged in LDS.  Halo cells are read
// straight from wherever they live: the chare itself, the neighbouring
// chare's storage (the device-side halo exchange between chares on the same
// GPU, Section IV intra-process path, fused into the compute kernel as in
// the kernel-fusion mitigation cited in Section I) or a Dirichlet face.
// Each addition and the final division by 6 are individually rounded
// (compiled with -ffp-contract=off), in the order x-, x+, y-, y+, z-, z+.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "kernels.hpp"

// Planes of the register column loaded ahead of the one being computed
// (beyond the plane above it).  One plane ahead at 8 waves per SIMD beats
// two ahead at 7 (512^3 fp64 ODF 4096: 455 vs 461 us; fp32 259 vs 266 us).
#ifndef OD_PREFETCH
#define OD_PREFETCH 1
#endif

namespace od {

// ---------------------------------------------------------------------------
// helpers

template <typename T>
struct V16;
template <>
struct V16<double> {
    typedef double __attribute__((ext_vector_type(2))) t;
    static constexpr int N = 2;
};
template <>
struct V16<float> {
    typedef float __attribute__((ext_vector_type(4))) t;
    static constexpr int N = 4;
};

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): idx-th output of the
// stream seeded with `seed` is the finaliser applied to seed + (idx+1)*gamma.
__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
template <typename T>
__device__ __forceinline__ T unit_from_bits(uint64_t h);
template <>
__device__ __forceinline__ double unit_from_bits<double>(uint64_t h) {
    return (double)(h >> 11) * 0x1.0p-53;
}
template <>
__device__ __forceinline__ float unit_from_bits<float>(uint64_t h) {
    return (float)(uint32_t)(h >> 40) * 0x1.0p-24f;
}

__device__ __forceinline__ int32_t owner_of(const LookupDev& lk, int64_t x, int64_t y, int64_t z) {
    if (lk.regular) {
        return (lk.cidx[2][z] * lk.k[1] + lk.cidx[1][y]) * lk.k[0] + lk.cidx[0][x];
    }
    const int64_t g = lk.gran;
    return lk.owner[((z / g) * lk.og[1] + (y / g)) * lk.og[0] + (x / g)];
}

// Workgroup max of a non-negative residual, folded into *slot as the bit
// pattern of a double (monotone for non-negative values).
template <typename T, int NT>
__device__ __forceinline__ void wg_residual(T r, unsigned long long* slot, T* red) {
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(r, off, 64);
        r = o > r ? o : r;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        T m = red[0];
        for (int w = 1; w < NT / 64; ++w) m = red[w] > m ? red[w] : m;
        atomicMax(slot, (unsigned long long)__double_as_longlong((double)m));
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// fused sweep of one tile

#ifndef OD_MERGED_HALO
#define OD_MERGED_HALO 1
#endif

template <typename T, int TX, int TY>
struct SW {
    static constexpr int VX = V16<T>::N;
    static constexpr int LX = TX / VX;        // threads along x
    static constexpr int NT = LX * TY;        // threads per workgroup
    static constexpr int LP = TX + 2 * VX;    // LDS row pitch (interior starts at VX: 16 B aligned)
    static constexpr int LR = TY + 2;         // LDS rows incl. y halo
    static constexpr int LDS = 2 * LP * LR;   // two plane buffers
    static_assert(TX % VX == 0, "TX must be a multiple of the vector width");
    static_assert(NT % 64 == 0 && NT <= 1024, "threads must be whole waves");
};

// XEXP: also write the tile's new x = 0 / x = ex - 1 column into the
// chare's x-column exports (multi-resolution grids; XExpDev).
template <typename T, int TX, int TY, bool XEXP = false>
__device__ __forceinline__ T sweep_tile(T* __restrict__ arena, const BlockDev* __restrict__ blocks,
                                        const TileDev& t, const int parity, T* __restrict__ lds,
                                        const int hints, const XExpDev* __restrict__ xexp = nullptr) {
    using S = SW<T, TX, TY>;
    using VT = typename V16<T>::t;
    constexpr int VX = S::VX;
    constexpr int64_t ES = (int64_t)sizeof(T);
    const int tid = threadIdx.x;
    const int lx = tid % S::LX;
    const int ly = tid / S::LX;
    const int x = lx * VX;
    const int nx = t.nx, ny = t.ny, nz = t.nz;
    const bool rowok = ly < ny;
    int nv = nx - x;
    nv = nv < 0 ? 0 : (nv > VX ? VX : nv);
    if (!rowok) nv = 0;
    const bool act = nv > 0;
    // mode bit 8: the 2D 5-point stencil on the (x, z) plane (no y terms, / 4)
    const bool five = (hints & 0x100) != 0;

    // Addressing: every load is a uniform 64-bit base (per tile and face,
    // held in scalar registers) plus a small 32-bit per-thread byte offset.
    // Lanes outside the tile clamp to its last valid row / vector column, so
    // every thread issues the same loads in the same order each plane and
    // every load is in bounds; only in-tile lanes stage or store results.
    // (A load behind a branch would make the compiler wait for all
    // outstanding loads before using any, serialising the prefetch.)
    const int xc = x < nx ? x : ((nx - 1) / VX) * VX;
    const int lc = ly < ny ? ly : ny - 1;
    const char* __restrict__ ab = reinterpret_cast<const char*>(arena);

    // Block descriptors are read field by field straight from global memory
    // (a dynamically indexed local copy would be placed in scratch).
    const BlockDev* __restrict__ B = blocks + t.blk;
    const int64_t own_py = B->py, own_pz = B->pz;
    const int64_t tile_el = t.x0 + (int64_t)t.y0 * own_py + (int64_t)t.z0 * own_pz;
    const char* own_b = ab + ((parity ? B->off[1] : B->off[0]) + tile_el) * ES;
    char* dst_b = reinterpret_cast<char*>(arena) + ((parity ? B->off[0] : B->off[1]) + tile_el) * ES;
    const uint32_t o_own = (uint32_t)((xc + (int64_t)lc * own_py) * ES);
    // x-column exports of the parity this sweep writes (uniform per tile)
    T* xe_m = nullptr;
    T* xe_p = nullptr;
    int64_t xe_ey = 0;
    if constexpr (XEXP) {
        const XExpDev& X = xexp[t.blk];
        const int64_t om = parity ? X.off[0][0] : X.off[0][1], op = parity ? X.off[1][0] : X.off[1][1];
        if (t.x0 == 0 && om >= 0) xe_m = arena + om;
        if (t.x0 + t.nx == B->ex && op >= 0) xe_p = arena + op;
        xe_ey = B->ey;
    }

    // face f: uniform base at its ghost slab's first cell, uniform plane pitch
    auto face = [&](const FaceDev& f, int64_t* fpy, int64_t* fpz) -> const char* {
        const BlockDev* __restrict__ F = blocks + f.src;
        *fpy = F->py;
        *fpz = F->pz;
        return ab + ((parity ? F->off[1] : F->off[0]) + f.sx + (int64_t)f.sy * F->py + (int64_t)f.sz * F->pz) * ES;
    };
    int64_t zm_py, zm_pz, zp_py, zp_pz, xm_py, xm_pz, xp_py, xp_pz, ym_py, ym_pz, yp_py, yp_pz;
    const char* zm_b = face(t.f[4], &zm_py, &zm_pz);
    const char* zp_b = face(t.f[5], &zp_py, &zp_pz);
    const char* xm_b = face(t.f[0], &xm_py, &xm_pz);
    const char* xp_b = face(t.f[1], &xp_py, &xp_pz);
    const char* ym_b = face(t.f[2], &ym_py, &ym_pz);
    const char* yp_b = face(t.f[3], &yp_py, &yp_pz);
    (void)zm_pz;
    (void)zp_pz;
    (void)ym_py;
    (void)yp_py;
    const uint32_t o_zm = (uint32_t)((xc + (int64_t)lc * zm_py) * ES);
    const uint32_t o_zp = (uint32_t)((xc + (int64_t)lc * zp_py) * ES);
    const uint32_t o_xm = (uint32_t)((int64_t)lc * xm_py * ES);
    const uint32_t o_xp = (uint32_t)((int64_t)lc * xp_py * ES);
    const uint32_t o_y = (uint32_t)((int64_t)xc * ES);

    const bool do_xm = rowok && lx == 0;
    const bool do_xp = rowok && lx == (nx - 1) / VX;
    const bool do_ym = act && ly == 0;
    const bool do_yp = act && ly == ny - 1;
#if OD_MERGED_HALO
    // merged halo loads: the x+ value sits in a lane other than column 0
    // (column 1 for a one-vector tile), the y+ row in a row other than 0
    // (row 1 for a one-row tile of a multi-row variant)
    int nvx = nx - x;
    nvx = nvx < 0 ? 0 : (nvx > VX ? VX : nvx);
    const int xp_lane = (nx - 1) / VX > 0 ? (nx - 1) / VX : 1;
    const int yp_row = TY == 1 ? 0 : (ny - 1 > 0 ? ny - 1 : 1);
    const bool mdo_xp = rowok && lx == xp_lane;
    const bool mdo_ym = nvx > 0 && ly == 0;
    const bool mdo_yp = nvx > 0 && ly == yp_row;
    (void)do_xp;
    (void)do_ym;
    (void)do_yp;
#endif

    auto L = [&](int b, int r, int c) -> T& { return lds[(b * S::LR + r) * S::LP + c]; };
    auto ldv = [](const char* p) -> VT { return *reinterpret_cast<const VT*>(p); };
    auto lds1 = [](const char* p) -> T { return *reinterpret_cast<const T*>(p); };
    // plane zz in [-1, nz]: -1 and nz come from the z faces
    auto plane = [&](int zz) -> VT {
        return zz < 0 ? ldv(zm_b + o_zm) : (zz >= nz ? ldv(zp_b + o_zp) : ldv(own_b + zz * own_pz * ES + o_own));
    };

    // register column pl[k] = plane z-1+k: below, current, above, and PF
    // planes prefetched ahead (clamped to the z+ face)
    constexpr int PF = OD_PREFETCH;
    VT pl[PF + 3];
#pragma unroll
    for (int k = 0; k < PF + 2; ++k) pl[k] = plane(k - 1 <= nz ? k - 1 : nz);
#if OD_MERGED_HALO
    // one load per plane for each halo direction: column-0 lanes read the
    // x- slab, the others the x+ slab (used by lane column xp_lane); with
    // two or more rows, row-0 lanes read the y- slab and the others the y+
    // slab (used by row yp_row)
    const bool xlo = lx == 0, ylo = ly == 0 || TY == 1;
    const char* x_b = xlo ? xm_b + o_xm : xp_b + o_xp;
    const int64_t x_pz = (xlo ? xm_pz : xp_pz) * ES;
    const char* y_b = ylo ? ym_b : yp_b;
    const int64_t y_pz = (ylo ? ym_pz : yp_pz) * ES;
    T hx = lds1(x_b);
    VT hy = ldv(y_b + o_y);
    VT hyp1 = TY == 1 ? ldv(yp_b + o_y) : hy;   // single-row tiles keep a separate y+ load
#else
    VT hym = ldv(ym_b + o_y), hyp = ldv(yp_b + o_y);
    T hxm = lds1(xm_b + o_xm), hxp = lds1(xp_b + o_xp);
#endif

    T r = 0;
    for (int z = 0; z < nz; ++z) {
        const int b = z & 1;
        // prefetch: plane z+PF+1 and the halo of z+1
        const int zq = z + PF + 1 <= nz ? z + PF + 1 : nz;
        pl[PF + 2] = plane(zq);
        const VT& p0 = pl[0];
        const VT& p1 = pl[1];
        const VT& p2 = pl[2];
        const int64_t zh = z + 1 < nz ? z + 1 : z;
#if OD_MERGED_HALO
        const T nx1 = lds1(x_b + zh * x_pz);
        const VT ny1 = ldv(y_b + zh * y_pz + o_y);
        const VT nyp1 = TY == 1 ? ldv(yp_b + zh * yp_pz * ES + o_y) : ny1;
#else
        const VT nym = ldv(ym_b + zh * ym_pz * ES + o_y), nyp = ldv(yp_b + zh * yp_pz * ES + o_y);
        const T nxm = lds1(xm_b + zh * xm_pz * ES + o_xm), nxp = lds1(xp_b + zh * xp_pz * ES + o_xp);
#endif

        // stage plane z with its x/y halo
        if (act) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nv) L(b, ly + 1, VX + x + i) = p1[i];
        }
#if OD_MERGED_HALO
        if (do_xm) L(b, ly + 1, VX - 1) = hx;
        if (mdo_xp) L(b, ly + 1, VX + nx) = hx;
        if (mdo_ym) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nvx) L(b, 0, VX + x + i) = hy[i];
        }
        if (mdo_yp) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nvx) L(b, ny + 1, VX + x + i) = (TY == 1 ? hyp1 : hy)[i];
        }
#else
        if (do_xm) L(b, ly + 1, VX - 1) = hxm;
        if (do_xp) L(b, ly + 1, VX + nx) = hxp;
        if (do_ym) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nv) L(b, 0, VX + x + i) = hym[i];
        }
        if (do_yp) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nv) L(b, ny + 1, VX + x + i) = hyp[i];
        }
#endif
        __syncthreads();

        if (act) {
            VT out;
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                // x neighbours inside the thread's vector come from registers,
                // the ones across its edges from LDS (same values either way)
                const T xm = i > 0 ? p1[i - 1] : L(b, ly + 1, VX + x - 1);
                const T xp = (i < VX - 1 && i + 1 < nv) ? p1[i + 1] : L(b, ly + 1, VX + x + i + 1);
                T s = xm;
                s = s + xp;
                if (!five) {
                    s = s + L(b, ly, VX + x + i);
                    s = s + L(b, ly + 2, VX + x + i);
                }
                s = s + p0[i];
                s = s + p2[i];
                const T v = five ? s / (T)4 : s / (T)6;
                out[i] = v;
                if (i < nv) {
                    T d = v - p1[i];
                    if (d < (T)0) d = -d;
                    if (d > r) r = d;
                }
            }
            if constexpr (XEXP) {
                const int64_t e = (int64_t)(t.y0 + ly) + (int64_t)(t.z0 + z) * xe_ey;
                if (xe_m && lx == 0) xe_m[e] = out[0];
                if (xe_p && x + VX > nx - 1) {
                    T v = out[0];
#pragma unroll
                    for (int i = 1; i < VX; ++i)
                        if (i == nx - 1 - x) v = out[i];
                    xe_p[e] = v;
                }
            }
            // a partial vector only occurs at the chare's row end, where the
            // lanes past nx land in the row's padding: store the whole vector
            VT* o = reinterpret_cast<VT*>(dst_b + (int64_t)z * own_pz * ES + o_own);
            if (hints & 1)
                __builtin_nontemporal_store(out, o);
            else
                *o = out;
        }
#pragma unroll
        for (int k = 0; k < PF + 2; ++k) pl[k] = pl[k + 1];
#if OD_MERGED_HALO
        hy = ny1;
        hyp1 = nyp1;
        hx = nx1;
#else
        hym = nym;
        hyp = nyp;
        hxm = nxm;
        hxp = nxp;
#endif
    }
    __syncthreads();   // LDS planes are reused by the next tile
    return r;
}

template <typename T, int TX, int TY, bool XEXP = false>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY)
k_sweep(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const TileDev* __restrict__ tiles,
        int parity, unsigned long long* __restrict__ res, int zero_lo, int zero_hi,
        const ImbDev imb, int64_t step, int hints, const XExpDev* __restrict__ xexp) {
    using S = SW<T, TX, TY>;
    __shared__ T lds[S::LDS];
    __shared__ T red[S::NT / 64];
    if (blockIdx.x == 0)
        for (int s = zero_lo + (int)threadIdx.x; s < zero_hi; s += S::NT) res[2 * s + parity] = 0ull;
    const TileDev& t = tiles[blockIdx.x];
    const int reps = 1 + imb_extra(imb, step, t.blk);
    T r = 0;
    for (int rep = 0; rep < reps; ++rep)
        r = sweep_tile<T, TX, TY, XEXP>(arena, blocks, t, parity, lds, hints, xexp);
    wg_residual<T, S::NT>(r, &res[2 * t.rslot + (parity ^ 1)], red);
}

// ---------------------------------------------------------------------------
// Two Jacobi steps per pass over memory.  Step t+1 is never stored: a tile
// computes it on itself and on the one-cell ring around it (the cells the
// second step's stencil reads), from time-t values up to two cells out
// (the face slabs one and two deep, the four (x, y) corner columns, and the
// ring's rows just above and below the tile), then computes step t+2 on the
// tile and writes it.  Every value of either step is the same expression in
// the same order as in a single step, so the result is bit-identical; a
// Dirichlet face's first step is its boundary value.
//
// z-march: iteration j in [-1, nz] stages time-t plane j (with its two-cell
// ring) in LDS, computes the first step of plane j (the tile; the ring's
// four arms for 0 <= j < nz) and stages it, then computes the second step
// of plane j - 1 from the staged first-step plane j - 1 and the first-step
// planes j - 2 and j held in registers.  Both LDS planes are double
// buffered, so one barrier per iteration orders every write and read.
//
// Lanes: as in the single step (row ly, VX cells from x = lx * VX) for the
// tile.  The ring is dealt out one cell per lane: lane k < 2 (nx + ny)
// holds one cell of the one-cell ring (x- arm rows, x+ arm rows, y- arm
// cells, y+ arm cells, in that order), keeps its time-t column (planes
// j-1 .. j+1) and computes its first step; lane k < 2 (nx + ny) + 4 also
// loads one cell two out (the same order, then the four corner columns).
// Every lane issues every load (lanes without a ring cell load a valid
// cell of their own and discard it), so no load sits behind a branch.
template <typename T, int TX, int TY>
struct SW2 {
    static constexpr int VX = V16<T>::N;
    static constexpr int LX = TX / VX;
    static constexpr int NT = LX * TY;
    static constexpr int LP = TX + 2 * VX;   // row pitch: column VX + x holds x in [-2, TX + 1]
    static constexpr int TR = TY + 4;        // time-t plane: row y + 2 holds y in [-2, TY + 1]
    static constexpr int UR = TY + 2;        // first-step plane: row y + 1 holds y in [-1, TY]
    static constexpr int LDS = 2 * LP * (TR + UR);
    static_assert(TX % VX == 0 && VX >= 2 && TY >= 2, "two-step tiles need vectors of >= 2 cells and >= 2 rows");
    static_assert(NT >= 2 * (TX + TY) + 4, "one lane per ring cell");
    static_assert(NT % 64 == 0 && NT <= 1024, "threads must be whole waves");
};

template <typename T, int TX, int TY>
__device__ __forceinline__ T sweep2_tile(T* __restrict__ arena, const BlockDev* __restrict__ blocks,
                                         const TileDev& t, const Tile2Dev& t2, const int parity,
                                         T* __restrict__ lds, const int hints) {
    using S = SW2<T, TX, TY>;
    using VT = typename V16<T>::t;
    constexpr int VX = S::VX, LX = S::LX, LP = S::LP;
    constexpr int64_t ES = (int64_t)sizeof(T);
    const int tid = threadIdx.x;
    const int lx = tid % LX, ly = tid / LX, x = lx * VX;
    const int nx = t.nx, ny = t.ny, nz = t.nz;
    const bool rowok = ly < ny;
    int nv = nx - x;
    nv = nv < 0 ? 0 : (nv > VX ? VX : nv);
    if (!rowok) nv = 0;
    const bool act = nv > 0;
    const int xc = x < nx ? x : ((nx - 1) / VX) * VX;
    const int lc = ly < ny ? ly : ny - 1;
    const int dir = t2.dir;
    const char* __restrict__ ab = reinterpret_cast<const char*>(arena);

    // interior: uniform bases, 32-bit per-lane byte offsets
    const BlockDev* __restrict__ B = blocks + t.blk;
    const int64_t own_py = B->py, own_pz = B->pz;
    const int64_t tile_el = t.x0 + (int64_t)t.y0 * own_py + (int64_t)t.z0 * own_pz;
    const char* own_b = ab + ((parity ? B->off[1] : B->off[0]) + tile_el) * ES;
    char* dst_b = reinterpret_cast<char*>(arena) + ((parity ? B->off[0] : B->off[1]) + tile_el) * ES;
    const uint32_t o_own = (uint32_t)((xc + (int64_t)lc * own_py) * ES);
    auto at = [&](const FaceDev& f, int64_t* py, int64_t* pz) -> const char* {
        const BlockDev* __restrict__ F = blocks + f.src;
        *py = F->py;
        *pz = F->pz;
        return ab + ((parity ? F->off[1] : F->off[0]) + f.sx + (int64_t)f.sy * F->py + (int64_t)f.sz * F->pz) * ES;
    };
    int64_t py, pz;
    const char* zm_b = at(t.f[4], &py, &pz);
    const uint32_t o_zm = (uint32_t)((xc + lc * py) * ES);
    const char* zp_b = at(t.f[5], &py, &pz);
    const uint32_t o_zp = (uint32_t)((xc + lc * py) * ES);
    const char* zm2_b = at(t2.r2[4], &py, &pz);
    const uint32_t o_zm2 = (uint32_t)((xc + lc * py) * ES);
    const char* zp2_b = at(t2.r2[5], &py, &pz);
    const uint32_t o_zp2 = (uint32_t)((xc + lc * py) * ES);

    // this lane's ring cells: kind 0..3 = x- arm, x+ arm, y- arm, y+ arm
    // (position p along it), kind 4 = corner p; -1 = none
    auto ring_cell = [&](int k, int* kind, int* p) {
        if (k < ny) {
            *kind = 0;
            *p = k;
        } else if (k < 2 * ny) {
            *kind = 1;
            *p = k - ny;
        } else if (k < 2 * ny + nx) {
            *kind = 2;
            *p = k - 2 * ny;
        } else if (k < 2 * (ny + nx)) {
            *kind = 3;
            *p = k - 2 * ny - nx;
        } else if (k < 2 * (ny + nx) + 4) {
            *kind = 4;
            *p = k - 2 * (ny + nx);
        } else {
            *kind = -1;
            *p = 0;
        }
    };
    int k1, p1, k2, p2;
    ring_cell(tid, &k1, &p1);
    ring_cell(tid, &k2, &p2);
    const bool r1 = k1 >= 0 && k1 < 4;   // holds a one-out cell
    const bool r2 = k2 >= 0;             // holds a two-out or corner cell
    // one-out cell: LDS position, face (Dirichlet bit), column pointers
    int r1y = 0, r1c = 0, r1f = 0;
    const char* r1_b = own_b;            // planes 0 .. nz-1
    const char* r1_lo = own_b;           // plane -1
    const char* r1_hi = own_b;           // plane nz
    int64_t r1_pz = own_pz * ES;
    if (r1) {
        const int side = k1 & 1, along = k1 >> 1;   // along: 0 = x arm (p = row), 1 = y arm (p = x)
        r1f = k1;
        r1y = along ? (side ? ny : -1) : p1;
        r1c = along ? VX + p1 : (side ? VX + nx : VX - 1);
        int64_t lpy, lpz;
        const char* b = at(t.f[k1], &lpy, &lpz);
        r1_b = b + (along ? (int64_t)p1 : p1 * lpy) * ES;
        r1_pz = lpz * ES;
        const char* lo = at(t2.e[along ? 8 + side : 4 + side], &lpy, &lpz);
        r1_lo = lo + (along ? (int64_t)p1 : p1 * lpy) * ES;
        const char* hi = at(t2.e[along ? 10 + side : 6 + side], &lpy, &lpz);
        r1_hi = hi + (along ? (int64_t)p1 : p1 * lpy) * ES;
    }
    // two-out or corner cell
    int r2y = 0, r2c = 0;
    const char* r2_b = own_b;
    int64_t r2_pz = own_pz * ES;
    if (r2) {
        int64_t lpy, lpz;
        if (k2 < 4) {
            const int side = k2 & 1, along = k2 >> 1;
            r2y = along ? (side ? ny + 1 : -2) : p2;
            r2c = along ? VX + p2 : (side ? VX + nx + 1 : VX - 2);
            r2_b = at(t2.r2[k2], &lpy, &lpz) + (along ? (int64_t)p2 : p2 * lpy) * ES;
        } else {
            r2y = (p2 & 2) ? ny : -1;
            r2c = (p2 & 1) ? VX + nx : VX - 1;
            r2_b = at(t2.e[p2], &lpy, &lpz);
        }
        r2_pz = lpz * ES;
    }
    const bool r1dir = r1 && ((dir >> r1f) & 1);

    auto ldv = [](const char* p) -> VT { return *reinterpret_cast<const VT*>(p); };
    auto lds1 = [](const char* p) -> T { return *reinterpret_cast<const T*>(p); };
    auto tpl = [&](int q) -> VT {   // interior plane q in [-2, nz + 1] (uniform)
        if (q >= 0 && q < nz) return ldv(own_b + q * own_pz * ES + o_own);
        if (q == -1) return ldv(zm_b + o_zm);
        if (q == -2) return ldv(zm2_b + o_zm2);
        if (q == nz) return ldv(zp_b + o_zp);
        return ldv(zp2_b + o_zp2);
    };
    auto rl1 = [&](int q) -> T {   // one-out cell, plane q in [-1, nz]
        return lds1(q < 0 ? r1_lo : (q >= nz ? r1_hi : r1_b + q * r1_pz));
    };
    auto lim = [&](int q) { return q < 0 ? 0 : (q > nz - 1 ? nz - 1 : q); };

    T* TL = lds;                      // [2][TR][LP]
    T* UL = lds + 2 * S::TR * LP;     // [2][UR][LP]
    auto tl = [&](int b, int y, int c) -> T& { return TL[(b * S::TR + y + 2) * LP + c]; };
    auto ul = [&](int b, int y, int c) -> T& { return UL[(b * S::UR + y + 1) * LP + c]; };
    // whole-vector LDS accesses at a lane's cells (16-byte aligned: the
    // row pitch and the interior's first column are multiples of VX)
    auto vref = [](T& e) -> VT& { return *reinterpret_cast<VT*>(&e); };

    constexpr int PF = OD_PREFETCH;
    VT tz[PF + 3];   // time-t column of the lane's cells: planes j-1 .. j+PF+1
#pragma unroll
    for (int k = 0; k < PF + 2; ++k) tz[k] = tpl(-2 + k <= nz + 1 ? -2 + k : nz + 1);
    T rc[4];         // one-out cell's column: planes j-1 .. j+2
    rc[0] = rl1(-1);
    rc[1] = rl1(-1);
    rc[2] = rl1(0);
    T c2 = lds1(r2_b);   // two-out / corner cell of plane j
    VT um1, um2;         // first step of planes j-1, j-2
    T r = 0;

    for (int j = -1; j <= nz; ++j) {
        const int b = j & 1;
        const bool inz = j >= 0 && j < nz;
        // loads for later planes
        tz[PF + 2] = tpl(j + PF + 1 <= nz + 1 ? j + PF + 1 : nz + 1);
        rc[3] = rl1(j + 2 > nz ? nz : j + 2);
        const T c2n = lds1(r2_b + lim(j + 1) * r2_pz);

        // stage time-t plane j
        if (nv == VX) {
            vref(tl(b, ly, VX + x)) = tz[1];
        } else if (act) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nv) tl(b, ly, VX + x + i) = tz[1][i];
        }
        if (r1) tl(b, r1y, r1c) = rc[1];
        if (r2 && inz) tl(b, r2y, r2c) = c2;
        __syncthreads();

        // first step of plane j on the tile (Dirichlet z plane: its value)
        const bool zfix = (j < 0 && (dir & 16)) || (j >= nz && (dir & 32));
        VT u;
        {
            const VT ym = vref(tl(b, ly - 1, VX + x)), yp = vref(tl(b, ly + 1, VX + x));
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                const T xm = i > 0 ? tz[1][i - 1] : tl(b, ly, VX + x - 1);
                const T xp = (i < VX - 1 && i + 1 < nv) ? tz[1][i + 1] : tl(b, ly, VX + x + i + 1);
                T s = xm;
                s = s + xp;
                s = s + ym[i];
                s = s + yp[i];
                s = s + tz[0][i];
                s = s + tz[2][i];
                u[i] = zfix ? tz[1][i] : s / (T)6;
            }
        }
        if (nv == VX) {
            vref(ul(b, ly, VX + x)) = u;
        } else if (act) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nv) ul(b, ly, VX + x + i) = u[i];
        }
        // first step of the one-out cell (Dirichlet face: its value)
        if (inz && r1) {
            T s = tl(b, r1y, r1c - 1);
            s = s + tl(b, r1y, r1c + 1);
            s = s + tl(b, r1y - 1, r1c);
            s = s + tl(b, r1y + 1, r1c);
            s = s + rc[0];
            s = s + rc[2];
            ul(b, r1y, r1c) = r1dir ? rc[1] : s / (T)6;
        }

        // second step of plane j - 1
        if (j >= 1) {
            const int c = b ^ 1;
            VT out;
            const VT ym = vref(ul(c, ly - 1, VX + x)), yp = vref(ul(c, ly + 1, VX + x));
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                const T xm = i > 0 ? um1[i - 1] : ul(c, ly, VX + x - 1);
                const T xp = (i < VX - 1 && i + 1 < nv) ? um1[i + 1] : ul(c, ly, VX + x + i + 1);
                T s = xm;
                s = s + xp;
                s = s + ym[i];
                s = s + yp[i];
                s = s + um2[i];
                s = s + u[i];
                const T v = s / (T)6;
                out[i] = v;
                if (i < nv) {
                    T d = v - um1[i];
                    if (d < (T)0) d = -d;
                    if (d > r) r = d;
                }
            }
            if (act) {
                VT* o = reinterpret_cast<VT*>(dst_b + (int64_t)(j - 1) * own_pz * ES + o_own);
                if (hints & 1)
                    __builtin_nontemporal_store(out, o);
                else
                    *o = out;
            }
        }
        um2 = um1;
        um1 = u;
#pragma unroll
        for (int k = 0; k < PF + 2; ++k) tz[k] = tz[k + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) rc[k] = rc[k + 1];
        c2 = c2n;
    }
    __syncthreads();   // LDS planes are reused by the next tile
    return r;
}

template <typename T, int TX, int TY>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY)
k_sweep2(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const TileDev* __restrict__ tiles,
         const Tile2Dev* __restrict__ tiles2, int parity, unsigned long long* __restrict__ res, int zero_lo,
         int zero_hi, int hints) {
    using S = SW2<T, TX, TY>;
    __shared__ __align__(16) T lds[S::LDS];
    __shared__ T red[S::NT / 64];
    if (blockIdx.x == 0)
        for (int s = zero_lo + (int)threadIdx.x; s < zero_hi; s += S::NT) res[2 * s + parity] = 0ull;
    const TileDev& t = tiles[blockIdx.x];
    const T r = sweep2_tile<T, TX, TY>(arena, blocks, t, tiles2[blockIdx.x], parity, lds, hints);
    wg_residual<T, S::NT>(r, &res[2 * t.rslot + (parity ^ 1)], red);
}

// ---------------------------------------------------------------------------
// Synchronisation between workgroups.  On gfx950 an agent-scope release
// writes back the XCD's L2 and an agent-scope acquire invalidates caches, so
// both are issued once per workgroup, never per wave and never inside a
// polling loop: polls are relaxed agent-scope loads (coherent across XCDs,
// no invalidation), and one acquire fence follows the poll that succeeds.
// Before one thread publishes for the workgroup, every wave waits for its
// own stores to complete (s_waitcnt 0) and the workgroup meets at a barrier.

__device__ __forceinline__ int32_t ld_rlx(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wg_stores_done() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// device-wide barrier for cooperative launches: one thread per workgroup
// arrives on a counter (acq_rel: publishes the workgroup's stores) and polls
// the generation.  The wait is bounded; on timeout the error flag is raised
// and every workgroup leaves.
// `reset` (may be null): 8 words the last arrival zeroes before releasing.
__device__ __forceinline__ bool grid_barrier(unsigned int* bar, unsigned int* err, int64_t wait_ticks,
                                             unsigned int* reset = nullptr) {
    __shared__ int ok;
    wg_stores_done();
    if (threadIdx.x == 0) {
        const unsigned int nb = gridDim.x;
        const unsigned int gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        if (arrived == nb - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (reset)
                for (int x = 0; x < 8; ++x) __hip_atomic_store(&reset[x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const int64_t t0 = wall_clock64();
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(8);
                if (wall_clock64() - t0 > wait_ticks ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// hwreg(HW_REG_XCC_ID, 0, 4): the XCD this wave runs on
constexpr int kXccIdReg = ((4 - 1) << 11) | (0 << 6) | 20;

// Tile counters of the persistent form's dynamic schedule: per step parity
// and XCD group one word, each on a 128-byte line of its own (counters of
// different groups never contend for one line).
constexpr int kCtrBase = 64, kCtrStride = 32;
__device__ __forceinline__ unsigned int* tile_ctr(unsigned int* bar, int par, int g) {
    return &bar[kCtrBase + kCtrStride * (8 * par + g)];
}

// Device-wide barrier with one L2 write-back per XCD.  The workgroups of an
// XCD share its L2: each drains its stores into it and arrives on the XCD's
// counter (relaxed); the last of them publishes for all of them with one
// release (write-back of that L2) on the device counter; the last XCD bumps
// the generation.  Bounded wait as in grid_barrier.  bar[32 + x]: arrivals
// of XCD x (zeroed by its last arrival), `xcd_wgs` workgroups on this XCD,
// `nxcd` XCDs with workgroups.  `reset` (may be null): 8 counters,
// kCtrStride words apart, that the releasing workgroup zeroes.
__device__ __forceinline__ bool xcd_barrier(unsigned int* bar, unsigned int* err, int64_t wait_ticks,
                                            unsigned int* reset, int xcd, unsigned int xcd_wgs,
                                            unsigned int nxcd) {
    __shared__ int ok;
    wg_stores_done();
    if (threadIdx.x == 0) {
        const unsigned int gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        bool released = false;
        const unsigned int a = __hip_atomic_fetch_add(&bar[32 + xcd], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == xcd_wgs - 1) {
            __hip_atomic_store(&bar[32 + xcd], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned int g = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (g == nxcd - 1) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (reset)
                    for (int x = 0; x < 8; ++x)
                        __hip_atomic_store(&reset[x * kCtrStride], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) {
            const int64_t t0 = wall_clock64();
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(8);
                if (wall_clock64() - t0 > wait_ticks ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// Persistent launches: each workgroup registers on its XCD (bar[40 + x]
// counts them), then one full barrier makes every count final.
__device__ __forceinline__ bool persist_register(unsigned int* bar, unsigned int* err, int64_t wait_ticks,
                                                 int* s_xcd, unsigned int* s_xwgs, unsigned int* s_nxcd) {
    if (threadIdx.x == 0) {
        *s_xcd = (int)(__builtin_amdgcn_s_getreg(kXccIdReg) & 7);
        __hip_atomic_fetch_add(&bar[40 + *s_xcd], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!grid_barrier(bar, err, wait_ticks)) return false;
    if (threadIdx.x == 0) {
        *s_xwgs = __hip_atomic_load(&bar[40 + *s_xcd], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned int nx = 0;
        for (int x = 0; x < 8; ++x)
            nx += __hip_atomic_load(&bar[40 + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        *s_nxcd = nx;
    }
    __syncthreads();
    return true;
}

// The last workgroup to leave a persistent launch clears the tile counters
// and the per-XCD barrier words for the next launch.
__device__ __forceinline__ void persist_cleanup(unsigned int* bar) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int prev = __hip_atomic_fetch_add(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            for (int x = 0; x < 16; ++x)
                __hip_atomic_store(tile_ctr(bar, x >> 3, x & 7), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int x = 32; x < 48; ++x) __hip_atomic_store(&bar[x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Counter schedules: the workgroup takes its next tile when the current one
// is done, so within an XCD group tiles start in the order workgroups
// finish, as the hardware starts a plain launch's workgroups: neighbouring
// tiles then run in step and share their halo lines in L2.  (Requesting the
// next index while a tile sweeps hides the atomic's latency but lets start
// order drift from finish order by the spread of tile durations: measured
// 8-12 % more HBM reads and up to 8 % longer iterations.)
__device__ __forceinline__ int32_t next_tile(unsigned int* ctr, int32_t* s_idx) {
    __syncthreads();
    if (threadIdx.x == 0)
        *s_idx = (int32_t)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*s_idx);
}

// DYN (a separate instantiation): tiles from per-XCD-group counters.  The
// static form's tile index is uniform by construction, so its tile
// descriptors stay in scalar registers (fewer VGPRs, more waves per SIMD);
// the counter form keeps its own register allocation and occupancy.
// Occupancy the persistent kernel is compiled for: without a request the
// compiler took 106 SGPRs and 73-88 VGPRs (6 or 5 waves per SIMD); asking
// for 7 (fp64) or 8 (fp32) waves fits it in 94 / 78 SGPRs and 70 / 64
// VGPRs without spilling.
template <typename T>
struct PersistWaves {
    static constexpr int value = sizeof(T) == 8 ? 7 : 8;
};

template <typename T, int TX, int TY, bool DYN>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY) __attribute__((amdgpu_waves_per_eu(PersistWaves<T>::value, 8)))
k_persistent(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const TileDev* __restrict__ tiles,
             int32_t ntiles, int parity, int64_t iters, unsigned long long* __restrict__ res, int32_t nres,
             unsigned int* bar, unsigned int* err, const ImbDev imb, int64_t iter_base, int64_t wait_ticks,
             int hints, unsigned long long* __restrict__ stamps, int chunked) {
    using S = SW<T, TX, TY>;
    __shared__ T lds[S::LDS];
    __shared__ T red[S::NT / 64];
    __shared__ int32_t s_idx;
    // XCD groups: launch index w runs on XCD w % 8 (cooperative launches
    // place workgroups like plain ones; checked with HW_REG_XCC_ID) and takes
    // tiles of list positions = w (mod 8), the spatial chunk the planner gave
    // that XCD.  Slots are taken in launch order (w / 8, then + G / 8):
    // assigning them in the order workgroups registered instead measured
    // 20 % more HBM reads.
    const int ng = (gridDim.x >= 8 && gridDim.x % 8 == 0) ? 8 : 1;
    const int xg = (int)(blockIdx.x % ng);
    int32_t first = (int32_t)(blockIdx.x / ng);
    int32_t step_w = (int32_t)(gridDim.x / ng);
    // chunked static schedule: slot k of the group's W slots takes a
    // contiguous run of the group's positions (spatial neighbours in a row)
    int32_t last = INT32_MAX;
    if (!DYN && chunked) {
        const int32_t W = (int32_t)(gridDim.x / ng);
        const int32_t npos = ntiles > xg ? (ntiles - xg + ng - 1) / ng : 0;
        const int32_t k = (int32_t)(blockIdx.x / ng);
        first = (int32_t)((int64_t)npos * k / W);
        last = (int32_t)((int64_t)npos * (k + 1) / W);
        step_w = 1;
    }
    __shared__ int s_xcd;
    __shared__ unsigned int s_xwgs, s_nxcd;
    if (iters > 1 && !persist_register(bar, err, wait_ticks, &s_xcd, &s_xwgs, &s_nxcd)) return;
    for (int64_t it = 0; it < iters; ++it) {
        const int p = parity ^ (int)(it & 1);
        // timeline (stamps != null): first and last workgroup to start
        // iteration it, first and last to finish its tiles
        const bool stamp = stamps && it < kStampIters && threadIdx.x == 0;
        if (stamp) {
            const unsigned long long t0 = (unsigned long long)wall_clock64();
            atomicMin(&stamps[4 * it + 0], t0);
            atomicMax(&stamps[4 * it + 1], t0);
        }
        if (blockIdx.x == 0)
            for (int s = (int)threadIdx.x; s < nres; s += S::NT) res[2 * s + p] = 0ull;
        T r = 0;
        int slot = -1;
        // DYN: tiles of this workgroup's XCD group, taken one at a time from
        // the group's counter when the previous tile is done (see
        // next_tile); otherwise the fixed stride w, w + G, w + 2G, ...
        unsigned int* ctr = tile_ctr(bar, (int)(it & 1), xg);
        if (DYN) {
            if (threadIdx.x == 0)
                s_idx = (int32_t)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
        // uniform by construction: the tile descriptor stays in scalar
        // registers.  idx counts group slots: list position xg + ng * idx
        int32_t idx = DYN ? __builtin_amdgcn_readfirstlane(s_idx) : first;
        for (;;) {
            const int32_t ti = xg + ng * idx;
            if (ti >= ntiles || idx >= last) break;
            const TileDev& t = tiles[ti];
            // (the static list's balanced last round may hold empty entries)
            const int reps = t.nz > 0 ? 1 + imb_extra(imb, iter_base + it, t.blk) : 0;
            T rr = 0;
            for (int rep = 0; rep < reps; ++rep) rr = sweep_tile<T, TX, TY>(arena, blocks, t, p, lds, hints);
            if (slot >= 0 && slot != t.rslot) {
                wg_residual<T, S::NT>(r, &res[2 * slot + (p ^ 1)], red);
                r = 0;
            }
            slot = t.rslot;
            r = rr > r ? rr : r;
            idx = DYN ? next_tile(ctr, &s_idx) : idx + step_w;
        }
        if (slot >= 0) wg_residual<T, S::NT>(r, &res[2 * slot + (p ^ 1)], red);
        if (stamp) {
            const unsigned long long t1 = (unsigned long long)wall_clock64();
            atomicMin(&stamps[4 * it + 2], t1);
            atomicMax(&stamps[4 * it + 3], t1);
        }
        if (it + 1 < iters) {
            // the last arrival clears the counters of the step after next
            if (!xcd_barrier(bar, err, wait_ticks, tile_ctr(bar, (int)((it + 1) & 1), 0), s_xcd, s_xwgs, s_nxcd))
                return;
        }
    }
    persist_cleanup(bar);
}

// Load imbalance in a two-step pass.  A chare drawn heavy at either step
// of the pass re-runs its work extra(t) + extra(t + 1) times before the
// pass: single sweeps from the pass's source parity into its own cells of
// the other parity, the region the pass then overwrites.  Nothing reads
// that region before the pass ends (the pass reads only its source
// parity), so the result is the pair's, and each extra costs one one-step
// sweep, as the re-runs of one-step sweeps do.  The one-step tile needs
// fewer LDS values than the two-step tile with the same threads.
template <typename T, int TX, int TY>
__device__ __forceinline__ void imb_extra_sweeps(T* __restrict__ arena, const BlockDev* __restrict__ blocks,
                                                 const TileDev& t, int parity, T* lds, const ImbDev& imb,
                                                 int64_t step, int hints) {
    static_assert(SW<T, TX, TY>::LDS <= SW2<T, TX, TY>::LDS && SW<T, TX, TY>::NT == SW2<T, TX, TY>::NT,
                  "the one-step tile runs in the two-step tile's workgroup");
    const int extra = imb_extra(imb, step, t.blk) + imb_extra(imb, step + 1, t.blk);
    for (int e = 0; e < extra; ++e) (void)sweep_tile<T, TX, TY>(arena, blocks, t, parity, lds, hints);
}

// Persistent form of the two-step pass (blocks at one resolution):
// `passes` passes of two steps each in one cooperative launch, the same
// per-XCD barrier between passes as k_persistent.  Workgroup w sweeps
// tiles w, w + G, ... of its XCD group, or with DYN takes them one at a
// time from the group's counter as each tile ends (next_tile).  With IMB,
// pass k covers steps iter_base + 2k and iter_base + 2k + 1 of the
// imbalance draw imb (a variant of its own: without it the uniform pass
// keeps its register allocation; the extra sweep's code raised its spill
// from 44 to 60 bytes per lane in fp64).
template <typename T, int TX, int TY, bool DYN, bool IMB>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_persistent2(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const TileDev* __restrict__ tiles,
              const Tile2Dev* __restrict__ tiles2, int32_t ntiles, int parity, int64_t passes,
              unsigned long long* __restrict__ res, int32_t nres, unsigned int* bar, unsigned int* err,
              int64_t wait_ticks, int hints, const ImbDev imb, int64_t iter_base) {
    using S = SW2<T, TX, TY>;
    __shared__ __align__(16) T lds[S::LDS];
    __shared__ T red[S::NT / 64];
    __shared__ int32_t s_idx;
    const int ng = (gridDim.x >= 8 && gridDim.x % 8 == 0) ? 8 : 1;
    const int xg = (int)(blockIdx.x % ng);
    const int32_t first = (int32_t)(blockIdx.x / ng), step_w = (int32_t)(gridDim.x / ng);
    __shared__ int s_xcd;
    __shared__ unsigned int s_xwgs, s_nxcd;
    if (passes > 1 && !persist_register(bar, err, wait_ticks, &s_xcd, &s_xwgs, &s_nxcd)) return;
    for (int64_t it = 0; it < passes; ++it) {
        const int p = parity ^ (int)(it & 1);
        if (blockIdx.x == 0)
            for (int s = (int)threadIdx.x; s < nres; s += S::NT) res[2 * s + p] = 0ull;
        T r = 0;
        int slot = -1;
        unsigned int* ctr = tile_ctr(bar, (int)(it & 1), xg);
        if (DYN) {
            if (threadIdx.x == 0)
                s_idx = (int32_t)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
        int32_t idx = DYN ? __builtin_amdgcn_readfirstlane(s_idx) : first;
        for (;;) {
            const int32_t ti = xg + ng * idx;
            if (ti >= ntiles) break;
            const TileDev& t = tiles[ti];
            if (IMB && t.nz > 0)
                imb_extra_sweeps<T, TX, TY>(arena, blocks, t, p, lds, imb, iter_base + 2 * it, hints);
            const T rr = t.nz > 0 ? sweep2_tile<T, TX, TY>(arena, blocks, t, tiles2[ti], p, lds, hints) : (T)0;
            if (slot >= 0 && slot != t.rslot) {
                wg_residual<T, S::NT>(r, &res[2 * slot + (p ^ 1)], red);
                r = 0;
            }
            slot = t.rslot;
            r = rr > r ? rr : r;
            idx = DYN ? next_tile(ctr, &s_idx) : idx + step_w;
        }
        if (slot >= 0) wg_residual<T, S::NT>(r, &res[2 * slot + (p ^ 1)], red);
        if (it + 1 < passes) {
            if (!xcd_barrier(bar, err, wait_ticks, tile_ctr(bar, (int)((it + 1) & 1), 0), s_xcd, s_xwgs, s_nxcd))
                return;
        }
    }
    persist_cleanup(bar);
}

// Fused two-step pass under load imbalance: k_sweep2 with each heavy
// chare's extra sweeps first (imb_extra_sweeps; the pass covers steps
// `step` and step + 1 of the draw).  A kernel of its own, so the pass of
// uniform work keeps its code.
template <typename T, int TX, int TY>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY)
k_sweep2_imb(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const TileDev* __restrict__ tiles,
             const Tile2Dev* __restrict__ tiles2, int parity, unsigned long long* __restrict__ res, int zero_lo,
             int zero_hi, int hints, const ImbDev imb, int64_t step) {
    using S = SW2<T, TX, TY>;
    __shared__ __align__(16) T lds[S::LDS];
    __shared__ T red[S::NT / 64];
    if (blockIdx.x == 0)
        for (int s = zero_lo + (int)threadIdx.x; s < zero_hi; s += S::NT) res[2 * s + parity] = 0ull;
    const TileDev& t = tiles[blockIdx.x];
    imb_extra_sweeps<T, TX, TY>(arena, blocks, t, parity, lds, imb, step, hints);
    const T r = sweep2_tile<T, TX, TY>(arena, blocks, t, tiles2[blockIdx.x], parity, lds, hints);
    wg_residual<T, S::NT>(r, &res[2 * t.rslot + (parity ^ 1)], red);
}

// Resolution-change ghost fill: one single-wave workgroup per rectangle.
// A ghost cell takes R = r*r source values (r = 1: the coarser or equal
// neighbour's cell; r > 1: the finer neighbour's r x r cells).  The wave
// loads a batch of up to 256 source values with every lane (4 loads in
// flight per lane; values of one cell are consecutive, so lanes read along
// the face's first tangential axis), stages them in LDS, then each lane
// takes every 64th ghost cell of the batch, sums its R values in the fixed
// order (q2 outer, q1 inner) and stores the mean.  (Summing in each lane straight from memory serialised
// the loads: r = 8 cells took 64 dependent loads each.  Batches of 1024
// values were slower: fewer waves fit.)  x-normal faces read the source
// chare's exported column (FillSeg::eoff, written by the sweep) instead of
// one value per row of its storage.
constexpr int kFillLanes = 64, kFillBatch = 256;

// Orders one wave's LDS stores before its later loads (the staging values
// of a fill batch are written and read by the same wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One rectangle of the fill by one wave (lane 0..63); vals: the wave's own
// kFillBatch staging values in LDS.
template <typename T>
__device__ __forceinline__ void fill_segment(T* __restrict__ arena, const BlockDev* __restrict__ blocks,
                                             const FillSeg& S, int parity, int lane, T* __restrict__ vals) {
    {
        const int d = S.d, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const BlockDev& N = blocks[S.src];
        const int64_t eo = parity ? S.eoff[1] : S.eoff[0];
        // x-normal faces read the neighbour's exported column when it has one
        const int64_t nb = eo >= 0 ? eo
                                   : (parity ? N.off[1] : N.off[0]) + (int64_t)S.lay * (d == 0 ? 1 : d == 1 ? N.py : N.pz);
        const int64_t s1 = eo >= 0 ? 1 : (t1 == 0 ? 1 : N.py);
        const int64_t s2 = eo >= 0 ? (int64_t)S.ey : (t2 == 1 ? N.py : N.pz);
        const BlockDev& D = blocks[S.dst];
        const int64_t ds1 = t1 == 0 ? 1 : D.py, ds2 = t2 == 1 ? D.py : D.pz;
        const int32_t rr = S.hc >> S.lhn, r = rr > 1 ? rr : 1, R = r * r;
        const int32_t cells = S.n1 * S.n2;
        const int32_t cpb = kFillBatch / R;   // cells per batch (r <= 16)
        for (int32_t cb = 0; cb < cells; cb += cpb) {
            const int32_t nc = cells - cb < cpb ? cells - cb : cpb, nval = nc * R;
            T v[kFillBatch / kFillLanes];
#pragma unroll
            for (int j = 0; j < kFillBatch / kFillLanes; ++j) {
                // whole waves of loads past the batch are skipped (uniform);
                // in the last one every lane loads a valid (clamped) value
                if (j * kFillLanes < nval) {
                    int32_t f = lane + j * kFillLanes;
                    f = f < nval ? f : nval - 1;
                    const int32_t cell = cb + f / R, q = f % R;
                    const int32_t c1 = cell % S.n1, c2 = cell / S.n1;
                    const int32_t i1 = ((S.r1 + c1 * S.hc) >> S.lhn) + q % r, i2 = ((S.r2 + c2 * S.hc) >> S.lhn) + q / r;
                    v[j] = arena[nb + (int64_t)i1 * s1 + (int64_t)i2 * s2];
                }
            }
#pragma unroll
            for (int j = 0; j < kFillBatch / kFillLanes; ++j)
                if (lane + j * kFillLanes < nval) vals[lane + j * kFillLanes] = v[j];
            wave_lds_sync();
            for (int32_t k = lane; k < nc; k += kFillLanes) {
                T sum = vals[k * R];
                for (int32_t q = 1; q < R; ++q) sum = sum + vals[k * R + q];
                const T m = R > 1 ? sum / (T)R : sum;
                const int32_t cell = cb + k, c1 = cell % S.n1, c2 = cell / S.n1;
                arena[D.off[0] + (int64_t)(S.a1 + c1) * ds1 + (int64_t)(S.a2 + c2) * ds2] = m;
            }
            wave_lds_sync();
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kFillLanes)
k_amr_fill(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const FillSeg* __restrict__ segs,
           int32_t nseg, int parity) {
    __shared__ T vals[kFillBatch];
    for (int32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x)
        fill_segment<T>(arena, blocks, segs[sg], parity, (int)threadIdx.x, vals);
}

// Persistent form of a multi-resolution grid: per iteration every wave of
// the grid fills resolution-change ghost rectangles (rectangle w, w + W,
// ... for global wave w of W; the host lists them by decreasing cost, so
// each wave gets a similar share; claiming them from one counter measured
// 2.7x slower, every wave contending for the one word), the grid meets at
// the per-XCD barrier,
// every workgroup sweeps tiles from its XCD group's counter (claimed as
// each tile ends) and exports the tiles' boundary x-columns for the next
// fill, and the grid meets again.  The fill stages its values in the
// sweep's LDS planes (the barriers separate the two uses).  (Asking for 6
// waves per SIMD, 80 VGPRs instead of the compiler's 87 and 5 waves,
// measured slower: 768^3 octree, 16 cells per leaf edge, 269 against 245 us
// per iteration.)
template <typename T, int TX, int TY>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY)
k_persistent_mr(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const TileDev* __restrict__ tiles,
                int32_t ntiles, int parity, int64_t iters, unsigned long long* __restrict__ res, int32_t nres,
                unsigned int* bar, unsigned int* err, int64_t wait_ticks, int hints,
                const FillSeg* __restrict__ segs, int32_t nseg, const XExpDev* __restrict__ xexp) {
    using S = SW<T, TX, TY>;
    constexpr int NW = S::NT / 64;
    static_assert(S::LDS >= NW * kFillBatch, "each wave stages its fill batch in the sweep's LDS");
    __shared__ __align__(16) T lds[S::LDS];
    __shared__ T red[NW];
    __shared__ int32_t s_idx;
    __shared__ int s_xcd;
    __shared__ unsigned int s_xwgs, s_nxcd;
    const int ng = (gridDim.x >= 8 && gridDim.x % 8 == 0) ? 8 : 1;
    const int xg = (int)(blockIdx.x % ng);
    const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    if (!persist_register(bar, err, wait_ticks, &s_xcd, &s_xwgs, &s_nxcd)) return;
    for (int64_t it = 0; it < iters; ++it) {
        const int p = parity ^ (int)(it & 1);
        if (blockIdx.x == 0)
            for (int s = (int)threadIdx.x; s < nres; s += S::NT) res[2 * s + p] = 0ull;
        for (int32_t sg = (int32_t)blockIdx.x * NW + wave; sg < nseg; sg += (int32_t)gridDim.x * NW)
            fill_segment<T>(arena, blocks, segs[sg], p, lane, lds + wave * kFillBatch);
        // the last arrival clears the tile counters of the next iteration
        // (this iteration's were cleared one iteration ago, or at launch)
        if (!xcd_barrier(bar, err, wait_ticks, tile_ctr(bar, (int)((it + 1) & 1), 0), s_xcd, s_xwgs, s_nxcd))
            return;
        unsigned int* ctr = tile_ctr(bar, (int)(it & 1), xg);
        if (threadIdx.x == 0)
            s_idx = (int32_t)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        int32_t idx = __builtin_amdgcn_readfirstlane(s_idx);
        T r = 0;
        int slot = -1;
        for (;;) {
            const int32_t ti = xg + ng * idx;
            if (ti >= ntiles) break;
            const TileDev& t = tiles[ti];
            const T rr = t.nz > 0 ? sweep_tile<T, TX, TY, true>(arena, blocks, t, p, lds, hints, xexp) : (T)0;
            if (slot >= 0 && slot != t.rslot) {
                wg_residual<T, S::NT>(r, &res[2 * slot + (p ^ 1)], red);
                r = 0;
            }
            slot = t.rslot;
            r = rr > r ? rr : r;
            idx = next_tile(ctr, &s_idx);
        }
        if (slot >= 0) wg_residual<T, S::NT>(r, &res[2 * slot + (p ^ 1)], red);
        if (it + 1 < iters && !xcd_barrier(bar, err, wait_ticks, nullptr, s_xcd, s_xwgs, s_nxcd)) return;
    }
    persist_cleanup(bar);
}

// ---------------------------------------------------------------------------
// message-driven schedulers

// Dependency-counting scheduler of a plain grid.  Tile c may run step k
// once it and every tile it reads halos from have finished step k-1.  The
// finishes count in pend[2c + (k&1)] (counts only grow); the finish that
// completes a multiple of (deg(c) + 1) queues c.  Step k+2 counts reach the
// same word only after c has run step k+1, i.e. after that round is whole.
//
// Queues are per XCD: group g of tiles (t mod 8 == g) lives in the queue of
// XCD g, or, if no workgroup of the launch runs on XCD g, of a present XCD
// (the groups of absent XCDs are dealt round-robin over the present ones).
// The workgroups of an XCD pop from its queue only, so a tile always runs
// on one XCD.  Every tile is queued once per step; a workgroup whose pop
// ticket passes its queue's total leaves.  Every wait is bounded (error
// flag 2).
//
// Publication.  A tile read only by tiles of its own XCD is published by
// the XCD's L2 (every wave drains its stores first).  A tile read from
// another XCD ("cross" tile) needs the L2 written back before its counts
// go out.  An XCD with enough workgroups sets one of them aside as its
// publisher: workers hand finished cross tiles to it through a list, and
// it writes the L2 back once per batch of up to 64 tiles, then counts
// them.  On an XCD with few workgroups each worker writes back itself.
//
// Queue / list x: ring of cap_x (power of two >= its tile count, so a push
// never waits for good) 64-bit slots at
// qslots + off_x (ready queue) and pslots + off_x (cross list).
// Cursor mode (launches with at least kCursorTasksPerWg tiles per
// workgroup): instead of ready queues, each XCD's workgroups claim ready
// tiles in the XCD's spatial order from a shared cursor; a tile's ready
// word holds the step it runs next (relative, plus one), set by the finish
// that completes its count.  Tiles that share halo lines then run at the
// same time, as in a fused launch, and find those lines in the XCD's L2.
// With fewer tiles per workgroup most probes would miss, and the queues
// are used.
constexpr int32_t kCursorTasksPerWg = 4;
__device__ __forceinline__ bool use_cursor(int32_t ntiles, int32_t grid) {
    return ntiles >= kCursorTasksPerWg * grid;
}

struct QueueMap {
    int32_t phys[8];   // queue (XCD) of tile group g
    int32_t off[8];    // first slot of queue x
    int32_t cap[8];    // slots of queue x (0 if XCD x is absent)
    int32_t n[8];      // tiles of queue x
    int32_t pre[8];    // queue position of the first tile of group g
};

constexpr int kQcHead = 0, kQcTail = 8, kQcMask = 16, kQcWgs = 24, kQcPTail = 32, kQcCross = 40, kQcLive = 48;
// An XCD sets a workgroup aside as publisher when it has at least 8 and
// at least two tasks per workgroup and step: then throughput matters more
// than the extra hop on the critical path (a small launch is bound by the
// latency of its dependency chain, and writes back itself).
__device__ __forceinline__ bool use_publisher(uint32_t wgs, uint32_t ntasks) {
    return wgs >= 8u && ntasks >= 2u * wgs;
}

__device__ __forceinline__ void queue_map(uint32_t mask, int32_t ntiles, QueueMap& m) {
    int32_t pres[8], np = 0;
    for (int x = 0; x < 8; ++x)
        if ((mask >> x) & 1u) pres[np++] = x;
    for (int x = 0; x < 8; ++x) m.n[x] = 0;
    for (int g = 0; g < 8; ++g) {
        m.phys[g] = ((mask >> g) & 1u) ? g : pres[g % np];
        m.pre[g] = m.n[m.phys[g]];
        m.n[m.phys[g]] += ntiles > g ? (ntiles - g + 7) / 8 : 0;
    }
    int32_t o = 0;
    for (int x = 0; x < 8; ++x) {
        int32_t c = 0;
        if ((mask >> x) & 1u) {
            c = 1;
            while (c < m.n[x]) c *= 2;
        }
        m.off[x] = o;
        m.cap[x] = c;
        o += c;
    }
}

struct NoQuit {
    __device__ bool operator()() const { return false; }
};

// A slot holds a 24-bit sequence (bits 63..40) and a 40-bit payload: ticket
// t's entry is filled when the sequence is (t+1) mod 2^24 and free for
// ticket t when it is t mod 2^24.  A launch takes fewer than 2^24 tickets
// per queue (the host splits longer runs), so no two tickets alias.
constexpr unsigned long long kSlotPayload = (1ull << 40) - 1;
__device__ __forceinline__ unsigned long long slot_word(uint32_t seq, unsigned long long payload) {
    return ((unsigned long long)(seq & 0xFFFFFFu) << 40) | payload;
}
__device__ __forceinline__ uint32_t slot_seq(unsigned long long v) { return (uint32_t)(v >> 40); }

// Append a payload to ring (base, cap) at a fresh ticket of *tail.  Gives
// up (false) when quit() turns true, or raises error flag 2 on timeout.
template <class Quit = NoQuit>
__device__ __forceinline__ bool ring_push(const MsgArgs& a, unsigned long long* q, uint32_t cap, unsigned int* tail,
                                          unsigned long long payload, Quit quit = Quit()) {
    const uint32_t t = __hip_atomic_fetch_add(tail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long* sl = &q[t & (cap - 1u)];
    const int64_t t0 = wall_clock64();
    while (slot_seq(__hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != (t & 0xFFFFFFu)) {
        if (quit()) return false;
        if (wall_clock64() - t0 > a.wait_ticks) {
            __hip_atomic_fetch_or(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(sl, slot_word(t + 1u, payload), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Take ticket t's payload from ring (base, cap): wait until it is filled,
// free the slot for ticket t + cap.  Returns -1 when quit() turns true, or
// on timeout or a raised error (then error flag 2 is raised).
template <class Quit = NoQuit>
__device__ __forceinline__ int64_t ring_take(const MsgArgs& a, unsigned long long* q, uint32_t cap, uint32_t t,
                                             Quit quit = Quit()) {
    unsigned long long* sl = &q[t & (cap - 1u)];
    const int64_t t0 = wall_clock64();
    for (;;) {
        const unsigned long long v = __hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (slot_seq(v) == ((t + 1u) & 0xFFFFFFu)) {
            __hip_atomic_store(sl, slot_word(t + cap, 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return (int64_t)(v & kSlotPayload);
        }
        if (quit()) return -1;
        if (wall_clock64() - t0 > a.wait_ticks ||
            __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            __hip_atomic_fetch_or(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Schedule check: wait a seeded 0..a.pert_ticks wall-clock ticks (bounded).
__device__ __forceinline__ void pert_delay(const MsgArgs& a, uint64_t salt, uint64_t idx) {
    if (a.pert_ticks <= 0) return;
    const int64_t d = (int64_t)(sm64(a.seed ^ salt, idx) % (uint64_t)(a.pert_ticks + 1));
    const int64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < d) __builtin_amdgcn_s_sleep(1);
}

// Schedule check (wave 0): every tile that tile c reads halos from (dep
// list) has finished step `step` - 1 and not yet step `step` + 1, i.e. its
// step counter is step or step + 1.  Raises kErrSchedule otherwise.
__device__ __forceinline__ void check_window(const MsgArgs& a, int32_t c, int32_t step) {
    const int lane = threadIdx.x;
    bool bad = false;
    for (int32_t i = a.dep_ptr[c] + lane; i < a.dep_ptr[c + 1]; i += 64) {
        const int32_t dv = ld_rlx(&a.done[a.dep_idx[i]]);
        bad |= dv < step || dv > step + 1;
    }
    if (__ballot(bad) != 0ull && lane == 0)
        __hip_atomic_fetch_or(a.err, kErrSchedule, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Plain-grid payload: the tile and the step it runs next, relative to the
// launch's first step d0 (a launch runs fewer than 2^16 steps).
__device__ __forceinline__ unsigned long long task_payload(int32_t tile, int32_t rel) {
    return ((unsigned long long)(uint32_t)tile << 16) | (uint32_t)rel;
}

// Count finish ns of tile c for its i-th counter (i = 0: c itself, else its
// (i-1)-th reader); queue the tile whose counter this completes, for the
// step that reads ns.
__device__ __forceinline__ void count_finish(const MsgArgs& a, const QueueMap& m, int32_t c, int32_t ns, int32_t d0,
                                             int32_t i, bool cursor) {
    const int32_t u = i == 0 ? c : a.dep_idx[a.dep_ptr[c] + i - 1];
    const int32_t need = a.dep_ptr[u + 1] - a.dep_ptr[u] + 1;
    const int32_t prev = __hip_atomic_fetch_add(&a.pend[2 * u + (ns & 1)], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((prev + 1) % need == 0) {
        if (cursor) {
            __hip_atomic_store(&a.ready[u], ns - d0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const int x = m.phys[u & 7];
            ring_push(a, a.qslots + m.off[x], (uint32_t)m.cap[x], &a.qhead[kQcTail + x], task_payload(u, ns - d0));
        }
    }
}

// Publisher of XCD x (wave 0 only): take the cross tiles workers list, in
// batches of up to 64, write the L2 back once per batch, then count them.
__device__ __forceinline__ void publisher_loop(const MsgArgs& a, const QueueMap& m, int x, uint32_t want, int32_t d0,
                                               bool cursor) {
    const int lane = threadIdx.x;
    unsigned long long* pl = a.pslots + m.off[x];
    const uint32_t cap = (uint32_t)m.cap[x];
    uint32_t h = 0;
    int64_t idle = wall_clock64();
    while (h < want) {
        uint32_t e = __hip_atomic_load(&a.qhead[kQcPTail + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (e > want) e = want;
        if (e == h) {
            if (wall_clock64() - idle > a.wait_ticks ||
                __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                if (lane == 0) __hip_atomic_fetch_or(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        if (e - h > 64u) e = h + 64u;
        int64_t pay = -1;
        if ((uint32_t)lane < e - h) pay = ring_take(a, pl, cap, h + (uint32_t)lane);
        if (__ballot(pay < 0 && (uint32_t)lane < e - h) != 0ull) return;   // timed out (flag raised)
        // every listed worker drained its stores into this XCD's L2 before
        // listing: one write-back publishes the whole batch
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (pay >= 0) {
            const int32_t c = (int32_t)(pay >> 16), ns = d0 + (int32_t)(pay & 0xFFFF);
            const int32_t cnt = a.dep_ptr[c + 1] - a.dep_ptr[c] + 1;
            for (int32_t i = 0; i < cnt; ++i) count_finish(a, m, c, ns, d0, i, cursor);
        }
        h = e;
        idle = wall_clock64();
    }
}

// Tile (plain grid) or launch position (serving) at cursor position p of
// XCD x: the positions of the groups dealt to x, in order.
__device__ __forceinline__ int32_t cursor_item(const QueueMap& m, int32_t n, int x, int32_t p) {
    int32_t u = -1;
    for (int g = 0; g < 8; ++g) {
        const int32_t ng = n > g ? (n - g + 7) / 8 : 0;
        if (m.phys[g] == x && p >= m.pre[g] && p < m.pre[g] + ng) u = g + 8 * (p - m.pre[g]);
    }
    return u;
}

// Cursor mode: take positions from XCD x's cursor until one holds a ready
// word, exchange it for 0 (exactly one claimer wins) and return the task
// payload (plain grid: the tile and its relative step; serving: the
// position).  Plain grids stop (-1) once every tile of the XCD has been
// claimed for its last step (counted in qhead[kQcTail + x]); serving stops
// when quit() turns true.  A run of misses backs off; the wait is bounded
// (error flag 2).
template <class Quit>
__device__ __forceinline__ int64_t cursor_claim(const MsgArgs& a, const QueueMap& m, int x, Quit quit) {
    unsigned int* qc = a.qhead;
    const bool plain = a.tile_list == nullptr;
    const int64_t t0 = wall_clock64();
    int32_t misses = 0;
    if (m.n[x] == 0) return -1;
    for (;;) {
        const int32_t p = (int32_t)(__hip_atomic_fetch_add(&qc[kQcHead + x], 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT) %
                                    (uint32_t)m.n[x]);
        const int32_t u = cursor_item(m, a.ntiles, x, p);
        // serving reads the word first (most positions of a launch hold no
        // ready solve step); plain grids exchange at once
        const int32_t v = u >= 0 && (plain || ld_rlx(&a.ready[u]) != 0)
                              ? __hip_atomic_exchange(&a.ready[u], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : 0;
        if (v != 0) {
            if (!plain) return u;
            if (v == a.qsteps) __hip_atomic_fetch_add(&qc[kQcTail + x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return (int64_t)task_payload(u, v - 1);
        }
        if (plain ? __hip_atomic_load(&qc[kQcTail + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (uint32_t)m.n[x]
                  : quit())
            return -1;
        if (++misses > 8) __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() - t0 > a.wait_ticks ||
            __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            __hip_atomic_fetch_or(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
    }
}

template <int NT, class SweepFn>
__device__ __forceinline__ void queue_loop(const MsgArgs& a, SweepFn sweep, double* red) {
    __shared__ QueueMap s_m;
    __shared__ int32_t s_tile, s_rel, s_stop, s_role;
    const int32_t G = gridDim.x, w = blockIdx.x;
    unsigned int* qc = a.qhead;
    const int x = (int)(__builtin_amdgcn_s_getreg(kXccIdReg) & 7);
    // every tile starts the launch at step d0 and ends it at tgt
    const int32_t tgt = ld_rlx(&a.target[0]), d0 = tgt - a.qsteps;
    const int claim_mode = a.sched & 3, pub_mode = (a.sched >> 2) & 3;
    const bool cursor = claim_mode == 0 ? use_cursor(a.ntiles, G) : claim_mode == 1;
    // launch start: find the XCDs this launch runs on (and how many
    // workgroups each has), lay out the queues, mark the cross tiles and
    // queue every tile for its next step
    if (threadIdx.x == 0) {
        const uint32_t rank = __hip_atomic_fetch_add(&qc[kQcWgs + x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_or(&qc[kQcMask], 1u << x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_role = rank == 0 ? 1 : 0;
    }
    if (!grid_barrier(a.bar, a.err, a.wait_ticks)) return;
    if (threadIdx.x == 0) queue_map(__hip_atomic_load(&qc[kQcMask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), a.ntiles, s_m);
    __syncthreads();
    const int64_t stride = (int64_t)G * NT, gtid = (int64_t)w * NT + threadIdx.x;
    for (int64_t i = gtid; i < a.ntiles; i += stride) {
        const int32_t u = (int32_t)i, xu = s_m.phys[u & 7], pos = s_m.pre[u & 7] + (u >> 3);
        if (cursor)
            a.ready[u] = 1;   // every tile runs step d0 first
        else
            a.qslots[s_m.off[xu] + pos] = slot_word((uint32_t)pos + 1u, task_payload(u, 0));
        a.pend[2 * u] = 0;
        a.pend[2 * u + 1] = 0;
        uint8_t cross = 0;
        for (int32_t q = a.dep_ptr[u]; q < a.dep_ptr[u + 1]; ++q) cross |= s_m.phys[a.dep_idx[q] & 7] != xu;
        a.xpub[u] = cross;
        if (cross) __hip_atomic_fetch_add(&qc[kQcCross + xu], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int y = 0; y < 8; ++y) {
        // (cursor mode keeps its ready words in this region)
        if (!cursor)
            for (int64_t i = s_m.n[y] + gtid; i < s_m.cap[y]; i += stride)
                a.qslots[s_m.off[y] + i] = slot_word((uint32_t)i, 0);
        for (int64_t i = gtid; i < s_m.cap[y]; i += stride) a.pslots[s_m.off[y] + i] = slot_word((uint32_t)i, 0);
    }
    if (!cursor && w == 0 && threadIdx.x < 8) qc[kQcTail + threadIdx.x] = (uint32_t)s_m.n[threadIdx.x];
    // schedule check: each XCD's cursor starts at a seeded position
    const bool check = (a.hints & kHintCheck) != 0;
    if (cursor && check && w == 0 && threadIdx.x < 8 && s_m.n[threadIdx.x] > 0)
        qc[kQcHead + threadIdx.x] = (uint32_t)(sm64(a.seed ^ 0x637572736F72ull, (uint64_t)d0 * 8 + threadIdx.x) %
                                               (uint64_t)s_m.n[threadIdx.x]);
    if (!grid_barrier(a.bar, a.err, a.wait_ticks)) return;

    const uint32_t xwgs = __hip_atomic_load(&qc[kQcWgs + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // a publisher needs at least one worker beside it on its XCD
    const bool haspub = pub_mode == 0 ? use_publisher(xwgs, (uint32_t)s_m.n[x]) : (pub_mode == 1 && xwgs >= 2u);
    if (haspub && s_role) {
        if (threadIdx.x >= 64 || a.qsteps < 2) return;
        const uint32_t ncross = __hip_atomic_load(&qc[kQcCross + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        publisher_loop(a, s_m, x, ncross * (uint32_t)(a.qsteps - 1), d0, cursor);
        return;
    }
    const uint32_t total = (uint32_t)s_m.n[x] * (uint32_t)a.qsteps;
    unsigned long long* q = a.qslots + s_m.off[x];
    const uint32_t cap = (uint32_t)s_m.cap[x];
    uint32_t ntask = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int64_t pay = -1;
            int32_t stop = 0;
            if (check) pert_delay(a, 0x636C61696Dull, ((uint64_t)w << 32) + ntask++);
            if (cursor) {
                if (total == 0) stop = 1;
                else pay = cursor_claim(a, s_m, x, [] { return false; });
            } else {
                const uint32_t t =
                    __hip_atomic_fetch_add(&qc[kQcHead + x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (t < total) pay = ring_take(a, q, cap, t);
            }
            if (pay < 0) stop = 1;
            // acquire side: the neighbours' step data
            else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_tile = pay < 0 ? -1 : (int32_t)(pay >> 16);
            s_rel = pay < 0 ? 0 : (int32_t)(pay & 0xFFFF);
            s_stop = stop;
        }
        __syncthreads();
        if (s_stop) break;
        // uniform across the workgroup: keep the tile descriptor in scalar
        // registers; the step travels with the task
        const int32_t c = __builtin_amdgcn_readfirstlane(s_tile);
        const int32_t step = d0 + __builtin_amdgcn_readfirstlane(s_rel);
        // the tile's step counter: `step` steps done so far (its last
        // finish stored it before counting, on this XCD); checked after the
        // sweep, so the load overlaps it
        const int32_t seen = __builtin_amdgcn_readfirstlane(ld_rlx(&a.done[c]));
        if (check && threadIdx.x < 64) check_window(a, c, step);
        const double r = sweep(c, step);
        const int32_t ns = step + 1;
        if (ns == tgt) wg_residual<double, NT>(r, &a.res[ns & 1], red);
        if (threadIdx.x == 0) {
            if (seen != step) __hip_atomic_fetch_or(a.err, kErrSchedule, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.done[c], ns, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        wg_stores_done();
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const bool cross = a.xpub[c] != 0;
            const bool listed = cross && haspub && ns < tgt;
            if (check && lane == 0) pert_delay(a, 0x7075626C697368ull, ((uint64_t)c << 20) + (uint64_t)step);
            if (lane == 0) {
                // no publisher on this XCD: write the L2 back before counting
                // (the launch's end publishes its last step)
                if (cross && !haspub && ns < tgt) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                if (listed) ring_push(a, a.pslots + s_m.off[x], cap, &qc[kQcPTail + x], task_payload(c, ns - d0));
            }
            if (ns < tgt && !listed) {
                const int32_t cnt = a.dep_ptr[c + 1] - a.dep_ptr[c] + 1;
                for (int32_t i = lane; i < cnt; i += 64) count_finish(a, s_m, c, ns, d0, i, cursor);
            }
        }
        __syncthreads();
    }
}

// Serving with the same queues.  Launch positions u index the launch's
// tile list (solves back to back, each padded to a multiple of 8, so a
// solve keeps its XCD groups); counters and steps are per tile id.
// Differences from a plain grid:
//  * decision steps (multiples of the solve's check_every, and its cap):
//    those finishes are not counted; the last tile of the solve to finish
//    one evaluates the residual, and either stops the solve or opens its
//    gate and queues every tile of the solve;
//  * a launch ends early when the host asks (yield) or every solve has
//    stopped, so queued tasks and uncounted finishes may be dropped.  At
//    launch start the counters are therefore rebuilt from the step
//    counters (the finishes each tile's current and next round already
//    have) and every ready tile is queued.
// Workgroup 0 forwards the host's yield flag to the device word, at most
// once per yield_poll_ticks (every workgroup reads the device word).
__device__ __forceinline__ void serve_poll_yield(const MsgArgs& a, int64_t& last_poll) {
    if (blockIdx.x != 0) return;
    const int64_t now = wall_clock64();
    if (now - last_poll < a.yield_poll_ticks) return;
    last_poll = now;
    if (__hip_atomic_load(a.yield_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)
        __hip_atomic_store(a.yield_dev, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The launch is ending: the host asked to yield, or every solve stopped.
struct ServeQuit {
    const MsgArgs* a;
    int64_t* last_poll;
    __device__ bool operator()() const {
        serve_poll_yield(*a, *last_poll);
        return __hip_atomic_load(a->yield_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
               __hip_atomic_load(&a->qhead[kQcLive], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    }
};

__device__ __forceinline__ bool serve_decision(const MsgArgs& a, int32_t sv, int32_t ns) {
    const int32_t ce = a.check_every[sv];
    return (ce > 0 && ns % ce == 0) || ns >= a.target[sv];
}

// Count ordinary finish ns of tile t for counter i (0 = t, else its
// (i-1)-th reader) and queue the reader whose round this completes.
__device__ __forceinline__ void serve_count(const MsgArgs& a, const QueueMap& m, int32_t t, int32_t ns, int32_t i,
                                            bool cursor) {
    const int32_t v = i == 0 ? t : a.dep_idx[a.dep_ptr[t] + i - 1];
    const int32_t need = a.dep_ptr[v + 1] - a.dep_ptr[v] + 1;
    const int32_t prev = __hip_atomic_fetch_add(&a.pend[2 * v + (ns & 1)], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((prev + 1) % need == 0) {
        const int32_t u = a.tile_pos[v];
        if (cursor) {
            __hip_atomic_store(&a.ready[u], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const int x = m.phys[u & 7];
            int64_t lp = 0;
            ring_push(a, a.qslots + m.off[x], (uint32_t)m.cap[x], &a.qhead[kQcTail + x], u, ServeQuit{&a, &lp});
        }
    }
}

// Serving in cursor mode: a tile is ready when its position's ready word
// is 1 (its step lives in done[]).
__device__ __forceinline__ void serve_ready(const MsgArgs& a, const QueueMap& m, int32_t u, bool cursor,
                                            const ServeQuit& quit) {
    if (cursor) {
        __hip_atomic_store(&a.ready[u], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        const int x = m.phys[u & 7];
        ring_push(a, a.qslots + m.off[x], (uint32_t)m.cap[x], &a.qhead[kQcTail + x], u, quit);
    }
}

template <int NT, class SweepFn>
__device__ __forceinline__ void serve_loop(const MsgArgs& a, SweepFn sweep, double* red) {
    __shared__ QueueMap s_m;
    __shared__ int32_t s_u, s_stop, s_role;
    const int32_t G = gridDim.x, w = blockIdx.x;
    unsigned int* qc = a.qhead;
    const int x = (int)(__builtin_amdgcn_s_getreg(kXccIdReg) & 7);
    int64_t last_poll = 0;
    const ServeQuit quit{&a, &last_poll};
    const bool cursor = use_cursor(a.ntiles, G);
    if (threadIdx.x == 0) {
        const uint32_t rank = __hip_atomic_fetch_add(&qc[kQcWgs + x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_or(&qc[kQcMask], 1u << x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_role = rank == 0 ? 1 : 0;
    }
    if (!grid_barrier(a.bar, a.err, a.wait_ticks)) return;
    if (threadIdx.x == 0) queue_map(__hip_atomic_load(&qc[kQcMask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), a.ntiles, s_m);
    __syncthreads();
    // launch start, part 1: free every slot; per position the cross flag,
    // the rebuilt counters and whether the tile is ready (bit 1; cursor
    // mode: its ready word, which lives in the ready-queue region)
    const int64_t stride = (int64_t)G * NT, gtid = (int64_t)w * NT + threadIdx.x;
    for (int y = 0; y < 8; ++y)
        for (int64_t i = gtid; i < s_m.cap[y]; i += stride) {
            if (!cursor) a.qslots[s_m.off[y] + i] = slot_word((uint32_t)i, 0);
            a.pslots[s_m.off[y] + i] = slot_word((uint32_t)i, 0);
        }
    for (int64_t i = gtid; i < a.ntiles; i += stride) {
        const int32_t u = (int32_t)i, t = a.tile_list[u];
        if (cursor) a.ready[u] = 0;
        if (t < 0) continue;
        const int32_t sv = a.tile_solve[t], d = ld_rlx(&a.done[t]);
        const int32_t fs = ld_rlx(&a.final_step[sv]);
        const int32_t fin = fs > 0 ? fs : a.target[sv];
        const int32_t ce = a.check_every[sv];
        const int32_t xu = s_m.phys[u & 7];
        int32_t c0 = 1, c1 = 0;
        uint8_t cross = 0;
        for (int32_t q = a.dep_ptr[t]; q < a.dep_ptr[t + 1]; ++q) {
            const int32_t v = a.dep_idx[q];
            const int32_t dv = ld_rlx(&a.done[v]);
            c0 += dv >= d;
            c1 += dv >= d + 1;
            cross |= s_m.phys[a.tile_pos[v] & 7] != xu;
        }
        const int32_t need = a.dep_ptr[t + 1] - a.dep_ptr[t] + 1;
        const bool gated = ce > 0 && d > 0 && d % ce == 0;
        const bool ready = d < fin && (gated ? ld_rlx(&a.gate[sv]) >= d : c0 == need);
        a.pend[2 * t + (d & 1)] = gated || ready ? 0 : c0;
        a.pend[2 * t + ((d + 1) & 1)] = ce > 0 && (d + 1) % ce == 0 ? 0 : c1;
        a.xpub[u] = cross | (ready ? 2 : 0);
        if (cursor && ready) a.ready[u] = 1;
    }
    if (w == 0 && threadIdx.x == 0) qc[kQcLive] = (uint32_t)a.nlive;
    const bool check = (a.hints & kHintCheck) != 0;
    if (cursor && check && w == 0 && threadIdx.x < 8 && s_m.n[threadIdx.x] > 0)
        qc[kQcHead + threadIdx.x] =
            (uint32_t)(sm64(a.seed ^ 0x637572736F72ull, threadIdx.x) % (uint64_t)s_m.n[threadIdx.x]);
    if (!grid_barrier(a.bar, a.err, a.wait_ticks)) return;
    // part 2: queue the ready tiles
    for (int64_t i = gtid; i < a.ntiles && !cursor; i += stride) {
        const int32_t u = (int32_t)i;
        if (a.tile_list[u] < 0 || !(a.xpub[u] & 2)) continue;
        const int xu = s_m.phys[u & 7];
        ring_push(a, a.qslots + s_m.off[xu], (uint32_t)s_m.cap[xu], &qc[kQcTail + xu], u, quit);
    }

    const bool haspub = use_publisher(__hip_atomic_load(&qc[kQcWgs + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                      (uint32_t)s_m.n[x]);
    const uint32_t cap = (uint32_t)s_m.cap[x];
    if (haspub && s_role) {
        // publisher of XCD x: batches of listed cross tiles, one L2
        // write-back each, then their counts; ends with the launch
        if (threadIdx.x >= 64) return;
        const int lane = threadIdx.x;
        unsigned long long* pl = a.pslots + s_m.off[x];
        uint32_t h = 0;
        for (;;) {
            if (quit()) return;
            uint32_t e = __hip_atomic_load(&qc[kQcPTail + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e == h) {
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            if (e - h > 64u) e = h + 64u;
            int32_t u = -1;
            if ((uint32_t)lane < e - h) u = (int32_t)ring_take(a, pl, cap, h + (uint32_t)lane, quit);
            if (__ballot(u < 0 && (uint32_t)lane < e - h) != 0ull) return;   // launch ending, or timed out
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (u >= 0) {
                const int32_t t = a.tile_list[u];
                const int32_t ns = ld_rlx(&a.done[t]);
                const int32_t cnt = a.dep_ptr[t + 1] - a.dep_ptr[t] + 1;
                for (int32_t i = 0; i < cnt; ++i) serve_count(a, s_m, t, ns, i, cursor);
            }
            h = e;
        }
    }
    unsigned long long* q = a.qslots + s_m.off[x];
    uint32_t ntask = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int32_t u = -1, stop = 0;
            if (check) pert_delay(a, 0x636C61696Dull, ((uint64_t)w << 32) + ntask++);
            if (quit() || __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                stop = 1;
            } else if (cursor) {
                u = (int32_t)cursor_claim(a, s_m, x, quit);
                if (u < 0) stop = 1;
                else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            } else {
                const uint32_t t = __hip_atomic_fetch_add(&qc[kQcHead + x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                u = (int32_t)ring_take(a, q, cap, t, quit);
                if (u < 0) stop = 1;
                else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_u = u;
            s_stop = stop;
        }
        __syncthreads();
        if (s_stop) break;
        const int32_t u = __builtin_amdgcn_readfirstlane(s_u);
        const int32_t t = a.tile_list[u];
        const int32_t sv = a.tile_solve[t];
        const int32_t step = __builtin_amdgcn_readfirstlane(ld_rlx(&a.done[t]));
        if (check && threadIdx.x < 64) check_window(a, t, step);
        const double r = sweep(t, step);
        const int32_t ns = step + 1;
        const bool dec = serve_decision(a, sv, ns);
        // decision steps record the solve's residual (every tile of the
        // solve waits there, so one slot per solve suffices)
        if (dec) wg_residual<double, NT>(r, &a.res[sv], red);
        wg_stores_done();
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const bool cross = (a.xpub[u] & 1) != 0;
            const bool listed = cross && haspub && !dec;
            int32_t decided = 0;   // lane 0: 1 = the solve goes on (queue all its tiles)
            if (check && lane == 0) pert_delay(a, 0x7075626C697368ull, ((uint64_t)t << 20) + (uint64_t)step);
            if (lane == 0) {
                // the step counter advances by exactly one (a tile claimed
                // twice, or run twice, would show here)
                const int32_t was = __hip_atomic_exchange(&a.done[t], ns, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (was != step) __hip_atomic_fetch_or(a.err, kErrSchedule, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // a decision lets tiles of any XCD go on: publish first
                if (cross && !listed) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __builtin_amdgcn_s_waitcnt(0);
                if (listed) ring_push(a, a.pslots + s_m.off[x], cap, &qc[kQcPTail + x], u, quit);
                if (dec) {
                    int32_t* cnt = &a.solve_count[sv];
                    const int32_t prev = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (prev == a.solve_ntiles[sv] - 1) {
                        // last tile of the solve to finish decision step ns
                        __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const unsigned long long rb =
                            __hip_atomic_exchange(&a.res[sv], 0ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                        const double rv = __longlong_as_double((long long)rb);
                        const int32_t ce = a.check_every[sv];
                        const bool fin = ns >= a.target[sv] || (ce > 0 && ns % ce == 0 && rv < a.tol[sv]);
                        if (fin) {
                            __hip_atomic_store(&a.final_step[sv], ns, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                            __threadfence_system();
                            if (a.host_res) a.host_res[sv] = rb;
                            if (a.host_done) a.host_done[sv] = ns;
                            __threadfence_system();
                            __hip_atomic_fetch_sub(&qc[kQcLive], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        } else {
                            __hip_atomic_store(&a.gate[sv], ns, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                            decided = 1;
                        }
                    }
                }
            }
            if (__shfl(decided, 0, 64)) {
                // the solve goes on: every tile of it has finished step ns
                const int32_t b0 = a.solve_base[sv], nt = a.solve_ntiles[sv];
                for (int32_t i = lane; i < nt; i += 64) serve_ready(a, s_m, b0 + i, cursor, quit);
            } else if (!dec && !listed) {
                const int32_t cnt = a.dep_ptr[t + 1] - a.dep_ptr[t] + 1;
                for (int32_t i = lane; i < cnt; i += 64) serve_count(a, s_m, t, ns, i, cursor);
            }
        }
        __syncthreads();
    }
}

// Minimum waves per SIMD the scheduler kernels are compiled for (0 = the
// compiler's choice).  The plain-grid kernel asks for 6: the compiler then
// fits 80 VGPRs with a few spills instead of taking 93-97 (5 or 4 waves),
// and the extra wave per SIMD measured 2 % faster (512^3 fp64 ODF 4096,
// 277 -> 283 GLUP/s; measured again with the current scheduler: 270 at 5
// waves, 290 at 6).  The serving kernel asks for 5: on its own it took 116 VGPRs and
// 4 waves; at 5 (96 VGPRs, no scratch) a saturated stream of 64 mixed
// requests ran 228.6 -> 236 GLUP/s (p50 4.28 -> 4.15 s at 1000 requests/s).
#ifndef OD_SCHED_WAVES
#define OD_SCHED_WAVES 5
#endif
#ifndef OD_MSG_WAVES
#define OD_MSG_WAVES 6
#endif
#if OD_SCHED_WAVES > 0
#define OD_SCHED_OCC __attribute__((amdgpu_waves_per_eu(OD_SCHED_WAVES, 8)))
#else
#define OD_SCHED_OCC
#endif
#if OD_MSG_WAVES > 0
#define OD_MSG_OCC __attribute__((amdgpu_waves_per_eu(OD_MSG_WAVES, 8)))
#else
#define OD_MSG_OCC
#endif

template <typename T, int TX, int TY>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY) OD_MSG_OCC k_msgdriven(MsgArgs a) {
    using S = SW<T, TX, TY>;
    __shared__ T lds[S::LDS];
    __shared__ double red[S::NT / 64];
    T* arena = reinterpret_cast<T*>(a.arena);
    auto sweep = [&](int32_t gid, int32_t step) -> double {
        const TileDev& t = a.tiles[gid];
        const int reps = 1 + imb_extra(a.imb, a.imb_base + step, t.blk);
        T r = 0;
        for (int rep = 0; rep < reps; ++rep) r = sweep_tile<T, TX, TY>(arena, a.blocks, t, step & 1, lds, a.hints);
        return (double)r;
    };
    queue_loop<S::NT>(a, sweep, red);
}

// Message-driven tasks of two steps (grids at one resolution): the same
// scheduler, each task one two-step pass of its tile (with IMB, scheduler
// step k covers steps imb_base + 2k and imb_base + 2k + 1 of the
// imbalance draw, as in k_persistent2).
// A scheduler step is a pass (the field's parity flips once per step), and
// the dependency lists reach every tile within two cells (face slabs two
// deep and the edge lines), so a tile still runs step k once everything it
// reads has finished step k - 1 and nothing that reads it still needs k - 1.
// Compiled for fewer waves than the one-step kernel: at 6 waves per SIMD
// the scheduler's state and the two-step sweep spilled 124 bytes per lane
// (512^3 fp64 ODF 4096, tile (32,16,32): 430 us per iteration); fp64 at 5
// waves (40 bytes) took 289, at 4 (no spill) 309; fp32 at 4 waves 175
// against 238 at 5 and 248 at 6.
template <typename T>
struct Msg2Waves {
    static constexpr int value = sizeof(T) == 8 ? 5 : 4;
};

template <typename T, int TX, int TY, bool IMB>
__global__ void __launch_bounds__((TX / V16<T>::N) * TY) __attribute__((amdgpu_waves_per_eu(Msg2Waves<T>::value, 8)))
k_msgdriven2(MsgArgs a) {
    using S = SW2<T, TX, TY>;
    __shared__ __align__(16) T lds[S::LDS];
    __shared__ double red[S::NT / 64];
    T* arena = reinterpret_cast<T*>(a.arena);
    auto sweep = [&](int32_t gid, int32_t step) -> double {
        const TileDev& t = a.tiles[gid];
        if (IMB)
            imb_extra_sweeps<T, TX, TY>(arena, a.blocks, t, step & 1, lds, a.imb, a.imb_base + 2 * (int64_t)step,
                                        a.hints);
        return (double)sweep2_tile<T, TX, TY>(arena, a.blocks, t, a.tiles2[gid], step & 1, lds, a.hints);
    };
    queue_loop<S::NT>(a, sweep, red);
}

// Serving: tiles of independent fp64 and fp32 solves in one launch.  The two
// tile variants have the same thread count; each task runs the variant of
// its solve's dtype on a shared LDS buffer.  Block offsets are in elements
// of the block's own dtype from the (256-byte aligned) arena base.
template <int TX8, int TY8, int TX4, int TY4>
__global__ void __launch_bounds__((TX8 / 2) * TY8) OD_SCHED_OCC k_serve(MsgArgs a) {
    using S8 = SW<double, TX8, TY8>;
    using S4 = SW<float, TX4, TY4>;
    static_assert(S8::NT == S4::NT, "fp64 and fp32 serving tiles need the same thread count");
    constexpr int LDSB = S8::LDS * 8 > S4::LDS * 4 ? S8::LDS * 8 : S4::LDS * 4;
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[LDSB];
    __shared__ double red[S8::NT / 64];
    auto sweep = [&](int32_t gid, int32_t step) -> double {
        const TileDev& t = a.tiles[gid];
        const int32_t sv = a.tile_solve[gid];
        if (a.solve_dtype[sv] == 8)
            return (double)sweep_tile<double, TX8, TY8>(reinterpret_cast<double*>(a.arena), a.blocks, t, step & 1,
                                                        reinterpret_cast<double*>(lds_raw), a.hints);
        return (double)sweep_tile<float, TX4, TY4>(reinterpret_cast<float*>(a.arena), a.blocks, t, step & 1,
                                                   reinterpret_cast<float*>(lds_raw), a.hints);
    };
    serve_loop<S8::NT>(a, sweep, red);
}

// ---------------------------------------------------------------------------
// Two steps per pass of the 2D 5-point stencil (Jacobi2D on the (x, z)
// plane, y extent 1): the same scheme as sweep2_tile on rows instead of
// planes.  The ring around a tile is one cell on each side along x (and
// the rows just below and above it), so four lanes hold the ring: lanes 0
// and 1 the cells one out (x = -1, nx) with their three-row columns, lanes
// 2 and 3 the cells two out (x = -2, nx + 1).
template <typename T, int TX>
struct SW2D {
    static constexpr int VX = V16<T>::N;
    static constexpr int LX = TX / VX;
    static constexpr int NT = LX;
    static constexpr int LP = TX + 2 * VX;   // column VX + x holds x in [-2, TX + 1]
    static constexpr int LDS = 4 * LP;       // time-t rows and first-step rows, double buffered
    static_assert(TX % VX == 0 && VX >= 2 && LX >= 4, "four ring lanes");
    static_assert(NT % 64 == 0 && NT <= 1024, "threads must be whole waves");
};

template <typename T, int TX>
__device__ __forceinline__ T sweep2d_tile(T* __restrict__ arena, const BlockDev* __restrict__ blocks,
                                          const TileDev& t, const Tile2Dev& t2, const int parity,
                                          T* __restrict__ lds, const int hints) {
    using S = SW2D<T, TX>;
    using VT = typename V16<T>::t;
    constexpr int VX = S::VX, LP = S::LP;
    constexpr int64_t ES = (int64_t)sizeof(T);
    const int lx = threadIdx.x, x = lx * VX;
    const int nx = t.nx, nz = t.nz;
    int nv = nx - x;
    nv = nv < 0 ? 0 : (nv > VX ? VX : nv);
    const bool act = nv > 0;
    const int xc = x < nx ? x : ((nx - 1) / VX) * VX;
    const int dir = t2.dir;
    const char* __restrict__ ab = reinterpret_cast<const char*>(arena);

    const BlockDev* __restrict__ B = blocks + t.blk;
    const int64_t own_pz = B->pz;
    const int64_t tile_el = t.x0 + (int64_t)t.y0 * B->py + (int64_t)t.z0 * own_pz;
    const char* own_b = ab + ((parity ? B->off[1] : B->off[0]) + tile_el) * ES;
    char* dst_b = reinterpret_cast<char*>(arena) + ((parity ? B->off[0] : B->off[1]) + tile_el) * ES;
    const uint32_t o_own = (uint32_t)(xc * ES);
    auto at = [&](const FaceDev& f, int64_t* pz) -> const char* {
        const BlockDev* __restrict__ F = blocks + f.src;
        *pz = F->pz;
        return ab + ((parity ? F->off[1] : F->off[0]) + f.sx + (int64_t)f.sy * F->py + (int64_t)f.sz * F->pz) * ES;
    };
    int64_t pz;
    const char* zm_b = at(t.f[4], &pz);
    const char* zp_b = at(t.f[5], &pz);
    const char* zm2_b = at(t2.r2[4], &pz);
    const char* zp2_b = at(t2.r2[5], &pz);

    // ring lanes: 0 / 1 the cell one out on the x- / x+ side, 2 / 3 the cell two out
    const int side = lx & 1;
    const bool r1 = lx < 2, r2 = lx >= 2 && lx < 4;
    const int r1c = side ? VX + nx : VX - 1, r2c = side ? VX + nx + 1 : VX - 2;
    int64_t r1_pz = own_pz * ES, r2_pz = own_pz * ES;
    const char* r1_b = own_b;
    const char* r1_lo = own_b;
    const char* r1_hi = own_b;
    const char* r2_b = own_b;
    if (r1) {
        r1_b = at(t.f[side], &pz);
        r1_pz = pz * ES;
        r1_lo = at(t2.e[4 + side], &pz);
        r1_hi = at(t2.e[6 + side], &pz);
    } else if (r2) {
        r2_b = at(t2.r2[side], &pz);
        r2_pz = pz * ES;
    }
    const bool r1dir = r1 && ((dir >> side) & 1);

    auto ldv = [](const char* p) -> VT { return *reinterpret_cast<const VT*>(p); };
    auto lds1 = [](const char* p) -> T { return *reinterpret_cast<const T*>(p); };
    auto tpl = [&](int q) -> VT {   // row q in [-2, nz + 1] (uniform)
        if (q >= 0 && q < nz) return ldv(own_b + q * own_pz * ES + o_own);
        if (q == -1) return ldv(zm_b + o_own);
        if (q == -2) return ldv(zm2_b + o_own);
        if (q == nz) return ldv(zp_b + o_own);
        return ldv(zp2_b + o_own);
    };
    auto rl1 = [&](int q) -> T { return lds1(q < 0 ? r1_lo : (q >= nz ? r1_hi : r1_b + q * r1_pz)); };
    auto lim = [&](int q) { return q < 0 ? 0 : (q > nz - 1 ? nz - 1 : q); };
    auto tl = [&](int b, int c) -> T& { return lds[b * LP + c]; };
    auto ul = [&](int b, int c) -> T& { return lds[(2 + b) * LP + c]; };
    auto vref = [](T& e) -> VT& { return *reinterpret_cast<VT*>(&e); };

    constexpr int PF = OD_PREFETCH;
    VT tz[PF + 3];   // rows j-1 .. j+PF+1 of the lane's cells
#pragma unroll
    for (int k = 0; k < PF + 2; ++k) tz[k] = tpl(-2 + k <= nz + 1 ? -2 + k : nz + 1);
    T rc[4];         // ring cell one out: rows j-1 .. j+2
    rc[0] = rl1(-1);
    rc[1] = rl1(-1);
    rc[2] = rl1(0);
    T c2 = lds1(r2_b);   // ring cell two out, row j
    VT um1, um2;
    T r = 0;

    for (int j = -1; j <= nz; ++j) {
        const int b = j & 1;
        const bool inz = j >= 0 && j < nz;
        tz[PF + 2] = tpl(j + PF + 1 <= nz + 1 ? j + PF + 1 : nz + 1);
        rc[3] = rl1(j + 2 > nz ? nz : j + 2);
        const T c2n = lds1(r2_b + lim(j + 1) * r2_pz);

        // stage time-t row j
        if (nv == VX) {
            vref(tl(b, VX + x)) = tz[1];
        } else if (act) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nv) tl(b, VX + x + i) = tz[1][i];
        }
        if (r1) tl(b, r1c) = rc[1];
        if (r2 && inz) tl(b, r2c) = c2;
        __syncthreads();

        // first step of row j (Dirichlet z row: its value)
        const bool zfix = (j < 0 && (dir & 16)) || (j >= nz && (dir & 32));
        VT u;
#pragma unroll
        for (int i = 0; i < VX; ++i) {
            const T xm = i > 0 ? tz[1][i - 1] : tl(b, VX + x - 1);
            const T xp = (i < VX - 1 && i + 1 < nv) ? tz[1][i + 1] : tl(b, VX + x + i + 1);
            T s = xm;
            s = s + xp;
            s = s + tz[0][i];
            s = s + tz[2][i];
            u[i] = zfix ? tz[1][i] : s / (T)4;
        }
        if (nv == VX) {
            vref(ul(b, VX + x)) = u;
        } else if (act) {
#pragma unroll
            for (int i = 0; i < VX; ++i)
                if (i < nv) ul(b, VX + x + i) = u[i];
        }
        // first step of the ring cell one out (Dirichlet face: its value)
        if (inz && r1) {
            T s = tl(b, r1c - 1);
            s = s + tl(b, r1c + 1);
            s = s + rc[0];
            s = s + rc[2];
            ul(b, r1c) = r1dir ? rc[1] : s / (T)4;
        }

        // second step of row j - 1
        if (j >= 1) {
            const int c = b ^ 1;
            VT out;
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                const T xm = i > 0 ? um1[i - 1] : ul(c, VX + x - 1);
                const T xp = (i < VX - 1 && i + 1 < nv) ? um1[i + 1] : ul(c, VX + x + i + 1);
                T s = xm;
                s = s + xp;
                s = s + um2[i];
                s = s + u[i];
                const T v = s / (T)4;
                out[i] = v;
                if (i < nv) {
                    T d = v - um1[i];
                    if (d < (T)0) d = -d;
                    if (d > r) r = d;
                }
            }
            if (act) {
                VT* o = reinterpret_cast<VT*>(dst_b + (int64_t)(j - 1) * own_pz * ES + o_own);
                if (hints & 1)
                    __builtin_nontemporal_store(out, o);
                else
                    *o = out;
            }
        }
        um2 = um1;
        um1 = u;
#pragma unroll
        for (int k = 0; k < PF + 2; ++k) tz[k] = tz[k + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) rc[k] = rc[k + 1];
        c2 = c2n;
    }
    __syncthreads();   // LDS rows are reused by the next tile
    return r;
}

template <typename T, int TX>
__global__ void __launch_bounds__(TX / V16<T>::N)
k_sweep2d(T* __restrict__ arena, const BlockDev* __restrict__ blocks, const TileDev* __restrict__ tiles,
          const Tile2Dev* __restrict__ tiles2, int parity, unsigned long long* __restrict__ res, int zero_lo,
          int zero_hi, int hints) {
    using S = SW2D<T, TX>;
    __shared__ __align__(16) T lds[S::LDS];
    __shared__ T red[S::NT / 64];
    if (blockIdx.x == 0)
        for (int s = zero_lo + (int)threadIdx.x; s < zero_hi; s += S::NT) res[2 * s + parity] = 0ull;
    const TileDev& t = tiles[blockIdx.x];
    const T r = sweep2d_tile<T, TX>(arena, blocks, t, tiles2[blockIdx.x], parity, lds, hints);
    wg_residual<T, S::NT>(r, &res[2 * t.rslot + (parity ^ 1)], red);
}

// ---------------------------------------------------------------------------
// variant table

#define OD_VARIANTS_F64(X) X(double, 32, 4) X(double, 32, 8) X(double, 32, 16) X(double, 32, 32) \
    X(double, 64, 4) X(double, 64, 8) X(double, 64, 16) X(double, 16, 8) X(double, 16, 16) X(double, 128, 4) \
    X(double, 128, 1) X(double, 256, 1) X(double, 512, 1)
#define OD_VARIANTS_F32(X) X(float, 32, 8) X(float, 32, 16) X(float, 32, 32) X(float, 64, 4) \
    X(float, 64, 8) X(float, 64, 16) X(float, 128, 4) X(float, 128, 8) X(float, 16, 16) X(float, 256, 1) \
    X(float, 512, 1) X(float, 1024, 1)

#define OD_VT_ENTRY(T, TX, TY) {TX, TY, SW<T, TX, TY>::NT},
static const SweepVariant kVariants64[] = {OD_VARIANTS_F64(OD_VT_ENTRY)};
static const SweepVariant kVariants32[] = {OD_VARIANTS_F32(OD_VT_ENTRY)};

const SweepVariant* sweep_variants(int dtype_bytes, int* count) {
    if (dtype_bytes == 8) {
        *count = (int)(sizeof(kVariants64) / sizeof(kVariants64[0]));
        return kVariants64;
    }
    *count = (int)(sizeof(kVariants32) / sizeof(kVariants32[0]));
    return kVariants32;
}

bool sweep_variant_ok(int dtype_bytes, int tx, int ty) { return sweep_threads(dtype_bytes, tx, ty) > 0; }

int sweep_threads(int dtype_bytes, int tx, int ty) {
    int n = 0;
    const SweepVariant* v = sweep_variants(dtype_bytes, &n);
    for (int i = 0; i < n; ++i)
        if (v[i].tx == tx && v[i].ty == ty) return v[i].threads;
    return 0;
}

hipError_t launch_sweep(int dtype_bytes, int tx, int ty, hipStream_t st, void* arena, const BlockDev* blocks,
                        const TileDev* tiles, int32_t ntiles, int parity, unsigned long long* res,
                        int32_t zero_lo, int32_t zero_hi, const ImbDev& imb, int64_t step, int hints,
                        const XExpDev* xexp) {
    if (ntiles <= 0) return hipSuccess;
#define OD_LAUNCH(T, TX, TY)                                                                          \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                      \
        if (xexp)                                                                                     \
            hipLaunchKernelGGL((k_sweep<T, TX, TY, true>), dim3(ntiles), dim3(SW<T, TX, TY>::NT), 0, st, \
                               reinterpret_cast<T*>(arena), blocks, tiles, parity, res, zero_lo, zero_hi, \
                               imb, step, hints, xexp);                                               \
        else                                                                                          \
            hipLaunchKernelGGL((k_sweep<T, TX, TY, false>), dim3(ntiles), dim3(SW<T, TX, TY>::NT), 0, st, \
                               reinterpret_cast<T*>(arena), blocks, tiles, parity, res, zero_lo, zero_hi, \
                               imb, step, hints, xexp);                                               \
        return hipGetLastError();                                                                     \
    }
    OD_VARIANTS_F64(OD_LAUNCH)
    OD_VARIANTS_F32(OD_LAUNCH)
#undef OD_LAUNCH
    return hipErrorInvalidValue;
}

#define OD_VARIANTS2_F64(X) X(double, 32, 32) X(double, 32, 16) X(double, 32, 8) X(double, 64, 8) \
    X(double, 64, 16) X(double, 16, 16)
#define OD_VARIANTS2_F32(X) X(float, 32, 32) X(float, 32, 16) X(float, 64, 16)

#define OD_VARIANTS2D(X) X(double, 128) X(double, 256) X(double, 512) X(float, 256) X(float, 512) X(float, 1024)

bool sweep2_variant_ok(int dtype_bytes, int tx, int ty, bool flat) {
    if (flat) {
#define OD_OK2D(T, TX) \
        if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == 1) return true;
        OD_VARIANTS2D(OD_OK2D)
#undef OD_OK2D
        return false;
    }
#define OD_OK2(T, TX, TY) \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) return true;
    OD_VARIANTS2_F64(OD_OK2)
    OD_VARIANTS2_F32(OD_OK2)
#undef OD_OK2
    return false;
}

hipError_t launch_sweep2(int dtype_bytes, int tx, int ty, hipStream_t st, void* arena, const BlockDev* blocks,
                         const TileDev* tiles, const Tile2Dev* tiles2, int32_t ntiles, int parity,
                         unsigned long long* res, int32_t zero_lo, int32_t zero_hi, int hints, const ImbDev& imb,
                         int64_t step) {
    if (ntiles <= 0) return hipSuccess;
    if (hints & 0x100) {   // the 2D 5-point stencil
        if (imb.heavy > 0) return hipErrorInvalidValue;
#define OD_LAUNCH2D(T, TX)                                                                               \
        if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == 1) {                                      \
            hipLaunchKernelGGL((k_sweep2d<T, TX>), dim3(ntiles), dim3(SW2D<T, TX>::NT), 0, st,           \
                               reinterpret_cast<T*>(arena), blocks, tiles, tiles2, parity, res, zero_lo,  \
                               zero_hi, hints);                                                          \
            return hipGetLastError();                                                                    \
        }
        OD_VARIANTS2D(OD_LAUNCH2D)
#undef OD_LAUNCH2D
        return hipErrorInvalidValue;
    }
#define OD_LAUNCH2(T, TX, TY)                                                                            \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                         \
        if (imb.heavy > 0)                                                                               \
            hipLaunchKernelGGL((k_sweep2_imb<T, TX, TY>), dim3(ntiles), dim3(SW2<T, TX, TY>::NT), 0, st, \
                               reinterpret_cast<T*>(arena), blocks, tiles, tiles2, parity, res, zero_lo,  \
                               zero_hi, hints, imb, step);                                               \
        else                                                                                             \
            hipLaunchKernelGGL((k_sweep2<T, TX, TY>), dim3(ntiles), dim3(SW2<T, TX, TY>::NT), 0, st,    \
                               reinterpret_cast<T*>(arena), blocks, tiles, tiles2, parity, res, zero_lo,  \
                               zero_hi, hints);                                                          \
        return hipGetLastError();                                                                        \
    }
    OD_VARIANTS2_F64(OD_LAUNCH2)
    OD_VARIANTS2_F32(OD_LAUNCH2)
#undef OD_LAUNCH2
    return hipErrorInvalidValue;
}

int64_t device_wait_ticks(double seconds) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;   // 100 MHz, the usual constant-rate counter
    return (int64_t)(seconds * 1e3 * (double)khz);
}

// LDS per CU and the granule a workgroup's LDS is allocated in on gfx950.
// A residency probe (plain launches of 128-thread workgroups that hold their
// CU for 2 ms; two rounds take twice as long) fit 12 per CU at 12 800 bytes
// each and not at 12 801, while the occupancy query still allowed 12 up to
// 13 653 bytes (and 13 at 12 288): it rounds to a finer granule.
constexpr int kLdsPerCu = 160 * 1024, kLdsGranule = 1280;

// Co-resident workgroups per CU of a cooperative kernel: the occupancy
// query `per` (exact for VGPRs), limited by the kernel's LDS in whole
// granules and by what its scalar registers allow (both from what the
// compiler recorded when the library was compiled; a kernel missing from the record is
// taken as 5 waves per SIMD), and by `max_waves` waves per SIMD (a
// scheduling choice).  A cooperative grid larger than what is resident
// would never complete its first device-wide barrier.
static int coop_per_cu(int per, int threads, const char* name, int max_waves) {
    int sg = 0, lds = 0;
    const bool rec = kernel_resources(name, &sg, nullptr, &lds);
    const int w_sgpr = rec ? waves_by_sgprs(sg) : 5;
    const int w = max_waves > 0 && max_waves < w_sgpr ? max_waves : w_sgpr;
    const int wpw = (threads + 63) / 64;
    int cap = (4 * w) / wpw;   // 4 SIMDs per CU
    if (rec && lds > 0) {
        const int by_lds = kLdsPerCu / ((lds + kLdsGranule - 1) / kLdsGranule * kLdsGranule);
        cap = by_lds < cap ? by_lds : cap;
    }
    return per < cap ? per : cap;
}

static std::string kernel_name(const char* base, int dtype_bytes, int tx, int ty, const char* extra) {
    return std::string("od::") + base + "<" + (dtype_bytes == 8 ? "double" : "float") + ", " + std::to_string(tx) +
           ", " + std::to_string(ty) + (extra ? extra : "") + ">";
}

// imb: the load-imbalance variant of a two-step kernel (kinds 3 - 5)
static std::string coop_name(int dtype_bytes, int tx, int ty, int kind, bool imb = false) {
    const char* i2 = imb ? ", true" : ", false";
    return kind == 1   ? kernel_name("k_msgdriven", dtype_bytes, tx, ty, nullptr)
           : kind == 5 ? kernel_name("k_msgdriven2", dtype_bytes, tx, ty, i2)
           : kind == 6 ? kernel_name("k_persistent_mr", dtype_bytes, tx, ty, nullptr)
           : kind >= 3 ? kernel_name("k_persistent2", dtype_bytes, tx, ty,
                                     (std::string(kind == 4 ? ", true" : ", false") + i2).c_str())
                       : kernel_name("k_persistent", dtype_bytes, tx, ty, kind == 2 ? ", true" : ", false");
}

static int sgpr_waves(const std::string& name) {
    int sg = 0;
    return kernel_resources(name.c_str(), &sg, nullptr, nullptr) ? waves_by_sgprs(sg) : 5;
}

// two-step kinds: the smaller of the uniform and imbalance variants, so a
// grid sized for the kind fits either
int coop_waves_limit(int dtype_bytes, int tx, int ty, int kind) {
    const int w = sgpr_waves(coop_name(dtype_bytes, tx, ty, kind));
    if (kind < 3 || kind > 5) return w;
    const int wi = sgpr_waves(coop_name(dtype_bytes, tx, ty, kind, true));
    return wi < w ? wi : w;
}

template <typename K>
static int coop_cap(K kernel, int threads, const std::string& name, int max_waves) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) return 0;
    return coop_per_cu(per, threads, name.c_str(), max_waves);
}

int persistent_max_grid(int dtype_bytes, int tx, int ty, int kind, int max_waves) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    // default choice: the counter form (imbalance, uneven blocks) measured
    // faster at 5 waves per SIMD than at 6
    if (max_waves <= 0) max_waves = kind == 2 ? 5 : 8;
    const std::string name = coop_name(dtype_bytes, tx, ty, kind);
    if (kind >= 3 && kind <= 5) {
        // the uniform and the load-imbalance variant: the smaller residency
        const std::string name_i = coop_name(dtype_bytes, tx, ty, kind, true);
#define OD_OCC2(T, TX, TY)                                                                            \
        if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                  \
            constexpr int NT = SW2<T, TX, TY>::NT;                                                    \
            const int c0 = kind == 5 ? coop_cap(k_msgdriven2<T, TX, TY, false>, NT, name, max_waves)  \
                           : kind == 4 ? coop_cap(k_persistent2<T, TX, TY, true, false>, NT, name, max_waves) \
                           : coop_cap(k_persistent2<T, TX, TY, false, false>, NT, name, max_waves);   \
            const int c1 = kind == 5 ? coop_cap(k_msgdriven2<T, TX, TY, true>, NT, name_i, max_waves) \
                           : kind == 4 ? coop_cap(k_persistent2<T, TX, TY, true, true>, NT, name_i, max_waves) \
                           : coop_cap(k_persistent2<T, TX, TY, false, true>, NT, name_i, max_waves);  \
            return (c1 < c0 ? c1 : c0) * ncu;                                                         \
        }
        OD_VARIANTS2_F64(OD_OCC2)
        OD_VARIANTS2_F32(OD_OCC2)
#undef OD_OCC2
        return 0;
    }
#define OD_OCC(T, TX, TY)                                                                             \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                      \
        hipError_t e = kind == 0                                                                      \
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<T, TX, TY, false>,      \
                                                           SW<T, TX, TY>::NT, 0)                      \
            : kind == 2                                                                               \
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<T, TX, TY, true>,       \
                                                           SW<T, TX, TY>::NT, 0)                      \
            : kind == 6                                                                               \
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent_mr<T, TX, TY>,          \
                                                           SW<T, TX, TY>::NT, 0)                      \
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_msgdriven<T, TX, TY>,              \
                                                           SW<T, TX, TY>::NT, 0);                     \
        if (e != hipSuccess) return 0;                                                                \
        return coop_per_cu(per, SW<T, TX, TY>::NT, name.c_str(), max_waves) * ncu;                   \
    }
    OD_VARIANTS_F64(OD_OCC)
    OD_VARIANTS_F32(OD_OCC)
#undef OD_OCC
    return 0;
}

hipError_t launch_persistent(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, void* arena,
                             const BlockDev* blocks, const TileDev* tiles, int32_t ntiles, int parity,
                             int64_t iters, unsigned long long* res, int32_t nres, unsigned int* bar,
                             unsigned int* err, const ImbDev& imb, int64_t iter_base, int hints, int dyn,
                             int64_t wait_ticks, unsigned long long* stamps, int chunked) {
    if (iters <= 0) return hipSuccess;
#define OD_LAUNCH(T, TX, TY)                                                                          \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                      \
        T* ar = reinterpret_cast<T*>(arena);                                                          \
        ImbDev im = imb;                                                                              \
        void* args[] = {&ar, &blocks, &tiles, &ntiles, &parity, &iters, &res, &nres, &bar, &err,      \
                        &im, &iter_base, &wait_ticks, &hints, &stamps, &chunked};                     \
        const void* fn = dyn ? reinterpret_cast<const void*>(k_persistent<T, TX, TY, true>)           \
                             : reinterpret_cast<const void*>(k_persistent<T, TX, TY, false>);         \
        return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(SW<T, TX, TY>::NT), args, 0, st);      \
    }
    OD_VARIANTS_F64(OD_LAUNCH)
    OD_VARIANTS_F32(OD_LAUNCH)
#undef OD_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_persistent_mr(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, void* arena,
                                const BlockDev* blocks, const TileDev* tiles, int32_t ntiles, int parity,
                                int64_t iters, unsigned long long* res, int32_t nres, unsigned int* bar,
                                unsigned int* err, int64_t wait_ticks, int hints, const FillSeg* segs, int32_t nseg,
                                const XExpDev* xexp) {
    if (iters <= 0) return hipSuccess;
#define OD_LAUNCH(T, TX, TY)                                                                          \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                      \
        T* ar = reinterpret_cast<T*>(arena);                                                          \
        void* args[] = {&ar, &blocks, &tiles, &ntiles, &parity, &iters, &res, &nres, &bar, &err,      \
                        &wait_ticks, &hints, &segs, &nseg, &xexp};                                    \
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_persistent_mr<T, TX, TY>), \
                                          dim3(grid), dim3(SW<T, TX, TY>::NT), args, 0, st);          \
    }
    OD_VARIANTS_F64(OD_LAUNCH)
    OD_VARIANTS_F32(OD_LAUNCH)
#undef OD_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_persistent2(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, void* arena,
                              const BlockDev* blocks, const TileDev* tiles, const Tile2Dev* tiles2, int32_t ntiles,
                              int parity, int64_t passes, unsigned long long* res, int32_t nres, unsigned int* bar,
                              unsigned int* err, int hints, int64_t wait_ticks, int dyn, const ImbDev& imb,
                              int64_t iter_base) {
    if (passes <= 0) return hipSuccess;
    ImbDev im = imb;
#define OD_LAUNCH2(T, TX, TY)                                                                         \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                      \
        T* ar = reinterpret_cast<T*>(arena);                                                          \
        void* args[] = {&ar, &blocks, &tiles, &tiles2, &ntiles, &parity, &passes, &res, &nres, &bar,  \
                        &err, &wait_ticks, &hints, &im, &iter_base};                                  \
        const void* fn = imb.heavy > 0                                                                \
            ? (dyn ? reinterpret_cast<const void*>(k_persistent2<T, TX, TY, true, true>)              \
                   : reinterpret_cast<const void*>(k_persistent2<T, TX, TY, false, true>))            \
            : (dyn ? reinterpret_cast<const void*>(k_persistent2<T, TX, TY, true, false>)             \
                   : reinterpret_cast<const void*>(k_persistent2<T, TX, TY, false, false>));          \
        return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(SW2<T, TX, TY>::NT), args, 0, st);     \
    }
    OD_VARIANTS2_F64(OD_LAUNCH2)
    OD_VARIANTS2_F32(OD_LAUNCH2)
#undef OD_LAUNCH2
    return hipErrorInvalidValue;
}

int serve_max_grid() {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_serve<kServeTx8, kServeTy8, kServeTx4, kServeTy4>,
                                                     SW<double, kServeTx8, kServeTy8>::NT, 0) != hipSuccess)
        return 0;
    const std::string name = "od::k_serve<" + std::to_string(kServeTx8) + ", " + std::to_string(kServeTy8) + ", " +
                             std::to_string(kServeTx4) + ", " + std::to_string(kServeTy4) + ">";
    return coop_per_cu(per, SW<double, kServeTx8, kServeTy8>::NT, name.c_str(), 8) * ncu;
}

hipError_t launch_serve(hipStream_t st, int grid, const MsgArgs& a) {
    MsgArgs ac = a;
    void* args[] = {&ac};
    return hipLaunchCooperativeKernel(
        reinterpret_cast<const void*>(k_serve<kServeTx8, kServeTy8, kServeTx4, kServeTy4>), dim3(grid),
        dim3(SW<double, kServeTx8, kServeTy8>::NT), args, 0, st);
}

hipError_t launch_msgdriven(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, const MsgArgs& a) {
    MsgArgs ac = a;
#define OD_LAUNCH(T, TX, TY)                                                                          \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                      \
        void* args[] = {&ac};                                                                         \
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_msgdriven<T, TX, TY>),     \
                                          dim3(grid), dim3(SW<T, TX, TY>::NT), args, 0, st);          \
    }
    OD_VARIANTS_F64(OD_LAUNCH)
    OD_VARIANTS_F32(OD_LAUNCH)
#undef OD_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_msgdriven2(int dtype_bytes, int tx, int ty, hipStream_t st, int grid, const MsgArgs& a) {
    if (a.tiles2 == nullptr) return hipErrorInvalidValue;
    MsgArgs ac = a;
#define OD_LAUNCH2(T, TX, TY)                                                                         \
    if (dtype_bytes == (int)sizeof(T) && tx == TX && ty == TY) {                                      \
        void* args[] = {&ac};                                                                         \
        const void* fn = a.imb.heavy > 0 ? reinterpret_cast<const void*>(k_msgdriven2<T, TX, TY, true>) \
                                         : reinterpret_cast<const void*>(k_msgdriven2<T, TX, TY, false>); \
        return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(SW2<T, TX, TY>::NT), args, 0, st);     \
    }
    OD_VARIANTS2_F64(OD_LAUNCH2)
    OD_VARIANTS2_F32(OD_LAUNCH2)
#undef OD_LAUNCH2
    return hipErrorInvalidValue;
}

__global__ void k_stamp_init(unsigned long long* stamps, int32_t n) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < 4 * n) stamps[i] = (i & 1) ? 0ull : ~0ull;   // minima start high, maxima low
}

hipError_t launch_stamp_init(hipStream_t st, unsigned long long* stamps, int32_t n) {
    hipLaunchKernelGGL(k_stamp_init, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, st, stamps, n);
    return hipGetLastError();
}

__global__ void k_queue_init(MsgArgs a, int32_t target, int32_t* target_word, unsigned long long* res_clear) {
    // heads, tails, present-XCD mask, workgroups per XCD, list tails and
    // cross-tile counts start at zero; the launch fills in the rest
    a.qhead[threadIdx.x] = 0u;
    if (target_word && threadIdx.x == 0) *target_word = target;
    if (res_clear && threadIdx.x < 2) res_clear[threadIdx.x] = 0ull;
}

hipError_t launch_queue_init(hipStream_t st, const MsgArgs& a, int32_t target, int32_t* target_word,
                             unsigned long long* res_clear) {
    hipLaunchKernelGGL(k_queue_init, dim3(1), dim3(64), 0, st, a, target, target_word, res_clear);
    return hipGetLastError();
}

__global__ void k_serve_positions(const int32_t* __restrict__ list, int32_t n, int32_t stride,
                                  int32_t* __restrict__ tpos, int32_t* __restrict__ sbase) {
    const int32_t q = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= n) return;
    const int32_t v = list[q];
    if (v < 0) return;
    tpos[v] = q;
    if (v % stride == 0) sbase[v / stride] = q;
}

hipError_t launch_serve_positions(hipStream_t st, const int32_t* list, int32_t n, int32_t stride, int32_t* tpos,
                                  int32_t* sbase) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_serve_positions, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, list, n, stride,
                       tpos, sbase);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initialisation and global-layout I/O

template <typename T>
__global__ void k_init(GridDev g, uint64_t seed) {
    T* arena = reinterpret_cast<T*>(g.arena);
    const int64_t nx = g.n[0], ny = g.n[1], total = g.n[0] * g.n[1] * g.n[2];
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < total;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = gi % nx, j = (gi / nx) % ny, k = gi / (nx * ny);
        const int32_t c = owner_of(g.lk, i, j, k);
        const BlockDev B = g.blocks[c];
        const int64_t lx = i - g.lk.corigin[3 * c], ly = j - g.lk.corigin[3 * c + 1], lz = k - g.lk.corigin[3 * c + 2];
        arena[B.off[0] + lx + ly * B.py + lz * B.pz] = unit_from_bits<T>(sm64(seed, (uint64_t)gi));
    }
}

// Multi-resolution initialisation: one chare per blockIdx.y step, its cells
// grid-strided over blockIdx.x.
template <typename T>
__global__ void k_init_cells(GridDev g, const int32_t* __restrict__ ccell, int32_t nchares, uint64_t seed) {
    T* arena = reinterpret_cast<T*>(g.arena);
    const int64_t nx = g.n[0], ny = g.n[1];
    for (int32_t c = blockIdx.y; c < nchares; c += gridDim.y) {
        const BlockDev B = g.blocks[c];
        const int64_t h = ccell[c];
        const int64_t ux = g.lk.corigin[3 * c], uy = g.lk.corigin[3 * c + 1], uz = g.lk.corigin[3 * c + 2];
        const int64_t cnt = (int64_t)B.ex * B.ey * B.ez;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x) {
            const int64_t x = e % B.ex, y = (e / B.ex) % B.ey, z = e / ((int64_t)B.ex * B.ey);
            const int64_t gi = ((uz + z * h) * ny + (uy + y * h)) * nx + (ux + x * h);
            arena[B.off[0] + x + y * B.py + z * B.pz] = unit_from_bits<T>(sm64(seed, (uint64_t)gi));
        }
    }
}


template <typename T>
__global__ void k_fill_pb(GridDev g, int32_t npb, const int32_t* pb_face, const int32_t* pb_block,
                          const double* bc) {
    T* arena = reinterpret_cast<T*>(g.arena);
    for (int32_t q = blockIdx.y; q < npb; q += gridDim.y) {
        const BlockDev B = g.blocks[pb_block[q]];
        const T v = (T)bc[pb_face[q]];
        const int64_t cnt = (int64_t)B.ex * B.ey * B.ez;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x) {
            const int64_t x = e % B.ex, y = (e / B.ex) % B.ey, z = e / ((int64_t)B.ex * B.ey);
            arena[B.off[0] + x + y * B.py + z * B.pz] = v;
        }
    }
}

// Address of padded global cell (I, J, K) (0..n+1) or -1 for shell edges.
__device__ __forceinline__ int64_t global_addr(const GridDev& g, int parity, int64_t I, int64_t J, int64_t K) {
    int64_t c3[3] = {I - 1, J - 1, K - 1};
    int outs = 0, f = -1;
    for (int d = 0; d < 3; ++d) {
        if (c3[d] < 0) {
            ++outs;
            f = 2 * d;
            c3[d] = 0;
        } else if (c3[d] >= g.n[d]) {
            ++outs;
            f = 2 * d + 1;
            c3[d] = g.n[d] - 1;
        }
    }
    if (outs >= 2) return -1;
    const int32_t c = owner_of(g.lk, c3[0], c3[1], c3[2]);
    int64_t l[3];
    for (int d = 0; d < 3; ++d) l[d] = c3[d] - g.lk.corigin[3 * c + d];
    int32_t b = c;
    if (outs == 1) {
        b = g.lk.dir_pb[6 * c + f];
        l[f / 2] = 0;
        if (b < 0) return -1;
    }
    const BlockDev B = g.blocks[b];
    return B.off[parity] + l[0] + l[1] * B.py + l[2] * B.pz;
}

template <typename T>
__global__ void k_gather(GridDev g, int parity, int64_t kz_lo, int64_t kz_hi, T* dst) {
    const T* arena = reinterpret_cast<const T*>(g.arena);
    const int64_t PX = g.n[0] + 2, PY = g.n[1] + 2;
    const int64_t total = (kz_hi - kz_lo) * PX * PY;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t I = e % PX, J = (e / PX) % PY, K = kz_lo + e / (PX * PY);
        const int64_t a = global_addr(g, parity, I, J, K);
        dst[e] = a < 0 ? (T)0 : arena[a];
    }
}

template <typename T>
__global__ void k_scatter(GridDev g, int parity, int64_t kz_lo, int64_t kz_hi, const T* src) {
    T* arena = reinterpret_cast<T*>(g.arena);
    const int64_t PX = g.n[0] + 2, PY = g.n[1] + 2;
    const int64_t total = (kz_hi - kz_lo) * PX * PY;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t I = e % PX, J = (e / PX) % PY, K = kz_lo + e / (PX * PY);
        const int64_t a = global_addr(g, parity, I, J, K);
        if (a >= 0) arena[a] = src[e];
    }
}

template <typename T>
__global__ void k_points(GridDev g, int parity, const int64_t* idx, int64_t count, T* dst) {
    const T* arena = reinterpret_cast<const T*>(g.arena);
    const int64_t nx = g.n[0], ny = g.n[1];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t gi = idx[e];
        const int64_t i = gi % nx, j = (gi / nx) % ny, k = gi / (nx * ny);
        dst[e] = arena[global_addr(g, parity, i + 1, j + 1, k + 1)];
    }
}

static int io_grid(int64_t total) {
    int64_t b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    return (int)(b < 1 ? 1 : b);
}

hipError_t launch_init(int dtype_bytes, hipStream_t st, const GridDev& g, int32_t nchares, uint64_t seed,
                       int32_t npb, const int32_t* pb_face, const int32_t* pb_block, const double* bc_dev,
                       bool interior) {
    (void)nchares;
    const int64_t total = g.n[0] * g.n[1] * g.n[2];
    if (interior) {
        if (dtype_bytes == 8)
            hipLaunchKernelGGL(k_init<double>, dim3(io_grid(total)), dim3(256), 0, st, g, seed);
        else
            hipLaunchKernelGGL(k_init<float>, dim3(io_grid(total)), dim3(256), 0, st, g, seed);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || npb <= 0) return e;
    dim3 grid(16, (unsigned)(npb < 65535 ? npb : 65535));
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_fill_pb<double>, grid, dim3(256), 0, st, g, npb, pb_face, pb_block, bc_dev);
    else
        hipLaunchKernelGGL(k_fill_pb<float>, grid, dim3(256), 0, st, g, npb, pb_face, pb_block, bc_dev);
    return hipGetLastError();
}

hipError_t launch_init_cells(int dtype_bytes, hipStream_t st, const GridDev& g, const int32_t* ccell,
                             int32_t nchares, uint64_t seed) {
    if (nchares <= 0) return hipSuccess;
    dim3 grid(8, (unsigned)(nchares < 65535 ? nchares : 65535));
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_init_cells<double>, grid, dim3(256), 0, st, g, ccell, nchares, seed);
    else
        hipLaunchKernelGGL(k_init_cells<float>, grid, dim3(256), 0, st, g, ccell, nchares, seed);
    return hipGetLastError();
}

template <typename T>
__global__ void k_xexp_refresh(T* __restrict__ arena, const BlockDev* __restrict__ blocks,
                               const XExpDev* __restrict__ xexp, int32_t nchares, int parity) {
    for (int32_t q = blockIdx.y; q < 2 * nchares; q += gridDim.y) {
        const int32_t c = q >> 1, side = q & 1;
        const int64_t eo = xexp[c].off[side][parity];
        if (eo < 0) continue;
        const BlockDev& B = blocks[c];
        const int64_t base = (parity ? B.off[1] : B.off[0]) + (side ? B.ex - 1 : 0);
        const int64_t cnt = (int64_t)B.ey * B.ez;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x) {
            const int64_t y = e % B.ey, z = e / B.ey;
            arena[eo + e] = arena[base + y * B.py + z * B.pz];
        }
    }
}

hipError_t launch_xexp_refresh(int dtype_bytes, hipStream_t st, void* arena, const BlockDev* blocks,
                               const XExpDev* xexp, int32_t nchares, int parity) {
    if (!xexp || nchares <= 0) return hipSuccess;
    const dim3 grid(4, (unsigned)std::min<int32_t>(2 * nchares, 65535));
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_xexp_refresh<double>, grid, dim3(256), 0, st, reinterpret_cast<double*>(arena), blocks,
                           xexp, nchares, parity);
    else
        hipLaunchKernelGGL(k_xexp_refresh<float>, grid, dim3(256), 0, st, reinterpret_cast<float*>(arena), blocks,
                           xexp, nchares, parity);
    return hipGetLastError();
}

hipError_t launch_amr_fill(int dtype_bytes, hipStream_t st, void* arena, const BlockDev* blocks,
                           const FillSeg* segs, int32_t nseg, int64_t total, int parity) {
    if (nseg <= 0 || total <= 0) return hipSuccess;
    const unsigned int grid = (unsigned int)(nseg < (1 << 20) ? nseg : (1 << 20));
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_amr_fill<double>, dim3(grid), dim3(kFillLanes), 0, st, reinterpret_cast<double*>(arena),
                           blocks, segs, nseg, parity);
    else
        hipLaunchKernelGGL(k_amr_fill<float>, dim3(grid), dim3(kFillLanes), 0, st, reinterpret_cast<float*>(arena),
                           blocks, segs, nseg, parity);
    return hipGetLastError();
}

hipError_t launch_gather(int dtype_bytes, hipStream_t st, const GridDev& g, int parity, int64_t kz_lo,
                         int64_t kz_hi, void* dst) {
    const int64_t total = (kz_hi - kz_lo) * (g.n[0] + 2) * (g.n[1] + 2);
    if (total <= 0) return hipSuccess;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_gather<double>, dim3(io_grid(total)), dim3(256), 0, st, g, parity, kz_lo, kz_hi,
                           reinterpret_cast<double*>(dst));
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(io_grid(total)), dim3(256), 0, st, g, parity, kz_lo, kz_hi,
                           reinterpret_cast<float*>(dst));
    return hipGetLastError();
}

hipError_t launch_scatter(int dtype_bytes, hipStream_t st, const GridDev& g, int parity, int64_t kz_lo,
                          int64_t kz_hi, const void* src) {
    const int64_t total = (kz_hi - kz_lo) * (g.n[0] + 2) * (g.n[1] + 2);
    if (total <= 0) return hipSuccess;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_scatter<double>, dim3(io_grid(total)), dim3(256), 0, st, g, parity, kz_lo, kz_hi,
                           reinterpret_cast<const double*>(src));
    else
        hipLaunchKernelGGL(k_scatter<float>, dim3(io_grid(total)), dim3(256), 0, st, g, parity, kz_lo, kz_hi,
                           reinterpret_cast<const float*>(src));
    return hipGetLastError();
}

hipError_t launch_points(int dtype_bytes, hipStream_t st, const GridDev& g, int parity, const int64_t* idx,
                         int64_t count, void* dst) {
    if (count <= 0) return hipSuccess;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_points<double>, dim3(io_grid(count)), dim3(256), 0, st, g, parity, idx, count,
                           reinterpret_cast<double*>(dst));
    else
        hipLaunchKernelGGL(k_points<float>, dim3(io_grid(count)), dim3(256), 0, st, g, parity, idx, count,
                           reinterpret_cast<float*>(dst));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-chare baseline: face messages

// Face f's message layout: x faces [z][y] (y fastest), y faces [z][x] and
// z faces [y][x], both with the chare's row pitch.
template <typename T>
__global__ void k_pack(const T* __restrict__ arena, BlockDev B, int parity, FaceSet out) {
    const int f = blockIdx.y;
    T* m = reinterpret_cast<T*>(out.p[f]);
    if (m == nullptr) return;
    const T* u = arena + B.off[parity];
    const int64_t cnt = out.cnt[f];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t x, y, z;
        if (f < 2) {
            y = e % B.ey;
            z = e / B.ey;
            x = (f == 0) ? 0 : B.ex - 1;
        } else if (f < 4) {
            x = e % B.py;
            z = e / B.py;
            y = (f == 2) ? 0 : B.ey - 1;
            if (x >= B.ex) continue;
        } else {
            x = e % B.py;
            y = e / B.py;
            z = (f == 4) ? 0 : B.ez - 1;
            if (x >= B.ex) continue;
        }
        m[e] = u[x + y * B.py + z * B.pz];
    }
}

template <typename T>
__global__ void k_unpack(FaceSet in, FaceSet ghost) {
    const int f = blockIdx.y;
    const T* s = reinterpret_cast<const T*>(in.p[f]);
    T* d = reinterpret_cast<T*>(ghost.p[f]);
    if (s == nullptr || d == nullptr) return;
    const int64_t cnt = in.cnt[f];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x)
        d[e] = s[e];
}

hipError_t launch_pack_b(int dtype_bytes, hipStream_t st, void* arena, const BlockDev& B, int parity,
                         const FaceSet& out) {
    int64_t mx = 1;
    for (int f = 0; f < 6; ++f) mx = out.cnt[f] > mx ? out.cnt[f] : mx;
    dim3 grid((unsigned)((mx + 255) / 256 < 1024 ? (mx + 255) / 256 : 1024), 6);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_pack<double>, grid, dim3(256), 0, st, reinterpret_cast<const double*>(arena), B, parity, out);
    else
        hipLaunchKernelGGL(k_pack<float>, grid, dim3(256), 0, st, reinterpret_cast<const float*>(arena), B, parity, out);
    return hipGetLastError();
}

hipError_t launch_unpack(int dtype_bytes, hipStream_t st, FaceSet in, FaceSet ghost) {
    int64_t mx = 1;
    for (int f = 0; f < 6; ++f) mx = in.cnt[f] > mx ? in.cnt[f] : mx;
    dim3 grid((unsigned)((mx + 255) / 256 < 1024 ? (mx + 255) / 256 : 1024), 6);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(k_unpack<double>, grid, dim3(256), 0, st, in, ghost);
    else
        hipLaunchKernelGGL(k_unpack<float>, grid, dim3(256), 0, st, in, ghost);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// streaming copy (HBM ceiling)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// HBM ceilings: streaming copy (KIND 0: dst <- src), read-only (KIND 1:
// every 16-byte vector of src is loaded and folded into a per-thread xor
// that is stored only if it equals `key`, which never holds for the data
// used, so the loads stay and nothing is written) and write-only (KIND 2:
// dst <- a per-element pattern).  U independent 16-byte accesses in flight
// per thread, grid-stride over the buffer.
template <int U, bool NT, int KIND>
__global__ void __launch_bounds__(256) k_stream(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int64_t n,
                                                uint32_t key, uint32_t* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (; e + (U - 1) * stride < n; e += U * stride) {
        u32x4 v[U];
        if (KIND != 2) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = NT ? __builtin_nontemporal_load(src + e + u * stride) : src[e + u * stride];
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t x = (uint32_t)(e + u * stride);
                v[u] = u32x4{x, x ^ key, x + key, ~x};
            }
        }
        if (KIND == 1) {
#pragma unroll
            for (int u = 0; u < U; ++u) acc ^= v[u];
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (NT)
                    __builtin_nontemporal_store(v[u], dst + e + u * stride);
                else
                    dst[e + u * stride] = v[u];
            }
        }
    }
    for (; e < n; e += stride) {
        if (KIND == 0) dst[e] = src[e];
        else if (KIND == 1) acc ^= src[e];
        else {
            const uint32_t x = (uint32_t)e;
            dst[e] = u32x4{x, x ^ key, x + key, ~x};
        }
    }
    if (KIND == 1) {
        const uint32_t f = acc[0] ^ acc[1] ^ acc[2] ^ acc[3];
        if (f == key) atomicOr(sink, 1u);
    }
}

// Chunked form: workgroup b streams its own contiguous range of `chunk`
// vectors (a few large sequential streams, which HBM serves faster than an
// interleaved grid stride), U accesses in flight per thread.
template <int U, bool NT, int KIND>
__global__ void __launch_bounds__(1024) k_stream_chunk(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                       int64_t n, int64_t chunk, uint32_t key,
                                                       uint32_t* __restrict__ sink) {
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    const int nt = blockDim.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (int64_t e = b0 + threadIdx.x; e < b1; e += (int64_t)U * nt) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = e + (int64_t)u * nt;
            if (q < b1) {
                if (KIND != 2) {
                    v[u] = NT ? __builtin_nontemporal_load(src + q) : src[q];
                } else {
                    const uint32_t x = (uint32_t)q;
                    v[u] = u32x4{x, x ^ key, x + key, ~x};
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = e + (int64_t)u * nt;
            if (q < b1) {
                if (KIND == 1)
                    acc ^= v[u];
                else if (NT)
                    __builtin_nontemporal_store(v[u], dst + q);
                else
                    dst[q] = v[u];
            }
        }
    }
    if (KIND == 1) {
        const uint32_t f = acc[0] ^ acc[1] ^ acc[2] ^ acc[3];
        if (f == key) atomicOr(sink, 1u);
    }
}

struct CopyVariant {
    int blocks_per_cu, unroll;
    bool nt;
    int chunk_threads;   // 0: grid-stride, 256 threads; else chunked with this many threads
};
static const CopyVariant kCopyVariants[] = {
    {32, 1, false, 0}, {16, 4, false, 0}, {16, 4, true, 0},  {64, 2, false, 0},   {64, 2, true, 0},
    {8, 8, true, 0},   {8, 8, false, 0},  {32, 4, false, 0}, {32, 4, true, 0},    {4, 8, true, 0},
    {1, 8, true, 1024}, {2, 8, true, 1024}, {4, 4, true, 1024}, {8, 8, true, 512}, {1, 4, false, 1024}};

int copy_variant_count() { return (int)(sizeof(kCopyVariants) / sizeof(kCopyVariants[0])); }

hipError_t launch_stream(hipStream_t st, void* dst, const void* src, size_t bytes, int variant, int kind,
                         uint32_t* sink) {
    const int64_t n = (int64_t)(bytes / 16);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 256;
    const CopyVariant& cv = kCopyVariants[variant % copy_variant_count()];
    const uint32_t key0 = 0x9E3779B9u;
    if (cv.chunk_threads > 0) {
        int64_t grid = (int64_t)ncu * cv.blocks_per_cu;
        const int64_t chunk = (n + grid - 1) / grid;
        grid = (n + chunk - 1) / chunk;
        if (grid < 1) grid = 1;
        const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
        u32x4* d4 = reinterpret_cast<u32x4*>(dst);
#define OD_CHUNK(UU, NTT, K)                                                                                   \
        if (cv.unroll == UU && cv.nt == NTT && kind == K) {                                                    \
            hipLaunchKernelGGL((k_stream_chunk<UU, NTT, K>), dim3((unsigned)grid), dim3(cv.chunk_threads), 0, st, \
                               s4, d4, n, chunk, key0, sink);                                                  \
            return hipGetLastError();                                                                          \
        }
#define OD_CHUNK_K(UU, NTT) OD_CHUNK(UU, NTT, 0) OD_CHUNK(UU, NTT, 1) OD_CHUNK(UU, NTT, 2)
        OD_CHUNK_K(8, true)
        OD_CHUNK_K(4, true)
        OD_CHUNK_K(4, false)
#undef OD_CHUNK_K
#undef OD_CHUNK
        return hipErrorInvalidValue;
    }
    int64_t grid = (n + 255) / 256;
    const int64_t cap = (int64_t)ncu * cv.blocks_per_cu;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
    u32x4* d4 = reinterpret_cast<u32x4*>(dst);
    const uint32_t key = 0x9E3779B9u;   // the sink is a valid word: a chance match only sets a bit in it
#define OD_STREAM(UU, NTT, K)                                                                             \
    if (cv.unroll == UU && cv.nt == NTT && kind == K) {                                                   \
        hipLaunchKernelGGL((k_stream<UU, NTT, K>), dim3((unsigned)grid), dim3(256), 0, st, s4, d4, n, key, \
                           sink);                                                                         \
        return hipGetLastError();                                                                         \
    }
#define OD_STREAM_K(UU, NTT) OD_STREAM(UU, NTT, 0) OD_STREAM(UU, NTT, 1) OD_STREAM(UU, NTT, 2)
    OD_STREAM_K(1, false)
    OD_STREAM_K(4, false)
    OD_STREAM_K(4, true)
    OD_STREAM_K(2, false)
    OD_STREAM_K(2, true)
    OD_STREAM_K(8, true)
    OD_STREAM_K(8, false)
#undef OD_STREAM_K
#undef OD_STREAM
    return hipErrorInvalidValue;
}

hipError_t launch_copy(hipStream_t st, void* dst, const void* src, size_t bytes, int variant) {
    return launch_stream(st, dst, src, bytes, variant, 0, nullptr);
}

}  // namespace od
