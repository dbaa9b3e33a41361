/*
 * Reference oracle for multi-resolution block Jacobi (octree leaves that
 * carry their own cell size, coupled across resolution changes by injection
 * and face averaging).
 *
 * TEST INFRASTRUCTURE ONLY, like jacobi_oracle.c (same library, same
 * flags); nothing in the product library links, loads or calls it.
 *
 * The paper motivates overdecomposition with adaptive mesh refinement
 * (Section I) and runs Jacobi iterations with halo exchange between chares
 * (Section V); it fixes no coupling between refinement levels.  Definition
 * used here, written out plainly:
 *   - the domain is nx x ny x nz grid units; block b covers the box
 *     [org_b, org_b + ext_b) (units) and holds (ext_b / h_b) cells per
 *     dimension, each an h_b^3 cube of units (h_b a power of two);
 *   - block b's interior cell (i,j,k) starts at unit q = org_b + (i,j,k)h_b
 *     and is initialised from SplitMix64 at unit index (q_z ny + q_y) nx + q_x
 *     (so h = 1 everywhere is the uniform grid of jacobi_oracle.c);
 *   - every iteration first fills each block's ghost layer from the current
 *     values: a ghost cell outside the domain takes the face's Dirichlet
 *     value; otherwise let N be the block owning the unit just across the
 *     face at the ghost cell's lower tangential corner; if h_N >= h_b the
 *     ghost takes N's cell containing that unit (copy, or injection from a
 *     coarser block); if h_N < h_b (N finer, r = h_b / h_N) it takes the
 *     mean of the r x r cells of N's layer touching the face that cover the
 *     ghost cell's face: summed with the second tangential index outer and
 *     the first inner (tangential axes in x, y, z order), then divided by
 *     r*r;
 *   - then every block does the 7-point Jacobi update of its own cells in
 *     the order of jacobi_oracle.c (x-, x+, y-, y+, z-, z+, then / 6);
 *   - residual = max over all cells of |u_new - u_old|.
 * Layout constraint (checked, -1 otherwise): across a face between blocks
 * with h_a > h_b, the finer block's tangential origin and extent are
 * multiples of h_a, so every averaged patch lies inside one block.
 *
 * Storage: block b's padded array ((m_z+2)(m_y+2)(m_x+2), x fastest, m =
 * ext / h) starts at element offs[b] of one flat array.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

uint64_t oracle_splitmix64(uint64_t seed, uint64_t idx);

static int64_t gcd64(int64_t a, int64_t b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

/* Element offsets of every block's padded array; returns the total count. */
int64_t oracle_ml_layout(int64_t nb, const int64_t* ext, const int64_t* h, int64_t* offs)
{
    int64_t o = 0;
    for (int64_t b = 0; b < nb; ++b) {
        offs[b] = o;
        int64_t m0 = ext[3 * b] / h[b], m1 = ext[3 * b + 1] / h[b], m2 = ext[3 * b + 2] / h[b];
        o += (m0 + 2) * (m1 + 2) * (m2 + 2);
    }
    return o;
}

/* Owner map over the domain at granularity g (units): cell -> block. */
typedef struct {
    int64_t n[3], g, og[3];
    int32_t* own;
} owner_map;

static int owner_build(owner_map* M, int64_t nb, const int64_t* org, const int64_t* ext, const int64_t n[3])
{
    int64_t g = 0;
    for (int d = 0; d < 3; ++d) g = gcd64(g, n[d]);
    for (int64_t b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) {
            g = gcd64(g, org[3 * b + d]);
            g = gcd64(g, ext[3 * b + d]);
        }
    M->g = g;
    for (int d = 0; d < 3; ++d) {
        M->n[d] = n[d];
        M->og[d] = n[d] / g;
    }
    size_t cells = (size_t)(M->og[0] * M->og[1] * M->og[2]);
    M->own = (int32_t*)malloc(cells * sizeof(int32_t));
    if (!M->own) return -1;
    for (size_t i = 0; i < cells; ++i) M->own[i] = -1;
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t z = org[3 * b + 2] / g; z < (org[3 * b + 2] + ext[3 * b + 2]) / g; ++z)
            for (int64_t y = org[3 * b + 1] / g; y < (org[3 * b + 1] + ext[3 * b + 1]) / g; ++y)
                for (int64_t x = org[3 * b] / g; x < (org[3 * b] + ext[3 * b]) / g; ++x)
                    M->own[(z * M->og[1] + y) * M->og[0] + x] = (int32_t)b;
    for (size_t i = 0; i < cells; ++i)
        if (M->own[i] < 0) return -1;
    return 0;
}

static int32_t owner_at(const owner_map* M, const int64_t p[3])
{
    return M->own[((p[2] / M->g) * M->og[1] + p[1] / M->g) * M->og[0] + p[0] / M->g];
}

#define PADI(i, j, k, m) ((((int64_t)(k) + 1) * ((m)[1] + 2) + ((int64_t)(j) + 1)) * ((m)[0] + 2) + ((int64_t)(i) + 1))

#define ML_DEFINE(T, SUF, UNIF)                                                                     \
void oracle_ml_init_##SUF(T* U, int64_t nb, const int64_t* org, const int64_t* ext, const int64_t* h, \
                          const int64_t* offs, int64_t nx, int64_t ny, int64_t nz, uint64_t seed)   \
{                                                                                                   \
    (void)nz;                                                                                       \
    for (int64_t b = 0; b < nb; ++b) {                                                              \
        int64_t m[3];                                                                               \
        for (int d = 0; d < 3; ++d) m[d] = ext[3 * b + d] / h[b];                                   \
        T* A = U + offs[b];                                                                         \
        memset(A, 0, sizeof(T) * (size_t)((m[0] + 2) * (m[1] + 2) * (m[2] + 2)));                  \
        for (int64_t k = 0; k < m[2]; ++k)                                                          \
            for (int64_t j = 0; j < m[1]; ++j)                                                      \
                for (int64_t i = 0; i < m[0]; ++i) {                                                \
                    int64_t qx = org[3 * b] + i * h[b], qy = org[3 * b + 1] + j * h[b];             \
                    int64_t qz = org[3 * b + 2] + k * h[b];                                         \
                    uint64_t g = (uint64_t)((qz * ny + qy) * nx + qx);                              \
                    A[PADI(i, j, k, m)] = UNIF(oracle_splitmix64(seed, g));                         \
                }                                                                                   \
    }                                                                                               \
}                                                                                                   \
                                                                                                    \
/* ghost layer of every block from the current values (see header) */                              \
static int ml_fill_##SUF(T* U, int64_t nb, const int64_t* org, const int64_t* ext, const int64_t* h, \
                         const int64_t* offs, const owner_map* M, const double* bc)                 \
{                                                                                                   \
    int bad = 0;                                                                                    \
    _Pragma("omp parallel for schedule(dynamic, 16) reduction(|:bad)")                              \
    for (int64_t b = 0; b < nb; ++b) {                                                              \
        int64_t m[3];                                                                               \
        for (int d = 0; d < 3; ++d) m[d] = ext[3 * b + d] / h[b];                                   \
        T* A = U + offs[b];                                                                         \
        for (int f = 0; f < 6; ++f) {                                                               \
            const int d = f / 2, hi = f % 2;                                                        \
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;                                     \
            for (int64_t c2 = 0; c2 < m[t2]; ++c2)                                                  \
                for (int64_t c1 = 0; c1 < m[t1]; ++c1) {                                            \
                    int64_t gi[3];                     /* ghost cell, block-local */                \
                    gi[t1] = c1;                                                                    \
                    gi[t2] = c2;                                                                    \
                    gi[d] = hi ? m[d] : -1;                                                         \
                    T v;                                                                            \
                    int64_t p[3];                      /* unit just across the face */              \
                    p[t1] = org[3 * b + t1] + c1 * h[b];                                            \
                    p[t2] = org[3 * b + t2] + c2 * h[b];                                            \
                    p[d] = hi ? org[3 * b + d] + ext[3 * b + d] : org[3 * b + d] - 1;               \
                    if (p[d] < 0 || p[d] >= M->n[d]) {                                              \
                        v = (T)bc[f];                                                               \
                    } else {                                                                        \
                        const int64_t N = owner_at(M, p);                                           \
                        int64_t mn[3];                                                              \
                        for (int q = 0; q < 3; ++q) mn[q] = ext[3 * N + q] / h[N];                  \
                        const T* B = U + offs[N];                                                   \
                        int64_t ni[3];                                                              \
                        for (int q = 0; q < 3; ++q) ni[q] = (p[q] - org[3 * N + q]) / h[N];         \
                        if (h[N] >= h[b]) {                                                         \
                            v = B[PADI(ni[0], ni[1], ni[2], mn)];                                   \
                        } else {                                                                    \
                            const int64_t r = h[b] / h[N];                                          \
                            if (ni[t1] + r > mn[t1] || ni[t2] + r > mn[t2]) {                       \
                                bad = 1;                                                            \
                                continue;                                                           \
                            }                                                                       \
                            T s = 0;                                                                \
                            int first = 1;                                                          \
                            for (int64_t q2 = 0; q2 < r; ++q2)                                      \
                                for (int64_t q1 = 0; q1 < r; ++q1) {                                \
                                    int64_t w[3] = {ni[0], ni[1], ni[2]};                           \
                                    w[t1] += q1;                                                    \
                                    w[t2] += q2;                                                    \
                                    const T x = B[PADI(w[0], w[1], w[2], mn)];                      \
                                    s = first ? x : (T)(s + x);                                     \
                                    first = 0;                                                      \
                                }                                                                   \
                            v = (T)(s / (T)(r * r));                                                \
                        }                                                                           \
                    }                                                                               \
                    A[PADI(gi[0], gi[1], gi[2], m)] = v;                                            \
                }                                                                                   \
        }                                                                                           \
    }                                                                                               \
    return bad ? -1 : 0;                                                                            \
}                                                                                                   \
                                                                                                    \
/* one Jacobi update of every block's cells from U (ghosts filled) into V */                        \
static T ml_sweep_##SUF(const T* U, T* V, int64_t nb, const int64_t* ext, const int64_t* h,         \
                        const int64_t* offs)                                                        \
{                                                                                                   \
    T r = 0;                                                                                        \
    _Pragma("omp parallel for schedule(dynamic, 16) reduction(max:r)")                              \
    for (int64_t b = 0; b < nb; ++b) {                                                              \
        int64_t m[3];                                                                               \
        for (int d = 0; d < 3; ++d) m[d] = ext[3 * b + d] / h[b];                                   \
        const T* A = U + offs[b];                                                                   \
        T* W = V + offs[b];                                                                         \
        for (int64_t k = 0; k < m[2]; ++k)                                                          \
            for (int64_t j = 0; j < m[1]; ++j)                                                      \
                for (int64_t i = 0; i < m[0]; ++i) {                                                \
                    T s = A[PADI(i - 1, j, k, m)];                                                  \
                    s = (T)(s + A[PADI(i + 1, j, k, m)]);                                           \
                    s = (T)(s + A[PADI(i, j - 1, k, m)]);                                           \
                    s = (T)(s + A[PADI(i, j + 1, k, m)]);                                           \
                    s = (T)(s + A[PADI(i, j, k - 1, m)]);                                           \
                    s = (T)(s + A[PADI(i, j, k + 1, m)]);                                           \
                    const T v = (T)(s / (T)6);                                                      \
                    T dv = (T)(v - A[PADI(i, j, k, m)]);                                            \
                    if (dv < 0) dv = -dv;                                                           \
                    if (dv > r) r = dv;                                                             \
                    W[PADI(i, j, k, m)] = v;                                                        \
                }                                                                                   \
    }                                                                                               \
    return r;                                                                                       \
}                                                                                                   \
                                                                                                    \
/* iters x (fill ghosts, update); the result ends in U.  Returns iterations  \
 * done, or -1 for a layout the definition does not cover. */                                       \
int64_t oracle_ml_jacobi_##SUF(T* U, T* V, int64_t nb, const int64_t* org, const int64_t* ext,      \
                               const int64_t* h, const int64_t* offs, int64_t nx, int64_t ny,       \
                               int64_t nz, const double* bc, int64_t iters, double* res_out)        \
{                                                                                                   \
    owner_map M;                                                                                    \
    const int64_t n[3] = {nx, ny, nz};                                                              \
    if (owner_build(&M, nb, org, ext, n) != 0) {                                                    \
        free(M.own);                                                                                \
        return -1;                                                                                  \
    }                                                                                               \
    int64_t total = 0;                                                                              \
    for (int64_t b = 0; b < nb; ++b)                                                                \
        total += (ext[3 * b] / h[b] + 2) * (ext[3 * b + 1] / h[b] + 2) * (ext[3 * b + 2] / h[b] + 2); \
    T r = 0;                                                                                        \
    int64_t it = 0;                                                                                 \
    for (; it < iters; ++it) {                                                                      \
        if (ml_fill_##SUF(U, nb, org, ext, h, offs, &M, bc) != 0) {                                 \
            free(M.own);                                                                            \
            return -1;                                                                              \
        }                                                                                           \
        r = ml_sweep_##SUF(U, V, nb, ext, h, offs);                                                 \
        memcpy(U, V, sizeof(T) * (size_t)total); /* ghost layers are refilled next iteration */     \
    }                                                                                               \
    free(M.own);                                                                                    \
    *res_out = (double)r;                                                                           \
    return it;                                                                                      \
}

#define ML_UNIF_F64(x) ((double)((x) >> 11) * 0x1.0p-53)
#define ML_UNIF_F32(x) ((float)((x) >> 40) * 0x1.0p-24f)

ML_DEFINE(double, f64, ML_UNIF_F64)
ML_DEFINE(float, f32, ML_UNIF_F32)
