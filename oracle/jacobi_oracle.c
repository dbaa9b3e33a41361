/*
 * Reference oracle for the overdecomposed Jacobi hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU path.
 *
 * What it computes is the plain, undecomposed definition of the method: the
 * Jacobi iterative method over one global structured grid with halo
 * (ghost) values held fixed (Section V, Jacobi2D workload: "Jacobi iterative
 * method on a grid ... halo exchanges ... iterations without convergence
 * checks").  Overdecomposition (Section III) splits that grid into chares
 * but, by construction, must not change what is computed; this file is the
 * result every decomposition has to reproduce bit for bit.
 *
 * Readings taken where the paper is silent (the paper fixes neither the
 * stencil's dimension for this workload, nor precision, boundary values,
 * summation order or residual norm):
 *   - 3D 7-point stencil, u'(i,j,k) = mean of the six face neighbours;
 *   - the six neighbours are added left to right in the order
 *     x-, x+, y-, y+, z-, z+, each addition rounded to T, then the sum is
 *     divided by 6 with one correctly rounded IEEE division;
 *   - storage is a padded (nz+2)(ny+2)(nx+2) array, x fastest, interior
 *     indices 0..n-1, ghost shell at -1 and n, held fixed (Dirichlet);
 *   - residual = max over interior points of |u_new - u_old| (max-norm of
 *     the update), exact in any evaluation order;
 *   - initial interior values come from SplitMix64 (Steele, Lea and Flood,
 *     "Fast splittable pseudorandom number generators", OOPSLA 2014): the
 *     value at global linear index g = (k*ny + j)*nx + i is the (g+1)-th
 *     output of the stream seeded with `seed`, mapped to [0,1) by keeping
 *     the top 53 (double) or 24 (float) bits.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * The OpenMP loop over z-planes only distributes independent points; the
 * per-point arithmetic and the max reduction are order independent.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- SplitMix64, written from its published definition ---------------- */
/* The generator's state advances by the odd constant GOLDEN; each output is
 * the state passed through the 64-bit finaliser (xor-shift / multiply
 * rounds with the constants of the published generator). */
#define SM64_GOLDEN 0x9E3779B97F4A7C15ULL

static uint64_t sm64_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* idx-th output (0-based) of the SplitMix64 stream seeded with `seed`. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t idx)
{
    return sm64_finalise(seed + (idx + 1ULL) * SM64_GOLDEN);
}

/* ---- threads ------------------------------------------------------------ */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- padded-array helpers ------------------------------------------------ */
#define PIDX(i, j, k, nx, ny) \
    ((((int64_t)(k) + 1) * ((int64_t)(ny) + 2) + ((int64_t)(j) + 1)) * ((int64_t)(nx) + 2) + ((int64_t)(i) + 1))

/*
 * One generic body per precision T.  Each function is written out once by
 * the macro below so the two precisions cannot drift apart.
 */
#define ORACLE_DEFINE(T, SUF, UNIF)                                                          \
                                                                                             \
/* Fill the padded array: ghost faces from bc (x-,x+,y-,y+,z-,z+), edges and \
 * corners of the shell (never read by a 7-point stencil) zero, interior     \
 * from SplitMix64. */                                                       \
void oracle_init_##SUF(T* U, int64_t nx, int64_t ny, int64_t nz, uint64_t seed,           \
                       const double bc[6])                                                 \
{                                                                                            \
    for (int64_t k = -1; k <= nz; ++k)                                                       \
        for (int64_t j = -1; j <= ny; ++j)                                                   \
            for (int64_t i = -1; i <= nx; ++i) {                                             \
                int out = (i < 0 || i >= nx) + (j < 0 || j >= ny) + (k < 0 || k >= nz);      \
                T v;                                                                         \
                if (out == 0) {                                                              \
                    uint64_t g = (uint64_t)((k * ny + j) * nx + i);                          \
                    v = UNIF(oracle_splitmix64(seed, g));                                    \
                } else if (out >= 2) {                                                       \
                    v = (T)0;                                                                \
                } else if (i < 0) {                                                          \
                    v = (T)bc[0];                                                            \
                } else if (i >= nx) {                                                        \
                    v = (T)bc[1];                                                            \
                } else if (j < 0) {                                                          \
                    v = (T)bc[2];                                                            \
                } else if (j >= ny) {                                                        \
                    v = (T)bc[3];                                                            \
                } else if (k < 0) {                                                          \
                    v = (T)bc[4];                                                            \
                } else {                                                                     \
                    v = (T)bc[5];                                                            \
                }                                                                            \
                U[PIDX(i, j, k, nx, ny)] = v;                                                \
            }                                                                                \
}                                                                                            \
                                                                                             \
/* Padded sub-box of the initial global field: box interior cells are the   \
 * global interior cells (ox..ox+bx-1, ...), the box shell holds whatever    \
 * the global padded field holds there (initial values inside the domain,   \
 * Dirichlet faces outside, zero on shell edges).  Used to evaluate single  \
 * outputs by domain of dependence. */                                       \
void oracle_init_box_##SUF(T* U, int64_t nx, int64_t ny, int64_t nz, uint64_t seed,        \
                           const double bc[6], int64_t ox, int64_t oy, int64_t oz,           \
                           int64_t bx, int64_t by, int64_t bz)                               \
{                                                                                            \
    for (int64_t k = -1; k <= bz; ++k)                                                       \
        for (int64_t j = -1; j <= by; ++j)                                                   \
            for (int64_t i = -1; i <= bx; ++i) {                                             \
                int64_t gi = ox + i, gj = oy + j, gk = oz + k;                               \
                int out = (gi < 0 || gi >= nx) + (gj < 0 || gj >= ny) + (gk < 0 || gk >= nz);\
                T v;                                                                         \
                if (gi < -1 || gi > nx || gj < -1 || gj > ny || gk < -1 || gk > nz) {        \
                    v = (T)0;                                                                \
                } else if (out == 0) {                                                       \
                    uint64_t g = (uint64_t)((gk * ny + gj) * nx + gi);                       \
                    v = UNIF(oracle_splitmix64(seed, g));                                    \
                } else if (out >= 2) {                                                       \
                    v = (T)0;                                                                \
                } else if (gi < 0) {                                                         \
                    v = (T)bc[0];                                                            \
                } else if (gi >= nx) {                                                       \
                    v = (T)bc[1];                                                            \
                } else if (gj < 0) {                                                         \
                    v = (T)bc[2];                                                            \
                } else if (gj >= ny) {                                                       \
                    v = (T)bc[3];                                                            \
                } else if (gk < 0) {                                                         \
                    v = (T)bc[4];                                                            \
                } else {                                                                     \
                    v = (T)bc[5];                                                            \
                }                                                                            \
                U[PIDX(i, j, k, bx, by)] = v;                                                \
            }                                                                                \
}                                                                                            \
                                                                                             \
/* One Jacobi sweep U -> V over the interior; V's ghost shell is not touched. \
 * Returns max |V - U| over the interior. */                                 \
T oracle_sweep_##SUF(const T* U, T* V, int64_t nx, int64_t ny, int64_t nz)                 \
{                                                                                            \
    T r = (T)0;                                                                              \
    _Pragma("omp parallel for schedule(static) reduction(max : r)")                         \
    for (int64_t k = 0; k < nz; ++k)                                                         \
        for (int64_t j = 0; j < ny; ++j)                                                     \
            for (int64_t i = 0; i < nx; ++i) {                                               \
                T s = U[PIDX(i - 1, j, k, nx, ny)];                                          \
                s = s + U[PIDX(i + 1, j, k, nx, ny)];                                        \
                s = s + U[PIDX(i, j - 1, k, nx, ny)];                                        \
                s = s + U[PIDX(i, j + 1, k, nx, ny)];                                        \
                s = s + U[PIDX(i, j, k - 1, nx, ny)];                                        \
                s = s + U[PIDX(i, j, k + 1, nx, ny)];                                        \
                T v = s / (T)6;                                                              \
                T u = U[PIDX(i, j, k, nx, ny)];                                              \
                T d = v - u;                                                                 \
                if (d < (T)0) d = -d;                                                        \
                if (d > r) r = d;                                                            \
                V[PIDX(i, j, k, nx, ny)] = v;                                                \
            }                                                                                \
    return r;                                                                                \
}                                                                                            \
                                                                                             \
/* Iterate from the padded field U (ghost shell included).  V is scratch of \
 * the same size.  Stops after iteration `it` when check_every > 0,          \
 * it % check_every == 0 and residual < tol (strict), or after max_iters.    \
 * The final field is left in U.  Returns iterations done; *residual gets   \
 * the last sweep's residual (0 when no sweep ran). */                       \
int64_t oracle_jacobi_##SUF(T* U, T* V, int64_t nx, int64_t ny, int64_t nz,                \
                            int64_t max_iters, double tol, int64_t check_every,            \
                            double* residual)                                               \
{                                                                                            \
    size_t total = (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2);                   \
    memcpy(V, U, total * sizeof(T));                                                         \
    T* a = U;                                                                                \
    T* b = V;                                                                                \
    T r = (T)0;                                                                              \
    int64_t it = 0;                                                                          \
    while (it < max_iters) {                                                                 \
        r = oracle_sweep_##SUF(a, b, nx, ny, nz);                                            \
        ++it;                                                                                \
        T* t = a; a = b; b = t;                                                              \
        if (check_every > 0 && it % check_every == 0 && (double)r < tol) break;              \
    }                                                                                        \
    if (a != U) memcpy(U, a, total * sizeof(T));                                             \
    if (residual) *residual = (double)r;                                                     \
    return it;                                                                               \
}

/*
 * The paper's own workload, Jacobi2D (Section V): the same iteration on a
 * 2D grid, 5-point stencil u'(i,j) = mean of the four edge neighbours,
 * added in the order x-, x+, y-, y+ and divided by 4.  Padded array
 * (ny+2)(nx+2), x fastest; bc = {x-, x+, y-, y+}; shell corners zero;
 * interior value at g = j*nx + i from SplitMix64 as in 3D.
 */
#define PIDX2(i, j, nx) ((((int64_t)(j) + 1) * ((int64_t)(nx) + 2)) + ((int64_t)(i) + 1))

#define ORACLE2D_DEFINE(T, SUF, UNIF)                                                        \
void oracle_init2d_##SUF(T* U, int64_t nx, int64_t ny, uint64_t seed, const double bc[4])  \
{                                                                                            \
    for (int64_t j = -1; j <= ny; ++j)                                                       \
        for (int64_t i = -1; i <= nx; ++i) {                                                 \
            int out = (i < 0 || i >= nx) + (j < 0 || j >= ny);                               \
            T v;                                                                             \
            if (out == 0) v = UNIF(oracle_splitmix64(seed, (uint64_t)(j * nx + i)));         \
            else if (out == 2) v = (T)0;                                                     \
            else if (i < 0) v = (T)bc[0];                                                    \
            else if (i >= nx) v = (T)bc[1];                                                  \
            else if (j < 0) v = (T)bc[2];                                                    \
            else v = (T)bc[3];                                                               \
            U[PIDX2(i, j, nx)] = v;                                                          \
        }                                                                                    \
}                                                                                            \
                                                                                             \
/* Padded sub-box (bx, by at global origin ox, oy) of the initial 2D field,  \
 * shell included, for evaluating single outputs by domain of dependence. */ \
void oracle_init2d_box_##SUF(T* U, int64_t nx, int64_t ny, uint64_t seed, const double bc[4], \
                             int64_t ox, int64_t oy, int64_t bx, int64_t by)               \
{                                                                                            \
    for (int64_t j = -1; j <= by; ++j)                                                       \
        for (int64_t i = -1; i <= bx; ++i) {                                                 \
            int64_t gi = ox + i, gj = oy + j;                                                \
            int out = (gi < 0 || gi >= nx) + (gj < 0 || gj >= ny);                           \
            T v;                                                                             \
            if (out == 0) v = UNIF(oracle_splitmix64(seed, (uint64_t)(gj * nx + gi)));      \
            else if (out == 2) v = (T)0;                                                     \
            else if (gi < 0) v = (T)bc[0];                                                   \
            else if (gi >= nx) v = (T)bc[1];                                                 \
            else if (gj < 0) v = (T)bc[2];                                                   \
            else v = (T)bc[3];                                                               \
            U[PIDX2(i, j, bx)] = v;                                                          \
        }                                                                                    \
}                                                                                            \
                                                                                             \
T oracle_sweep2d_##SUF(const T* U, T* V, int64_t nx, int64_t ny)                           \
{                                                                                            \
    T r = (T)0;                                                                              \
    _Pragma("omp parallel for schedule(static) reduction(max : r)")                         \
    for (int64_t j = 0; j < ny; ++j)                                                         \
        for (int64_t i = 0; i < nx; ++i) {                                                   \
            T s = U[PIDX2(i - 1, j, nx)];                                                    \
            s = s + U[PIDX2(i + 1, j, nx)];                                                  \
            s = s + U[PIDX2(i, j - 1, nx)];                                                  \
            s = s + U[PIDX2(i, j + 1, nx)];                                                  \
            T v = s / (T)4;                                                                  \
            T d = v - U[PIDX2(i, j, nx)];                                                    \
            if (d < (T)0) d = -d;                                                            \
            if (d > r) r = d;                                                                \
            V[PIDX2(i, j, nx)] = v;                                                          \
        }                                                                                    \
    return r;                                                                                \
}                                                                                            \
                                                                                             \
int64_t oracle_jacobi2d_##SUF(T* U, T* V, int64_t nx, int64_t ny, int64_t max_iters,        \
                              double tol, int64_t check_every, double* residual)             \
{                                                                                            \
    size_t total = (size_t)(nx + 2) * (size_t)(ny + 2);                                      \
    memcpy(V, U, total * sizeof(T));                                                         \
    T* a = U;                                                                                \
    T* b = V;                                                                                \
    T r = (T)0;                                                                              \
    int64_t it = 0;                                                                          \
    while (it < max_iters) {                                                                 \
        r = oracle_sweep2d_##SUF(a, b, nx, ny);                                              \
        ++it;                                                                                \
        T* t = a; a = b; b = t;                                                              \
        if (check_every > 0 && it % check_every == 0 && (double)r < tol) break;              \
    }                                                                                        \
    if (a != U) memcpy(U, a, total * sizeof(T));                                             \
    if (residual) *residual = (double)r;                                                     \
    return it;                                                                               \
}

#define UNIF_F64(h) ((double)((h) >> 11) * 0x1.0p-53)
#define UNIF_F32(h) ((float)((h) >> 40) * 0x1.0p-24f)

ORACLE_DEFINE(double, f64, UNIF_F64)
ORACLE_DEFINE(float, f32, UNIF_F32)
ORACLE2D_DEFINE(double, f64, UNIF_F64)
ORACLE2D_DEFINE(float, f32, UNIF_F32)
