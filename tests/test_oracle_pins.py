"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something a plausible mistake would
break: published generator outputs, closed forms, invariants of the
discrete Laplacian, symmetry, and an independent pure-Python brute force.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---- SplitMix64: published reference outputs -------------------------------

def test_splitmix64_published_vectors(oracle_mod):
    g = _golden("splitmix64_vectors.json")
    for case in g["cases"]:
        seed = case["seed"]
        for idx, want in enumerate(case["outputs"]):
            assert oracle_mod.splitmix64(seed, idx) == want
            assert brute.splitmix64(seed, idx) == want


def test_init_maps_linear_index_to_stream_position(oracle_mod):
    # A 5x1x1 interior takes the first five outputs of the stream, x fastest;
    # a 1x1x5 grid (z fastest varying index) must take the same five values.
    g = _golden("splitmix64_vectors.json")["cases"][0]
    seed, outs = g["seed"], g["outputs"]
    for dims in ((5, 1, 1), (1, 5, 1), (1, 1, 5)):
        U = oracle_mod.init_field(dims, np.float64, seed, bc=(9, 9, 9, 9, 9, 9))
        interior = U[1:-1, 1:-1, 1:-1].reshape(-1)
        want = np.array([(h >> 11) * 2.0 ** -53 for h in outs])
        assert np.array_equal(interior, want)
        U32 = oracle_mod.init_field(dims, np.float32, seed, bc=(9, 9, 9, 9, 9, 9))
        want32 = np.array([(h >> 40) * 2.0 ** -24 for h in outs], dtype=np.float32)
        assert np.array_equal(U32[1:-1, 1:-1, 1:-1].reshape(-1), want32)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_init_ghost_shell_and_range(oracle_mod, dtype):
    bc = (1.0, 0.25, 0.5, 0.125, 2.0, 4.0)
    nx, ny, nz = 6, 5, 4
    U = oracle_mod.init_field((nx, ny, nz), dtype, 7, bc)
    assert U.shape == (nz + 2, ny + 2, nx + 2)
    I = U[1:-1, 1:-1, 1:-1]
    assert I.min() >= 0.0 and I.max() < 1.0
    assert np.all(U[1:-1, 1:-1, 0] == dtype(bc[0]))
    assert np.all(U[1:-1, 1:-1, -1] == dtype(bc[1]))
    assert np.all(U[1:-1, 0, 1:-1] == dtype(bc[2]))
    assert np.all(U[1:-1, -1, 1:-1] == dtype(bc[3]))
    assert np.all(U[0, 1:-1, 1:-1] == dtype(bc[4]))
    assert np.all(U[-1, 1:-1, 1:-1] == dtype(bc[5]))
    # edges and corners of the shell are zero
    assert U[0, 0, 0] == 0 and U[0, 0, 3] == 0 and U[3, 0, 0] == 0 and U[-1, -1, -1] == 0


# ---- invariants of the discrete Laplacian -----------------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_constant_field_is_fixed(oracle_mod, dtype):
    c = 0.75
    U = oracle_mod.init_field((7, 6, 5), dtype, 1, bc=(c,) * 6)
    U[...] = dtype(c)
    out, it, r = oracle_mod.jacobi(U, 13)
    assert it == 13 and r == 0.0
    assert np.all(out[1:-1, 1:-1, 1:-1] == dtype(c))


def _linear_field(nx, ny, nz, dtype, a=3.0, b=1.0, c=-2.0, d=5.0):
    k, j, i = np.meshgrid(np.arange(-1, nz + 1), np.arange(-1, ny + 1),
                          np.arange(-1, nx + 1), indexing="ij")
    return (a + b * i + c * j + d * k).astype(dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_linear_field_is_fixed(oracle_mod, dtype):
    # A linear function is discrete-harmonic: its six face neighbours sum
    # to exactly 6u, so with matching Dirichlet values it is a fixed point.
    U = _linear_field(9, 7, 8, dtype)
    out, it, r = oracle_mod.jacobi(U, 5)
    assert r == 0.0
    assert np.array_equal(out, U)


def test_linear_field_catches_a_dropped_or_swapped_term(oracle_mod):
    # One sweep must change nothing; a field that is linear in x only checks
    # that x- and x+ both enter with weight 1/6 (a dropped or doubled term
    # would move the interior).
    U = _linear_field(6, 6, 6, np.float64, a=0.0, b=1.0, c=0.0, d=0.0)
    V, r = oracle_mod.sweep(U)
    assert r == 0.0 and np.array_equal(V, U)


# ---- closed form: eigenfunctions of the Jacobi operator ---------------------

@pytest.mark.parametrize("pqr", [(1, 1, 1), (2, 1, 3), (4, 2, 1)])
def test_spectral_eigenfunction(oracle_mod, pqr):
    nx, ny, nz = 10, 8, 6
    p, q, r_ = pqr
    k, j, i = np.meshgrid(np.arange(-1, nz + 1), np.arange(-1, ny + 1),
                          np.arange(-1, nx + 1), indexing="ij")
    U = (np.sin(np.pi * p * (i + 1) / (nx + 1)) * np.sin(np.pi * q * (j + 1) / (ny + 1))
         * np.sin(np.pi * r_ * (k + 1) / (nz + 1)))
    # the Dirichlet shell is zero (sin vanishes there up to rounding)
    U[:, :, 0] = U[:, :, -1] = 0
    U[:, 0, :] = U[:, -1, :] = 0
    U[0, :, :] = U[-1, :, :] = 0
    lam = (np.cos(np.pi * p / (nx + 1)) + np.cos(np.pi * q / (ny + 1))
           + np.cos(np.pi * r_ / (nz + 1))) / 3.0
    V, _ = oracle_mod.sweep(U)
    err = np.abs(V[1:-1, 1:-1, 1:-1] - lam * U[1:-1, 1:-1, 1:-1]).max()
    assert err < 1e-15


def test_residual_decay_rate_is_spectral_radius(oracle_mod):
    # Max-norm of the update decays like rho^t with rho = cos(pi/(N+1));
    # the update's shape has period 2 (the +rho and -rho modes), so compare
    # two steps apart.
    n = 8
    U0 = oracle_mod.init_field(n, np.float64, 5)
    rs = []
    U = U0
    for t in range(304):
        U, r = oracle_mod.sweep(U)
        rs.append(r)
    rho = math.cos(math.pi / (n + 1))
    assert abs(rs[302] / rs[300] - rho ** 2) < 1e-6


# ---- symmetry and superposition -------------------------------------------

def test_face_superposition_and_centre_value(oracle_mod):
    # With bc = 1 on one face and 0 elsewhere, summing the six single-face
    # solutions gives the all-ones solution; by cube symmetry each one is
    # 1/6 at the centre of an odd grid.
    n = 9
    total = None
    centre = []
    for f in range(6):
        bc = [0.0] * 6
        bc[f] = 1.0
        U = oracle_mod.init_field(n, np.float64, 3, bc)
        U[1:-1, 1:-1, 1:-1] = 0.0
        out, it, r = oracle_mod.jacobi(U, 5000, tol=1e-15, check_every=1)
        assert r < 1e-15
        I = out[1:-1, 1:-1, 1:-1]
        centre.append(I[n // 2, n // 2, n // 2])
        total = I if total is None else total + I
    assert np.abs(total - 1.0).max() < 1e-12
    for c in centre:
        assert abs(c - 1.0 / 6.0) < 1e-13
    # orientation: with bc on x- the values fall with i
    bc = [1.0, 0, 0, 0, 0, 0]
    U = oracle_mod.init_field(n, np.float64, 3, bc)
    U[1:-1, 1:-1, 1:-1] = 0.0
    out, _, _ = oracle_mod.jacobi(U, 2000)
    row = out[n // 2 + 1, n // 2 + 1, 1:-1]
    assert np.all(np.diff(row) < 0)


# ---- stopping rule ----------------------------------------------------------

def test_stopping_rule_first_checked_iteration_below_tol(oracle_mod):
    U0 = oracle_mod.init_field(6, np.float64, 11)
    rs, U = [], U0
    for _ in range(400):
        U, r = oracle_mod.sweep(U)
        rs.append(r)
    tol, every = 1e-3, 7
    want = next(t for t in range(every, 401, every) if rs[t - 1] < tol)
    out, it, r = oracle_mod.jacobi(U0, 400, tol=tol, check_every=every)
    assert it == want and r == rs[want - 1]


# ---- independent brute force -------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("dims", [(5, 4, 3), (6, 6, 6), (1, 7, 2)])
def test_brute_force_bit_identical(oracle_mod, dtype, dims):
    nx, ny, nz = dims
    bc = (1.0, 0.0, 0.5, 0.0, 0.0, 0.25)
    seed = 12734
    Ub = brute.init_field(nx, ny, nz, dtype, seed, bc)
    Uc = oracle_mod.init_field(dims, dtype, seed, bc)
    assert np.array_equal(brute.to_numpy(Ub, dtype), Uc)
    Ob, itb, rb = brute.jacobi(Ub, 6)
    Oc, itc, rc = oracle_mod.jacobi(Uc, 6)
    assert itb == itc == 6
    assert np.array_equal(brute.to_numpy(Ob, dtype), Oc)
    assert rb == rc


def test_threads_do_not_change_bits(oracle_mod):
    U = oracle_mod.init_field((17, 9, 13), np.float64, 2)
    oracle_mod.set_threads(1)
    a, _, ra = oracle_mod.jacobi(U, 20)
    oracle_mod.set_threads(4)
    b, _, rb = oracle_mod.jacobi(U, 20)
    oracle_mod.set_threads(oracle_mod.max_threads())
    assert np.array_equal(a, b) and ra == rb


# ---- the mean is one correctly rounded division of the rounded sum ----------

def _round_fraction(q, dtype):
    """Round an exact rational to the nearest dtype value (ties to even)."""
    from fractions import Fraction
    x = dtype(float(q))
    best = None
    for c in (np.nextafter(x, dtype(-np.inf)), x, np.nextafter(x, dtype(np.inf))):
        d = abs(Fraction(float(c)) - q)
        key = (d, int(np.frombuffer(np.array([c], dtype=dtype).tobytes(),
                                    dtype=np.uint64 if dtype == np.float64 else np.uint32)[0]) & 1)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_division_by_six_is_correctly_rounded(oracle_mod, dtype):
    from fractions import Fraction
    rng = np.random.default_rng(0)
    n = 6
    U = oracle_mod.init_field(n, dtype, 99)
    U[1:-1, 1:-1, 1:-1] = rng.random((n, n, n)).astype(dtype)
    V, _ = oracle_mod.sweep(U)
    mism = 0
    for k in range(1, n + 1):
        for j in range(1, n + 1):
            for i in range(1, n + 1):
                s = U[k, j, i - 1]
                for v in (U[k, j, i + 1], U[k, j - 1, i], U[k, j + 1, i], U[k - 1, j, i], U[k + 1, j, i]):
                    s = dtype(s + v)
                want = _round_fraction(Fraction(float(s)) / 6, dtype)
                assert V[k, j, i] == want
                # the reciprocal-multiply shortcut differs on a sizeable share
                if dtype(s * dtype(1.0 / 6.0)) != want:
                    mism += 1
    assert mism > 0


# ---- domain-of-dependence point evaluation (used at sizes the full oracle
# cannot reach) agrees with the full oracle everywhere ------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_point_values_match_full_oracle(oracle_mod, dtype):
    n = (11, 9, 7)
    bc = (1.0, 0.0, 0.25, 0.0, 0.5, 0.0)
    full, _, _ = oracle_mod.solve(n, dtype, seed=4, iters=5, bc=bc)
    rng = np.random.default_rng(1)
    pts = [(int(rng.integers(0, n[0])), int(rng.integers(0, n[1])), int(rng.integers(0, n[2])))
           for _ in range(40)] + [(0, 0, 0), (10, 8, 6), (5, 0, 6)]
    vals = oracle_mod.point_values(n, pts, 5, dtype, seed=4, bc=bc)
    want = np.array([full[k + 1, j + 1, i + 1] for (i, j, k) in pts], dtype=dtype)
    assert np.array_equal(vals, want)


# ---- Jacobi2D (the paper's own workload, Section V) -------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_2d_brute_force_bit_identical(oracle_mod, dtype):
    bc = (1.0, 0.0, 0.5, 0.25)
    for nx, ny in ((7, 5), (1, 6), (9, 9)):
        Ub = brute.init_field2d(nx, ny, dtype, 9, bc)
        Uc = oracle_mod.init_field2d((nx, ny), dtype, 9, bc)
        assert np.array_equal(np.array(Ub, dtype=dtype), Uc)
        r_b = None
        for _ in range(5):
            Ub, r_b = brute.sweep2d(Ub)
        Oc, it, r_c = oracle_mod.jacobi2d(Uc, 5)
        assert np.array_equal(np.array(Ub, dtype=dtype), Oc) and float(r_b) == r_c


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_2d_constant_and_linear_fixed(oracle_mod, dtype):
    U = oracle_mod.init_field2d((8, 6), dtype, 1, (0.5,) * 4)
    U[...] = dtype(0.5)
    O, _, r = oracle_mod.jacobi2d(U, 9)
    assert r == 0.0 and np.all(O[1:-1, 1:-1] == dtype(0.5))
    j, i = np.meshgrid(np.arange(-1, 7), np.arange(-1, 9), indexing="ij")
    L = (2.0 + 3.0 * i - 1.0 * j).astype(dtype)
    O, _, r = oracle_mod.jacobi2d(L, 4)
    assert r == 0.0 and np.array_equal(O, L)


def test_2d_spectral_eigenfunction_and_decay(oracle_mod):
    nx, ny = 12, 9
    j, i = np.meshgrid(np.arange(-1, ny + 1), np.arange(-1, nx + 1), indexing="ij")
    U = np.sin(np.pi * 2 * (i + 1) / (nx + 1)) * np.sin(np.pi * 3 * (j + 1) / (ny + 1))
    U[:, 0] = U[:, -1] = 0
    U[0, :] = U[-1, :] = 0
    lam = (np.cos(2 * np.pi / (nx + 1)) + np.cos(3 * np.pi / (ny + 1))) / 2
    V, _ = oracle_mod.sweep2d(U)
    assert np.abs(V[1:-1, 1:-1] - lam * U[1:-1, 1:-1]).max() < 1e-15
    # residual decays two steps at a time like cos^2(pi/(N+1)) on a square
    n = 10
    U = oracle_mod.init_field2d(n, np.float64, 4)
    rs = []
    for _ in range(404):
        U, r = oracle_mod.sweep2d(U)
        rs.append(r)
    assert abs(rs[402] / rs[400] - np.cos(np.pi / (n + 1)) ** 2) < 1e-6


def test_2d_superposition_centre_quarter(oracle_mod):
    n = 9
    total, centre = None, []
    for f in range(4):
        bc = [0.0] * 4
        bc[f] = 1.0
        U = oracle_mod.init_field2d(n, np.float64, 2, bc)
        U[1:-1, 1:-1] = 0.0
        O, _, r = oracle_mod.jacobi2d(U, 5000, tol=1e-15, check_every=1)
        I = O[1:-1, 1:-1]
        centre.append(I[n // 2, n // 2])
        total = I if total is None else total + I
    assert np.abs(total - 1.0).max() < 1e-12
    assert all(abs(c - 0.25) < 1e-13 for c in centre)


def test_2d_point_values_match_full_oracle(oracle_mod):
    n2 = (13, 11)
    full, _, _ = oracle_mod.solve2d(n2, np.float64, seed=6, iters=6)
    pts = [(0, 0), (12, 10), (6, 5), (1, 9), (12, 0)]
    got = oracle_mod.point_values2d(n2, pts, 6, np.float64, seed=6)
    assert np.array_equal(got, np.array([full[j + 1, i + 1] for i, j in pts]))
