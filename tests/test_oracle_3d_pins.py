"""Pins of the 3D oracle (oracle_csr3_*, oracle_spmv3, oracle_cg3 in
cg_oracle.c): the unscaled 7-point Laplacian on an nx x ny x nz grid with zero
Dirichlet boundary, unknown (i, j, l) at (l ny + j) nx + i.

Checked against closed forms (eigenvalues 6 - 2cos(a pi/(nx+1))
- 2cos(b pi/(ny+1)) - 2cos(c pi/(nz+1)) and their sine eigenvectors), the
Kronecker-sum form of the operator built with scipy, dense Cholesky, finite
termination and the agreement of the two CG variants."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL

MODES = (MODE_SEQUENTIAL, MODE_CANONICAL)
GPU_LIKE = oracle.Order(2, 64, 4, 8, 256)
SMALL = [(1, 1, 1), (1, 1, 5), (3, 4, 5), (2, 3, 1), (5, 5, 5), (6, 1, 4)]


def dense_A3(nx, ny, nz, order=0):
    rp, col, val = oracle.csr3(nx, ny, nz, order)
    n = nx * ny * nz
    return sp.csr_matrix((val, col, rp), shape=(n, n))


def kron_A3(nx, ny, nz):
    """The operator as I (x) I (x) T_x + I (x) T_y (x) I + T_z (x) I (x) I with
    T_m = tridiag(-1, 2, -1) of size m (unknowns ordered with x fastest)."""
    def T(m):
        return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(Iz, sp.kron(Iy, T(nx))) + sp.kron(Iz, sp.kron(T(ny), Ix)) +
            sp.kron(T(nz), sp.kron(Iy, Ix)))


def lam3(nx, ny, nz, a, b, c):
    """4 sin^2 form of 2 - 2cos: no cancellation for the lowest modes."""
    return (4 * math.sin(a * math.pi / (2 * (nx + 1))) ** 2 +
            4 * math.sin(b * math.pi / (2 * (ny + 1))) ** 2 +
            4 * math.sin(c * math.pi / (2 * (nz + 1))) ** 2)


def mode3(nx, ny, nz, a, b, c):
    i = np.arange(1, nx + 1)[None, None, :]
    j = np.arange(1, ny + 1)[None, :, None]
    l = np.arange(1, nz + 1)[:, None, None]
    v = (np.sin(a * np.pi * i / (nx + 1)) * np.sin(b * np.pi * j / (ny + 1)) *
         np.sin(c * np.pi * l / (nz + 1)))
    return v.reshape(ny * nz, nx)


@pytest.mark.parametrize("nx,ny,nz", SMALL)
def test_eigenvalues_closed_form(nx, ny, nz):
    ev = np.linalg.eigvalsh(dense_A3(nx, ny, nz).toarray())
    want = sorted(lam3(nx, ny, nz, a, b, c) for a in range(1, nx + 1)
                  for b in range(1, ny + 1) for c in range(1, nz + 1))
    np.testing.assert_allclose(ev, want, atol=1e-13)


@pytest.mark.parametrize("nx,ny,nz", SMALL)
@pytest.mark.parametrize("order", [0, 1])
def test_kronecker_sum_and_structure(nx, ny, nz, order):
    A = dense_A3(nx, ny, nz, order)
    K = kron_A3(nx, ny, nz)
    assert (A != A.T).nnz == 0
    assert abs(A - K).max() == 0
    # row sums = the number of that unknown's faces on the Dirichlet boundary
    k = np.arange(nx * ny * nz)
    i, j, l = k % nx, (k // nx) % ny, k // (nx * ny)
    faces = ((i == 0).astype(int) + (i == nx - 1) + (j == 0) + (j == ny - 1) + (l == 0) +
             (l == nz - 1))
    np.testing.assert_array_equal(np.asarray(A.sum(axis=1)).ravel(), faces)


def test_canonical_entry_order():
    """Canonical rows list centre, west, east, south, north, below, above."""
    nx, ny, nz = 4, 3, 3
    rp, col, val = oracle.csr3(nx, ny, nz, 1)
    k = (1 * ny + 1) * nx + 1  # the interior unknown (1, 1, 1)
    got = list(col[rp[k]:rp[k + 1]])
    assert got == [k, k - 1, k + 1, k - nx, k + nx, k - nx * ny, k + nx * ny]
    assert list(val[rp[k]:rp[k + 1]]) == [6, -1, -1, -1, -1, -1, -1]


@pytest.mark.parametrize("nx,ny,nz", [(20, 17, 9), (64, 1, 3)])
def test_eigenvector_identity_and_spmv(nx, ny, nz):
    for a, b, c in ((1, 1, 1), (3, 1, 2), (nx, ny, nz)):
        phi = mode3(nx, ny, nz, a, b, c)
        for order in (0, 1):
            y = oracle.spmv3(phi, nx, ny, nz, order)
            np.testing.assert_allclose(y, lam3(nx, ny, nz, a, b, c) * phi, atol=1e-13)
    u = np.random.default_rng(2).uniform(-1, 1, (ny * nz, nx))
    np.testing.assert_allclose(oracle.spmv3(u, nx, ny, nz),
                               (kron_A3(nx, ny, nz) @ u.ravel()).reshape(u.shape), atol=1e-14)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("mode", MODES)
def test_solve_vs_dense_cholesky(variant, mode):
    nx, ny, nz = 6, 5, 4
    A = dense_A3(nx, ny, nz).toarray()
    b = np.random.default_rng(5).uniform(-1, 1, (ny * nz, nx))
    xs = sla.cho_solve(sla.cho_factor(A), b.ravel()).reshape(b.shape)
    o = GPU_LIKE if mode == MODE_CANONICAL else None
    x, r = oracle.cg3(b, nx, ny, nz, variant=variant, tol=1e-12, maxit=500, mode=mode, order=o)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    assert r.status == 0 and r.rel_res_recursive <= 1e-12
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 2 * 1e-12 * kappa


@pytest.mark.parametrize("variant", [0, 1])
def test_single_mode_and_finite_termination(variant):
    nx, ny, nz = 9, 7, 5
    phi = mode3(nx, ny, nz, 2, 3, 1)
    lam = lam3(nx, ny, nz, 2, 3, 1)
    x, r = oracle.cg3(phi, nx, ny, nz, variant=variant, tol=1e-12, maxit=50)
    assert r.status == 0 and r.iterations == 1
    np.testing.assert_allclose(x, phi / lam, rtol=0, atol=1e-14)
    # four modes with distinct eigenvalues: four iterations (or five)
    modes = [(1, 1, 1), (2, 1, 3), (4, 5, 2), (9, 7, 5)]
    b = sum(mode3(nx, ny, nz, *m) * (k + 1) for k, m in enumerate(modes))
    xw = sum(mode3(nx, ny, nz, *m) * (k + 1) / lam3(nx, ny, nz, *m)
             for k, m in enumerate(modes))
    x, r = oracle.cg3(b, nx, ny, nz, variant=variant, tol=1e-12, maxit=50)
    assert r.status == 0 and r.iterations in (4, 5)
    assert np.linalg.norm(x - xw) <= 1e-11 * np.linalg.norm(xw)


@pytest.mark.parametrize("nx,ny,nz", [(6, 5, 4), (16, 16, 16), (1, 9, 13)])
def test_variant_agreement(nx, ny, nz):
    """Algorithms 1 and 2 give the same iterates in exact arithmetic."""
    b = np.random.default_rng(nx + ny + nz).uniform(-1, 1, (ny * nz, nx))
    for k in range(1, 21):
        xc, rc = oracle.cg3(b, nx, ny, nz, variant=0, tol=0.0, maxit=k)
        xp, rp = oracle.cg3(b, nx, ny, nz, variant=1, tol=0.0, maxit=k)
        assert rc.iterations == rp.iterations == k
        assert np.linalg.norm(xp - xc) <= 1e-12 * np.linalg.norm(xc), k


def test_nz_one_is_the_2d_operator_plus_2():
    nx, ny = 7, 6
    A3 = dense_A3(nx, ny, 1).toarray()
    rp, col, val = oracle.csr(nx, ny, 0)
    A2 = sp.csr_matrix((val, col, rp), shape=(nx * ny, nx * ny)).toarray()
    np.testing.assert_array_equal(A3, A2 + 2 * np.eye(nx * ny))


def test_edge_cases_and_rejections():
    nx, ny, nz = 5, 4, 3
    b = np.random.default_rng(1).uniform(-1, 1, (ny * nz, nx))
    for v in (0, 1):
        x, r = oracle.cg3(np.zeros_like(b), nx, ny, nz, variant=v, x0=np.ones_like(b))
        assert r.status == 0 and r.iterations == 0 and not x.any()
        x, r = oracle.cg3(b, nx, ny, nz, variant=v, tol=1e-14, maxit=3)
        assert r.status == 2 and r.iterations == 3
    for bad in ((0, 1, 1), (1, 0, 1), (1, 1, 0)):
        with pytest.raises(ValueError):
            oracle.cg3(np.zeros(0), *bad)


# --------------------------------------------------- z-march tile order --

ZMARCH = [oracle.Order.zmarch(2, 64, 4, 8, 256, 0), oracle.Order.zmarch(1, 4, 3, 2, 8, 0),
          oracle.Order.zmarch(2, 64, 4, 64, 256, 0)]


@pytest.mark.parametrize("nx,ny,nz", [(1, 1, 2), (7, 5, 3), (130, 7, 5), (37, 40, 23),
                                      (257, 30, 9)])
@pytest.mark.parametrize("k", range(len(ZMARCH)))
def test_zmarch_order_exact_on_integers(nx, ny, nz, k):
    """Integer data and position weights: every term of the 3D grid is counted
    exactly once by the z-march order (a dropped, repeated or misplaced row,
    plane or column would change the exact sum)."""
    base = ZMARCH[k]
    o = oracle.Order.zmarch(base.cols_per_lane, base.lanes, base.waves, base.rows,
                            base.threads2, ny)
    rows = ny * nz
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    a = rng.integers(-8, 9, size=(rows, nx)).astype(float)
    b = rng.integers(-8, 9, size=(rows, nx)).astype(float)
    exact = float(np.sum(a.astype(np.int64) * b.astype(np.int64)))
    assert oracle.dot(a, b, nx, rows, MODE_CANONICAL, o) == exact
    w = np.arange(1, nx * rows + 1, dtype=float).reshape(rows, nx)
    assert oracle.dot(w, np.ones((rows, nx)), nx, rows, MODE_CANONICAL, o) == \
        (nx * rows) * (nx * rows + 1) / 2


def test_zmarch_order_sums_each_row_over_the_planes():
    """One column, a 2 x 3 (y, z) grid, one tile of two wavefronts (y = 0, 1)
    over all three planes.  The wavefront of y sums its values in ascending z:
    y = 0 holding 1, 1e16, -1e16 at z = 0, 1, 2 gives (1 + 1e16) - 1e16 = 0
    (descending z would give 1).  The tile adds the wavefronts: 1e16 + 1 at
    y = 0 against -1e16 at y = 1 gives 1e16 - 1e16 = 0, where the stacked-row
    order (rows z * 2 + y in sequence) cancels 1e16 first and keeps the 1."""
    o = oracle.Order.zmarch(1, 1, 2, 3, 1, 2)
    one = np.ones((6, 1))
    def grid(v):  # v[y][z] -> rows z * 2 + y
        return np.array([v[y][z] for z in range(3) for y in range(2)]).reshape(6, 1)
    assert oracle.dot(grid([[1.0, 1e16, -1e16], [0.0, 0.0, 0.0]]), one, 1, 6,
                      MODE_CANONICAL, o) == 0.0
    assert oracle.dot(grid([[-1e16, 1e16, 1.0], [0.0, 0.0, 0.0]]), one, 1, 6,
                      MODE_CANONICAL, o) == 1.0
    cross = grid([[1e16, 1.0, 0.0], [-1e16, 0.0, 0.0]])
    assert oracle.dot(cross, one, 1, 6, MODE_CANONICAL, o) == 0.0
    assert oracle.dot(cross, one, 1, 6, MODE_CANONICAL, oracle.Order(1, 1, 2, 3, 1)) == 1.0


def test_zmarch_solves_agree_with_the_tile_order():
    """CG in the z-march order: the same iterations as in the stacked-row tile
    order and solutions equal to rounding (two valid summation orders)."""
    nx, ny, nz = 37, 40, 23
    b = np.random.default_rng(5).uniform(-1, 1, (ny * nz, nx))
    for v in (0, 1):
        x1, r1 = oracle.cg3(b, nx, ny, nz, variant=v, tol=1e-10, mode=MODE_CANONICAL,
                            order=GPU_LIKE)
        x2, r2 = oracle.cg3(b, nx, ny, nz, variant=v, tol=1e-10, mode=MODE_CANONICAL,
                            order=oracle.Order.zmarch(2, 64, 4, 8, 256, ny))
        assert abs(r1.iterations - r2.iterations) <= 1
        assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x1)
        with pytest.raises(ValueError):
            oracle.cg3(b, nx, ny, nz, variant=v, mode=MODE_CANONICAL,
                       order=oracle.Order.zmarch(2, 64, 4, 8, 256, 41))
