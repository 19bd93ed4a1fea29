"""Pins of the variable-coefficient oracle (oracle_csr_vc_assemble,
oracle_spmv_vc, oracle_cg_vc in cg_oracle.c): the finite-volume operator of
-div(k grad u) with face conductivities kx (ny x (nx+1)) and ky ((ny+1) x nx)
and zero Dirichlet boundary.

Checked against the paper's operator (k = 1), a sum of face contributions
k (e_a - e_b)(e_a - e_b)^T built independently with numpy, the spectrum of a
separable case (eigenvalues of two 1D tridiagonal matrices summed), dense
Cholesky and the agreement of the two CG variants."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL

MODES = (MODE_SEQUENTIAL, MODE_CANONICAL)
GPU_LIKE = oracle.Order(2, 64, 4, 8, 256)
SHAPES = [(1, 1), (1, 6), (5, 1), (7, 5), (12, 9)]


def faces(nx, ny, seed, lo=0.25, hi=4.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (ny, nx + 1)), rng.uniform(lo, hi, (ny + 1, nx))


def dense(nx, ny, kx, ky, order=0):
    rp, col, val = oracle.csr_vc(nx, ny, kx, ky, order)
    return sp.csr_matrix((val, col, rp), shape=(nx * ny, nx * ny)).toarray()


def face_sum(nx, ny, kx, ky):
    """sum over faces: k (e_a - e_b)(e_a - e_b)^T, or k e_a e_a^T on the boundary."""
    n = nx * ny
    A = np.zeros((n, n))

    def add(a, b, k):
        A[a, a] += k
        if b is not None:
            A[b, b] += k
            A[a, b] -= k
            A[b, a] -= k

    for j in range(ny):
        for i in range(nx + 1):
            a = j * nx + i - 1 if i > 0 else None
            b = j * nx + i if i < nx else None
            if a is None:
                add(b, None, kx[j, i])
            else:
                add(a, b, kx[j, i])
    for j in range(ny + 1):
        for i in range(nx):
            a = (j - 1) * nx + i if j > 0 else None
            b = j * nx + i if j < ny else None
            if a is None:
                add(b, None, ky[j, i])
            else:
                add(a, b, ky[j, i])
    return A


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("order", [0, 1])
def test_unit_coefficients_give_the_paper_operator(nx, ny, order):
    kx, ky = np.ones((ny, nx + 1)), np.ones((ny + 1, nx))
    rp, col, val = oracle.csr(nx, ny, order)
    rpv, colv, valv = oracle.csr_vc(nx, ny, kx, ky, order)
    np.testing.assert_array_equal(rp, rpv)
    np.testing.assert_array_equal(col, colv)
    np.testing.assert_array_equal(val, valv)


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_face_sum_symmetry_and_row_sums(nx, ny):
    kx, ky = faces(nx, ny, nx * ny)
    A = dense(nx, ny, kx, ky)
    np.testing.assert_allclose(A, face_sum(nx, ny, kx, ky), rtol=0, atol=1e-14)
    np.testing.assert_array_equal(A, A.T)
    # a row sums to the conductivities of its cell's boundary faces
    want = np.zeros((ny, nx))
    want[:, 0] += kx[:, 0]
    want[:, -1] += kx[:, -1]
    want[0, :] += ky[0, :]
    want[-1, :] += ky[-1, :]
    np.testing.assert_allclose(A.sum(axis=1), want.ravel(), rtol=0, atol=1e-13)
    assert np.linalg.eigvalsh(A)[0] > 0


def test_canonical_entry_order_and_constant_scaling():
    nx, ny = 6, 5
    kx, ky = faces(nx, ny, 3)
    rp, col, val = oracle.csr_vc(nx, ny, kx, ky, 1)
    j, i = 2, 3
    k = j * nx + i
    assert list(col[rp[k]:rp[k + 1]]) == [k, k - 1, k + 1, k - nx, k + nx]
    kw, ke, ks, kn = kx[j, i], kx[j, i + 1], ky[j, i], ky[j + 1, i]
    assert list(val[rp[k]:rp[k + 1]]) == [((kw + ke) + ks) + kn, -kw, -ke, -ks, -kn]
    # every diagonal is ((kW + kE) + kS) + kN in that order (the GPU's contract),
    # summed here one IEEE addition at a time
    for j in range(ny):
        for i in range(nx):
            k = j * nx + i
            d = ((float(kx[j, i]) + float(kx[j, i + 1])) + float(ky[j, i])) + float(ky[j + 1, i])
            assert val[rp[k]] == d, (i, j)
    # a constant k = 0.375 (exact in binary) scales the paper's operator exactly
    c = 0.375
    A = dense(nx, ny, np.full((ny, nx + 1), c), np.full((ny + 1, nx), c))
    rp, col, val = oracle.csr(nx, ny, 0)
    A0 = sp.csr_matrix((val, col, rp), shape=(nx * ny, nx * ny)).toarray()
    np.testing.assert_array_equal(A, c * A0)


def test_separable_spectrum():
    """kx depending on i only and ky on j only: A = I (x) T_x + T_y (x) I with
    1D tridiagonal T's, so its eigenvalues are all sums of theirs."""
    nx, ny = 9, 7
    rng = np.random.default_rng(11)
    gx, gy = rng.uniform(0.5, 3, nx + 1), rng.uniform(0.5, 3, ny + 1)
    kx, ky = np.tile(gx, (ny, 1)), np.tile(gy[:, None], (1, nx))

    def T(g):
        m = len(g) - 1
        return np.diag(g[:-1] + g[1:]) - np.diag(g[1:-1], 1) - np.diag(g[1:-1], -1)

    ex, ey = np.linalg.eigvalsh(T(gx)), np.linalg.eigvalsh(T(gy))
    want = np.sort((ex[None, :] + ey[:, None]).ravel())
    np.testing.assert_allclose(np.linalg.eigvalsh(dense(nx, ny, kx, ky)), want, atol=1e-12)


@pytest.mark.parametrize("nx,ny", [(12, 9), (64, 3)])
def test_spmv_matches_the_matrix(nx, ny):
    kx, ky = faces(nx, ny, 7)
    u = np.random.default_rng(2).uniform(-1, 1, (ny, nx))
    A = dense(nx, ny, kx, ky)
    for order in (0, 1):
        np.testing.assert_allclose(oracle.spmv_vc(u, nx, ny, kx, ky, order).ravel(), A @ u.ravel(),
                                   rtol=0, atol=1e-13)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("mode", MODES)
def test_solve_vs_dense_cholesky(variant, mode):
    nx, ny = 14, 11
    kx, ky = faces(nx, ny, 5)
    A = dense(nx, ny, kx, ky)
    b = np.random.default_rng(8).uniform(-1, 1, (ny, nx))
    xs = sla.cho_solve(sla.cho_factor(A), b.ravel()).reshape(ny, nx)
    o = GPU_LIKE if mode == MODE_CANONICAL else None
    x, r = oracle.cg_vc(b, nx, ny, kx, ky, variant=variant, tol=1e-12, maxit=2000, mode=mode,
                        order=o)
    ev = np.linalg.eigvalsh(A)
    assert r.status == 0 and r.rel_res_recursive <= 1e-12
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 2 * 1e-12 * ev[-1] / ev[0]


@pytest.mark.parametrize("nx,ny", [(7, 5), (16, 16), (1, 13)])
def test_variant_agreement(nx, ny):
    kx, ky = faces(nx, ny, nx + ny)
    b = np.random.default_rng(nx).uniform(-1, 1, (ny, nx))
    for k in range(1, min(21, nx * ny + 1)):
        xc, rc = oracle.cg_vc(b, nx, ny, kx, ky, variant=0, tol=0.0, maxit=k)
        xp, rp = oracle.cg_vc(b, nx, ny, kx, ky, variant=1, tol=0.0, maxit=k)
        assert rc.iterations == rp.iterations == k
        assert np.linalg.norm(xp - xc) <= 1e-12 * np.linalg.norm(xc), k


def test_edge_cases_and_rejections():
    nx, ny = 6, 4
    kx, ky = faces(nx, ny, 1)
    b = np.random.default_rng(1).uniform(-1, 1, (ny, nx))
    for v in (0, 1):
        x, r = oracle.cg_vc(np.zeros_like(b), nx, ny, kx, ky, variant=v, x0=np.ones_like(b))
        assert r.status == 0 and r.iterations == 0 and not x.any()
        x, r = oracle.cg_vc(b, nx, ny, kx, ky, variant=v, tol=1e-15, maxit=3)
        assert r.status == 2 and r.iterations == 3
    with pytest.raises(ValueError):
        oracle.cg_vc(b, nx, ny, kx[:, :-1], ky)
