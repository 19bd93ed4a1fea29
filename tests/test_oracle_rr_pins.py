"""Pins of residual replacement in the oracle's pipelined CG (oracle_cg_rr,
oracle_cg_vc_rr in cg_oracle.c): every rr_period iterations q = A p, z = A q,
r = b - A x and w = A r are recomputed from their definitions.

Replacement changes nothing in exact arithmetic, so the iterates still agree
with classic CG on small grids, and with a period longer than the solve the
run is bitwise the plain one; what it buys is attainable accuracy, shown on a
variable-coefficient grid where plain pipelined CG breaks down before tol and
the replaced run reaches a true residual of tol with classic CG's iteration
count.  Copies of the oracle built with a planted mistake in the replacement
(w or z not recomputed) fail that pin."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL, VARIANT_CLASSIC, VARIANT_PIPELINED
from paper_1803_03797_amd import workloads

GPU_LIKE = oracle.Order(2, 64, 4, 8, 256)


def dense_A(nx, ny):
    rp, col, val = oracle.csr(nx, ny)
    return sp.csr_matrix((val, col, rp), shape=(nx * ny, nx * ny)).toarray()


@pytest.mark.parametrize("mode", [MODE_SEQUENTIAL, MODE_CANONICAL])
def test_period_past_the_solve_is_the_plain_run(mode):
    nx, ny = 40, 30
    b = np.random.default_rng(1).uniform(-1, 1, (ny, nx))
    kw = dict(variant=VARIANT_PIPELINED, tol=1e-9, maxit=400, mode=mode,
              order=GPU_LIKE if mode == MODE_CANONICAL else None)
    x0, r0 = oracle.cg(b, nx, ny, **kw)
    x1, r1 = oracle.cg(b, nx, ny, rr_period=r0.iterations + 1, **kw)
    assert r0.iterations == r1.iterations
    np.testing.assert_array_equal(x0, x1)


@pytest.mark.parametrize("nx,ny", [(6, 5), (16, 16), (9, 14)])
@pytest.mark.parametrize("period", [2, 4, 10])
def test_iterates_agree_with_classic_cg(nx, ny, period):
    """Replacement is exact in exact arithmetic: after each m iterations the
    replaced pipelined iterate equals classic CG's to rounding."""
    b = np.random.default_rng(nx * ny + period).uniform(-1, 1, (ny, nx))
    for m in (3, 7, 12, 20):
        xc, rc = oracle.cg(b, nx, ny, variant=VARIANT_CLASSIC, tol=0.0, maxit=m)
        xp, rp = oracle.cg(b, nx, ny, variant=VARIANT_PIPELINED, tol=0.0, maxit=m,
                           rr_period=period)
        assert np.linalg.norm(xp - xc) <= 1e-12 * np.linalg.norm(xc)


@pytest.mark.parametrize("nx,ny", [(12, 12), (16, 9)])
def test_solution_vs_dense_cholesky(nx, ny):
    b = np.random.default_rng(3).uniform(-1, 1, (ny, nx))
    A = dense_A(nx, ny)
    xs = sla.cho_solve(sla.cho_factor(A), b.ravel())
    w = np.linalg.eigvalsh(A)
    tol = 1e-12
    x, r = oracle.cg(b, nx, ny, variant=VARIANT_PIPELINED, tol=tol, maxit=1000, rr_period=6)
    assert r.status == oracle.OR_OK
    assert np.linalg.norm(x.ravel() - xs) / np.linalg.norm(xs) <= 2 * tol * w[-1] / w[0]


def vc_case(n=256):
    kx, ky = workloads.vc_faces(n, n)
    return kx, ky, workloads.vc_rhs(n, n)


def test_attainable_accuracy_restored():
    """256 x 256, conductivities over two decades, tol 1e-12: plain pipelined
    CG breaks down (its recursive residual has drifted from the true one);
    with replacement every 50 iterations the true residual reaches tol within
    2% of classic CG's iteration count."""
    n, tol = 256, 1e-12
    kx, ky, b = vc_case(n)
    xc, rc = oracle.cg_vc(b, n, n, kx, ky, variant=VARIANT_CLASSIC, tol=tol, maxit=60000)
    xp, rp = oracle.cg_vc(b, n, n, kx, ky, variant=VARIANT_PIPELINED, tol=tol, maxit=60000)
    xr, rr = oracle.cg_vc(b, n, n, kx, ky, variant=VARIANT_PIPELINED, tol=tol, maxit=60000,
                          rr_period=50)
    assert rc.status == oracle.OR_OK and rc.rel_res_true <= 1.5 * tol
    assert rp.status != oracle.OR_OK or rp.rel_res_true > 100 * tol
    assert rr.status == oracle.OR_OK and rr.rel_res_true <= 1.5 * tol
    assert abs(rr.iterations - rc.iterations) <= 0.02 * rc.iterations
    # the true residual recomputed independently (scipy CSR of the faces)
    rp_, col, val = oracle.csr_vc(n, n, kx, ky)
    A = sp.csr_matrix((val, col, rp_), shape=(n * n, n * n))
    assert np.linalg.norm(b.ravel() - A @ xr.ravel()) / np.linalg.norm(b) <= 1.5 * tol
    assert np.linalg.norm(xr - xc) <= 1e-9 * np.linalg.norm(xc)


def test_five_point_true_residual_tracks_the_recursive_one():
    """The 5-point operator at 256^2 and tol 1e-10: with replacement the true
    residual at the stop is within 20% of the recursive one."""
    n = 256
    b = np.random.default_rng(7).uniform(-1, 1, (n, n))
    x, r = oracle.cg(b, n, n, variant=VARIANT_PIPELINED, tol=1e-10, maxit=20000, rr_period=100)
    assert r.status == oracle.OR_OK and r.rel_res_true <= 1.2 * r.rel_res_recursive


@pytest.mark.parametrize("mutant", [4, 5])
def test_pins_catch_planted_mistakes(tmp_path, mutant):
    """Copies built with w = A r (4) or z = A q (5) left out of the
    replacement do not restore the accuracy: they fail the pin above."""
    from oracle import oracle as om
    src = os.path.join(os.path.dirname(oracle.lib_path()), "cg_oracle.c")
    lib_path = str(tmp_path / ("mutant%d.so" % mutant))
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-Wno-unknown-pragmas", "-DORACLE_MUTANT=%d" % mutant, "-o",
                    lib_path, src, "-lm"], check=True)
    lib = C.CDLL(lib_path)
    P = C.c_void_p
    f = lib.oracle_cg_vc_rr
    f.restype = C.c_int
    f.argtypes = [C.c_int32, C.c_int32, P, C.c_int32, C.c_int32, P, P, P, P, P, C.c_double,
                  C.c_int32, C.c_int32, C.POINTER(om._Result)]
    n, tol = 256, 1e-12
    kx, ky, b = (np.ascontiguousarray(a) for a in vc_case(n))
    x = np.zeros_like(b)
    res = om._Result()
    assert f(VARIANT_PIPELINED, MODE_SEQUENTIAL, None, n, n, kx.ctypes.data, ky.ctypes.data,
             b.ctypes.data, None, x.ctypes.data, tol, 60000, 50, C.byref(res)) >= 0
    assert not (res.status == oracle.OR_OK and res.rel_res_true <= 1.5 * tol)
