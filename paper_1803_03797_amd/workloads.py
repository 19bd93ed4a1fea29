"""Seeded synthetic inputs for the workload shapes (inputs only).

This module holds no arithmetic of the method: it draws right-hand sides,
manufactured solutions, grid sizes, tolerances and arrival times.  Both the
GPU path (through its callers) and the CPU oracle take their inputs from
here.  Every array is float64 of shape (ny, nx), C order, so that unknown
(i, j) is element [j, i] (flat index j*nx + i).

Seeds: workload c uses numpy Generator(PCG64(SeedSequence(1803037900 + c)));
per-item streams come from SeedSequence.spawn so item m is reproducible on its
own (a request is the same bits alone and inside a mix).

The paper (Section III) runs synthetic Laplace problems on square grids up to
100x100 without stating the right-hand side; these generators stand in for
them with the shapes and distributions listed below.
"""
import math

import numpy as np

SEED_BASE = 1803037900


def generator(config: int, item: int = None) -> np.random.Generator:
    if item is None:
        ss = np.random.SeedSequence(SEED_BASE + config)
    else:  # the same child SeedSequence.spawn would give as child number `item`
        ss = np.random.SeedSequence(SEED_BASE + config, spawn_key=(item,))
    return np.random.Generator(np.random.PCG64(ss))


def uniform_rhs(nx: int, ny: int, rng: np.random.Generator) -> np.ndarray:
    """b i.i.d. uniform[-1, 1]."""
    return rng.uniform(-1.0, 1.0, size=(ny, nx))


def normal_rhs(nx: int, ny: int, rng: np.random.Generator) -> np.ndarray:
    """b i.i.d. standard normal."""
    return rng.standard_normal(size=(ny, nx))


def sine_mode_plus_noise(nx: int, ny: int, rng: np.random.Generator,
                         noise: float = 1e-3) -> np.ndarray:
    """Manufactured solution x*(i, j) = sin(pi (i+1)/(nx+1)) sin(pi (j+1)/(ny+1))
    + noise * uniform[-1, 1] (the lowest grid mode plus a little noise); the
    right-hand side is then b = A x*, formed by the caller."""
    si = np.sin(np.pi * np.arange(1, nx + 1) / (nx + 1))
    sj = np.sin(np.pi * np.arange(1, ny + 1) / (ny + 1))
    return np.outer(sj, si) + noise * rng.uniform(-1.0, 1.0, size=(ny, nx))


# -- workload 0: 100 x 100, b ~ U[-1,1], tol 1e-8, maxit 2000, both variants --
SMALL = dict(nx=100, ny=100, tol=1e-8, maxit=2000)


def small_problem():
    return uniform_rhs(SMALL["nx"], SMALL["ny"], generator(0))


# -- workload 1: 4096 x 4096, b = A x*, tol 1e-8 and a fixed 500 iterations --
LARGE = dict(nx=4096, ny=4096, tol=1e-8, fixed_iterations=500, maxit=20000)


def large_solution(nx: int = 4096, ny: int = 4096):
    return sine_mode_plus_noise(nx, ny, generator(1))


# -- workload 2: 256 solves, sides uniform over {64..1024} per axis, p-CG --
BATCH_SIDES = (64, 128, 256, 512, 1024)
BATCH = dict(count=256, tol=1e-8, maxit=20000)


def batch_shapes(count: int = 256, sides=BATCH_SIDES):
    rng = generator(2)
    nx = rng.choice(np.asarray(sides), size=count)
    ny = rng.choice(np.asarray(sides), size=count)
    return [(int(a), int(b)) for a, b in zip(nx, ny)]


def batch_rhs(m: int, nx: int, ny: int):
    return uniform_rhs(nx, ny, generator(2, m))


# -- batches of the other operators: 3D grids with sides i.i.d. from
#    {16, 32, 48, 64, 96} per axis (workload 7), or the 2D batch's grids with
#    face conductivities i.i.d. uniform[0.5, 2] (workload 8); b ~ U[-1, 1]
#    per item --
BATCH3_SIDES = (16, 32, 48, 64, 96)


def batch_shapes3(count: int = 256, sides=BATCH3_SIDES):
    rng = generator(7)
    n = rng.choice(np.asarray(sides), size=(count, 3))
    return [(int(a), int(b), int(c)) for a, b, c in n]


def batch_rhs3(m: int, nx: int, ny: int, nz: int):
    """b of item m on an nx x ny x nz grid, as ny*nz rows of nx."""
    return uniform_rhs(nx, ny * nz, generator(7, m))


def batch_faces(m: int, nx: int, ny: int, lo: float = 0.5, hi: float = 2.0):
    """(kx, ky) of item m: (ny, nx + 1) and (ny + 1, nx), i.i.d. uniform[lo, hi]."""
    rng = generator(8, m)
    return rng.uniform(lo, hi, (ny, nx + 1)), rng.uniform(lo, hi, (ny + 1, nx))


# -- workload 3: 8192 x 8192, b ~ N(0,1), refinement to 1e-10, inner 1e-4 --
HUGE = dict(nx=8192, ny=8192, tol=1e-10, inner_tol=1e-4, maxit=200000)


def huge_rhs(nx: int = 8192, ny: int = 8192):
    return normal_rhs(nx, ny, generator(3))


# -- workload 4: request stream, sides log-uniform [32, 2048], tol 1e-6/1e-8 --
SERVE = dict(count=10000, side_lo=32, side_hi=2048, tols=(1e-6, 1e-8), maxit=200000)


def serve_requests(count: int = 10000, lo: int = 32, hi: int = 2048):
    """(nx, ny, tol) per request: sides round(exp(U[ln lo, ln hi])) per axis,
    tol 1e-6 or 1e-8 by a fair coin."""
    rng = generator(4)
    a = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(int)
    b = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(int)
    t = np.where(rng.integers(0, 2, size=count) == 0, SERVE["tols"][0], SERVE["tols"][1])
    return [(int(x), int(y), float(z)) for x, y, z in zip(a, b, t)]


def serve_rhs(m: int, nx: int, ny: int):
    return uniform_rhs(nx, ny, generator(4, m + 1))


# -- fixed point: the paper's synthesized grids and iteration counts (Section
# III tables: N = 16, 32, 40, 100 with 33, 60, 80, 120 iterations, 50-bit
# values with 20 integer bits); b ~ U[-1, 1] keeps (b, b) far below the
# format's 2^19 ceiling.  The measured batch: 256 solves of the largest grid.
FIXED = dict(sides=(16, 32, 40, 100), iterations=(33, 60, 80, 120), batch=256)


def fixed_rhs(n: int, item: int = 0):
    """b ~ U[-1, 1] on the n x n grid; stream (6, n * 1000 + item)."""
    return uniform_rhs(n, n, generator(6, n * 1000 + item))


def poisson_arrivals(count: int, rate: float, seed_item: int = 0):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = generator(5, seed_item)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# -- the 3D 7-point operator: n x n x n, b ~ U[-1,1], tol 1e-8 and a fixed 500
#    iterations (256^3 has the 16.8M unknowns of the 4096^2 workload) --
CUBE = dict(n=256, tol=1e-8, maxit=20000, iterations=500)


def cube_rhs(n: int) -> np.ndarray:
    """b i.i.d. uniform[-1, 1] on an n^3 grid, as n*n rows of n (plane-major)."""
    return uniform_rhs(n, n * n, generator(5))


# -- the variable-coefficient 5-point operator: 4096 x 4096, face
#    conductivities i.i.d. log-uniform over two decades [0.1, 10], b ~ U[-1,1],
#    a fixed 500 iterations, then tol 1e-8 --
VC = dict(n=4096, tol=1e-8, maxit=60000, iterations=500, k_lo=0.1, k_hi=10.0)


def vc_faces(nx: int, ny: int, lo: float = 0.1, hi: float = 10.0):
    """(kx, ky): conductivities of the faces between columns, (ny, nx + 1), and
    between rows, (ny + 1, nx), each i.i.d. exp(U[log lo, log hi])."""
    rng = generator(6)
    kx = np.exp(rng.uniform(math.log(lo), math.log(hi), (ny, nx + 1)))
    ky = np.exp(rng.uniform(math.log(lo), math.log(hi), (ny + 1, nx)))
    return kx, ky


def vc_rhs(nx: int, ny: int) -> np.ndarray:
    """b i.i.d. uniform[-1, 1] for the variable-coefficient workload."""
    return uniform_rhs(nx, ny, generator(6, 1))
