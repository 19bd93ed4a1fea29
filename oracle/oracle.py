"""ctypes front end of cg_oracle.c (test infrastructure; see the C file header).

Vectors are dense float64 arrays of shape (ny, nx), C order, so that unknown
(i, j) sits at [j, i], i.e. flat index k = j*nx + i.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

MODE_SEQUENTIAL, MODE_CANONICAL = 0, 1
VARIANT_CLASSIC, VARIANT_PIPELINED = 0, 1
OR_OK, OR_NOT_CONVERGED, OR_BREAKDOWN, OR_E_INVALID, OR_E_NOMEM = 0, 2, 3, -1, -2


class Order(C.Structure):
    """Reduction order of the canonical mode: layout 0 = tiles (dot_canonical in
    the C file), layout 1 = column segments (dot_segments), layout 2 = the 3D
    z-march tiles (dot_zmarch: `waves` in-plane rows by `rows` planes, plane =
    rows per plane)."""
    _fields_ = [("cols_per_lane", C.c_int32), ("lanes", C.c_int32), ("waves", C.c_int32),
                ("rows", C.c_int32), ("threads2", C.c_int32), ("layout", C.c_int32),
                ("seg_cols", C.c_int32), ("alt", C.c_int32), ("plane", C.c_int32)]

    @classmethod
    def segments(cls, rows, lanes, waves, seg_cols):
        """Column-segment order: waves*lanes threads, `rows` rows per thread,
        seg_cols threads per row of segments (those of columns >= nx idle)."""
        return cls(1, lanes, waves, rows, 0, 1, seg_cols)

    @classmethod
    def zmarch(cls, cols_per_lane, lanes, waves, planes, threads2, plane):
        """3D z-march order: tiles of `waves` in-plane rows by `planes` planes,
        each wavefront summing its row over the planes in ascending z."""
        return cls(cols_per_lane, lanes, waves, planes, threads2, 2, 0, 0, plane)


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32),
                ("outer_iterations", C.c_int32), ("pad_", C.c_int32),
                ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double)]


class _History(C.Structure):
    _fields_ = [("max_hist", C.c_int32), ("count", C.c_int32),
                ("gamma", C.c_void_p), ("r", C.c_void_p), ("p", C.c_void_p), ("x", C.c_void_p)]


_lib = None


def lib_path():
    return _build.LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _build.stale():
        _build.build()
    lib = C.CDLL(_build.LIB)
    P = C.c_void_p
    lib.oracle_csr_nnz.restype = C.c_int64
    lib.oracle_csr_nnz.argtypes = [C.c_int32, C.c_int32]
    lib.oracle_csr_assemble.restype = C.c_int64
    lib.oracle_csr_assemble.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P]
    lib.oracle_spmv.restype = C.c_int
    lib.oracle_spmv.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P]
    lib.oracle_dot.restype = C.c_double
    lib.oracle_dot.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(Order), P, P]
    lib.oracle_cg.restype = C.c_int
    lib.oracle_cg.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.c_int32, C.c_int32,
                              P, P, P, C.c_double, C.c_int32, C.POINTER(_Result),
                              C.POINTER(_History)]
    lib.oracle_cheb_coeffs.restype = C.c_int
    lib.oracle_cheb_coeffs.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P]
    lib.oracle_cheb_apply.restype = C.c_int
    lib.oracle_cheb_apply.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P]
    lib.oracle_pcg.restype = C.c_int
    lib.oracle_pcg.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.POINTER(Order),
                               C.c_int32, C.c_int32, C.c_int32, P, P, P, C.c_double, C.c_int32,
                               C.POINTER(_Result)]
    I64 = C.c_int64
    lib.oracle_fx_quantize.restype = I64
    lib.oracle_fx_quantize.argtypes = [C.c_double]
    lib.oracle_fx_value.restype = C.c_double
    lib.oracle_fx_value.argtypes = [I64]
    lib.oracle_fx_mul.restype = I64
    lib.oracle_fx_mul.argtypes = [I64, I64]
    for f in (lib.oracle_fx_axpy, lib.oracle_fx_axmy):
        f.restype = I64
        f.argtypes = [I64, I64, I64]
    lib.oracle_fx_div.restype = I64
    lib.oracle_fx_div.argtypes = [I64, I64]
    lib.oracle_fx_dot.restype = I64
    lib.oracle_fx_dot.argtypes = [I64, P, P]
    lib.oracle_fx_spmv.restype = C.c_int
    lib.oracle_fx_spmv.argtypes = [C.c_int32, C.c_int32, P, P]
    lib.oracle_cg_fixed.restype = C.c_int
    lib.oracle_cg_fixed.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, C.c_double,
                                    C.c_int32, C.POINTER(_Result)]
    lib.oracle_last_solve_seconds.restype = C.c_double
    lib.oracle_threads.restype = C.c_int
    lib.oracle_refine.restype = C.c_int
    lib.oracle_refine.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_double, C.c_double,
                                  C.c_int32, C.POINTER(_Result)]
    lib.oracle_cheb_apply_f32.restype = C.c_int
    lib.oracle_cheb_apply_f32.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P]
    lib.oracle_refine_pc.restype = C.c_int
    lib.oracle_refine_pc.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_double, C.c_double,
                                     C.c_int32, C.c_int32, C.POINTER(_Result)]
    lib.oracle_csr3_nnz.restype = C.c_int64
    lib.oracle_csr3_nnz.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    lib.oracle_csr3_assemble.restype = C.c_int64
    lib.oracle_csr3_assemble.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P]
    lib.oracle_spmv3.restype = C.c_int
    lib.oracle_spmv3.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P]
    lib.oracle_cg3.restype = C.c_int
    lib.oracle_cg3.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.c_int32, C.c_int32,
                               C.c_int32, P, P, P, C.c_double, C.c_int32, C.POINTER(_Result)]
    lib.oracle_csr_vc_assemble.restype = C.c_int64
    lib.oracle_csr_vc_assemble.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int32, P, P, P]
    lib.oracle_spmv_vc.restype = C.c_int
    lib.oracle_spmv_vc.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int32, P, P]
    lib.oracle_cg_rr.restype = C.c_int
    lib.oracle_cg_rr.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.c_int32, C.c_int32,
                                 P, P, P, C.c_double, C.c_int32, C.c_int32, C.POINTER(_Result)]
    lib.oracle_cg_vc_rr.restype = C.c_int
    lib.oracle_cg_vc_rr.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.c_int32,
                                    C.c_int32, P, P, P, P, P, C.c_double, C.c_int32, C.c_int32,
                                    C.POINTER(_Result)]
    lib.oracle_cg_vc.restype = C.c_int
    lib.oracle_cg_vc.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.c_int32, C.c_int32,
                                 P, P, P, P, P, C.c_double, C.c_int32, C.POINTER(_Result)]
    _lib = lib
    return lib


def _vec(a, nx, ny):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != nx * ny:
        raise ValueError("vector has %d entries, grid %dx%d needs %d" % (a.size, nx, ny, nx * ny))
    return a.reshape(ny, nx)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def csr(nx, ny, order=0):
    """The matrix A as (row_ptr int64, col int32, val float64)."""
    lib = _load()
    nnz = lib.oracle_csr_nnz(nx, ny)
    if nnz < 0:
        raise ValueError("bad grid")
    rp = np.zeros(nx * ny + 1, np.int64)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    got = lib.oracle_csr_assemble(nx, ny, order, _ptr(rp), _ptr(col), _ptr(val))
    assert got == nnz
    return rp, col, val


def csr3(nx, ny, nz, order=0):
    """The 7-point matrix of an nx x ny x nz grid as (row_ptr, col, val)."""
    lib = _load()
    nnz = lib.oracle_csr3_nnz(nx, ny, nz)
    if nnz < 0:
        raise ValueError("bad grid")
    rp = np.zeros(nx * ny * nz + 1, np.int64)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    got = lib.oracle_csr3_assemble(nx, ny, nz, order, _ptr(rp), _ptr(col), _ptr(val))
    assert got == nnz
    return rp, col, val


def spmv3(u, nx, ny, nz, order=0):
    """A u for the 7-point operator; u has nz*ny rows of nx (any shape of that size)."""
    u = _vec(u, nx, ny * nz)
    y = np.zeros_like(u)
    rc = _load().oracle_spmv3(nx, ny, nz, order, _ptr(u), _ptr(y))
    if rc:
        raise RuntimeError("oracle_spmv3 failed: %d" % rc)
    return y


def cg3(b, nx, ny, nz, variant=VARIANT_CLASSIC, tol=1e-8, maxit=2000, x0=None,
        mode=MODE_SEQUENTIAL, order=None):
    """Solve the 7-point system on an nx x ny x nz grid (vectors as ny*nz rows of
    nx; canonical orders see those rows)."""
    b = _vec(b, nx, ny * nz)
    x0a = _vec(x0, nx, ny * nz) if x0 is not None else None
    x = np.zeros_like(b)
    res = _Result()
    o = C.byref(order) if order is not None else None
    rc = _load().oracle_cg3(variant, mode, o, nx, ny, nz, _ptr(b), _ptr(x0a), _ptr(x), tol,
                            maxit, C.byref(res))
    if rc < 0:
        raise ValueError("oracle_cg3 rejected the call: %d" % rc)
    return x, Result(status=res.status, iterations=res.iterations,
                     outer_iterations=res.outer_iterations,
                     rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)


def _faces(kx, ky, nx, ny):
    kx = np.ascontiguousarray(kx, dtype=np.float64)
    ky = np.ascontiguousarray(ky, dtype=np.float64)
    if kx.size != ny * (nx + 1) or ky.size != (ny + 1) * nx:
        raise ValueError("kx needs %d x %d faces, ky %d x %d" % (ny, nx + 1, ny + 1, nx))
    return kx, ky


def csr_vc(nx, ny, kx, ky, order=0):
    """The variable-coefficient matrix as (row_ptr, col, val)."""
    kx, ky = _faces(kx, ky, nx, ny)
    nnz = _load().oracle_csr_nnz(nx, ny)
    rp = np.zeros(nx * ny + 1, np.int64)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    got = _load().oracle_csr_vc_assemble(nx, ny, _ptr(kx), _ptr(ky), order, _ptr(rp), _ptr(col),
                                         _ptr(val))
    assert got == nnz
    return rp, col, val


def spmv_vc(u, nx, ny, kx, ky, order=0):
    kx, ky = _faces(kx, ky, nx, ny)
    u = _vec(u, nx, ny)
    y = np.zeros_like(u)
    rc = _load().oracle_spmv_vc(nx, ny, _ptr(kx), _ptr(ky), order, _ptr(u), _ptr(y))
    if rc:
        raise RuntimeError("oracle_spmv_vc failed: %d" % rc)
    return y


def cg_vc(b, nx, ny, kx, ky, variant=VARIANT_CLASSIC, tol=1e-8, maxit=2000, x0=None,
          mode=MODE_SEQUENTIAL, order=None, rr_period=0):
    """Solve the variable-coefficient 5-point system (face conductivities kx of
    shape (ny, nx + 1) and ky of shape (ny + 1, nx)); rr_period as in cg()."""
    kx, ky = _faces(kx, ky, nx, ny)
    b = _vec(b, nx, ny)
    x0a = _vec(x0, nx, ny) if x0 is not None else None
    x = np.zeros_like(b)
    res = _Result()
    o = C.byref(order) if order is not None else None
    rc = _load().oracle_cg_vc_rr(variant, mode, o, nx, ny, _ptr(kx), _ptr(ky), _ptr(b),
                                 _ptr(x0a), _ptr(x), tol, maxit, rr_period, C.byref(res))
    if rc < 0:
        raise ValueError("oracle_cg_vc rejected the call: %d" % rc)
    return x, Result(status=res.status, iterations=res.iterations,
                     outer_iterations=res.outer_iterations,
                     rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)


def spmv(u, nx, ny, order=0):
    u = _vec(u, nx, ny)
    y = np.zeros_like(u)
    rc = _load().oracle_spmv(nx, ny, order, _ptr(u), _ptr(y))
    if rc:
        raise RuntimeError("oracle_spmv failed: %d" % rc)
    return y


def dot(a, b, nx, ny, mode=MODE_SEQUENTIAL, order=None):
    a, b = _vec(a, nx, ny), _vec(b, nx, ny)
    o = C.byref(order) if order is not None else None
    if mode == MODE_CANONICAL and order is None:
        raise ValueError("canonical mode needs an Order")
    return _load().oracle_dot(nx, ny, mode, o, _ptr(a), _ptr(b))


class Result(dict):
    __getattr__ = dict.__getitem__


def cg(b, nx, ny, variant=VARIANT_CLASSIC, tol=1e-8, maxit=2000, x0=None,
       mode=MODE_SEQUENTIAL, order=None, history=0, rr_period=0, all_cores=False):
    """Solve A x = b.  Returns (x, Result); with history=m also returns a dict of
    the first m records (gamma, r, p, x after 0, 1, ... updates).  rr_period
    > 0: the pipelined variant replaces its residuals every rr_period
    iterations (no history then).  all_cores: the OpenMP build, for large
    canonical-mode solves: its canonical mode gives the same bits (tile
    partials formed independently and summed in tile order, the SpMV and the
    axpys element by element); its sequential-mode dots sum per-thread
    partials, so they differ from the single-thread ones in rounding."""
    lib = _load_omp() if all_cores else _load()
    if rr_period:
        if history:
            raise ValueError("no history with residual replacement")
        b = _vec(b, nx, ny)
        x0a = _vec(x0, nx, ny) if x0 is not None else None
        x = np.zeros_like(b)
        res = _Result()
        o = C.byref(order) if order is not None else None
        rc = lib.oracle_cg_rr(variant, mode, o, nx, ny, _ptr(b), _ptr(x0a), _ptr(x), tol,
                              maxit, rr_period, C.byref(res))
        if rc < 0:
            raise ValueError("oracle_cg_rr rejected the call: %d" % rc)
        return x, Result(status=res.status, iterations=res.iterations,
                         outer_iterations=res.outer_iterations,
                         rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)
    b = _vec(b, nx, ny)
    x0a = _vec(x0, nx, ny) if x0 is not None else None
    x = np.zeros_like(b)
    res = _Result()
    o = C.byref(order) if order is not None else None
    hist = None
    h = None
    if history:
        n = nx * ny
        hist = dict(gamma=np.zeros(history), r=np.zeros((history, n)),
                    p=np.zeros((history, n)), x=np.zeros((history, n)))
        h = _History(history, 0, _ptr(hist["gamma"]), _ptr(hist["r"]), _ptr(hist["p"]),
                     _ptr(hist["x"]))
    rc = lib.oracle_cg(variant, mode, o, nx, ny, _ptr(b), _ptr(x0a), _ptr(x), tol, maxit,
                       C.byref(res), C.byref(h) if h is not None else None)
    if rc < 0:
        raise ValueError("oracle_cg rejected the call: %d" % rc)
    out = Result(status=res.status, iterations=res.iterations,
                 outer_iterations=res.outer_iterations,
                 rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)
    if history:
        c = h.count
        hist = {k: v[:c] for k, v in hist.items()}
        return x, out, hist
    return x, out


_lib_omp = None


def _load_omp():
    """The all-core OpenMP timing build of the same sources (CPU baseline)."""
    global _lib_omp
    if _lib_omp is None:
        if _build.stale(omp=True):
            _build.build(omp=True)
        lib = C.CDLL(_build.LIB_OMP)
        P = C.c_void_p
        lib.oracle_cg.restype = C.c_int
        lib.oracle_cg.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.c_int32, C.c_int32,
                                  P, P, P, C.c_double, C.c_int32, C.POINTER(_Result),
                                  C.POINTER(_History)]
        lib.oracle_cg_rr.restype = C.c_int
        lib.oracle_cg_rr.argtypes = [C.c_int32, C.c_int32, C.POINTER(Order), C.c_int32,
                                     C.c_int32, P, P, P, C.c_double, C.c_int32, C.c_int32,
                                     C.POINTER(_Result)]
        lib.oracle_last_solve_seconds.restype = C.c_double
        lib.oracle_threads.restype = C.c_int
        _lib_omp = lib
    return _lib_omp


def last_solve_seconds():
    """Seconds the last solve of this thread spent in its iterations (the CSR
    assembly excluded): oracle.cg, cg3 and cg_vc."""
    return _load().oracle_last_solve_seconds()


def cg_timed(b, nx, ny, variant=VARIANT_CLASSIC, tol=0.0, maxit=10, all_cores=False):
    """The sequential-mode solve, timed: returns (Result, seconds of the
    iterations without the CSR assembly, threads used).  all_cores: the
    OpenMP build (rows split over the threads, per-thread partial sums added
    in thread order)."""
    lib = _load_omp() if all_cores else _load()
    b = _vec(b, nx, ny)
    x = np.zeros_like(b)
    res = _Result()
    rc = lib.oracle_cg(variant, MODE_SEQUENTIAL, None, nx, ny, _ptr(b), None, _ptr(x), tol, maxit,
                       C.byref(res), None)
    if rc < 0:
        raise ValueError("oracle_cg rejected the call: %d" % rc)
    out = Result(status=res.status, iterations=res.iterations,
                 rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)
    return out, lib.oracle_last_solve_seconds(), lib.oracle_threads()


def cheb_coeffs(nx, ny, s):
    """(c0, c1[s-1], c2[s-1]) of the Chebyshev preconditioner with s steps."""
    c0 = np.zeros(1)
    c1 = np.zeros(max(s - 1, 1))
    c2 = np.zeros(max(s - 1, 1))
    rc = _load().oracle_cheb_coeffs(nx, ny, s, _ptr(c0), _ptr(c1), _ptr(c2))
    if rc:
        raise ValueError("oracle_cheb_coeffs rejected the call: %d" % rc)
    return float(c0[0]), c1[:s - 1].copy(), c2[:s - 1].copy()


def cheb_apply(r, nx, ny, s, mode=MODE_SEQUENTIAL):
    """z = p_s(A) r, the Chebyshev preconditioner with s steps."""
    r = _vec(r, nx, ny)
    z = np.zeros_like(r)
    rc = _load().oracle_cheb_apply(nx, ny, mode, s, _ptr(r), _ptr(z))
    if rc:
        raise ValueError("oracle_cheb_apply rejected the call: %d" % rc)
    return z


def cheb_apply_f32(r, nx, ny, s):
    """z = M^-1 r in binary32 (r rounded to binary32 first)."""
    r32 = np.ascontiguousarray(np.asarray(r, dtype=np.float32).reshape(ny, nx))
    z = np.zeros_like(r32)
    rc = _load().oracle_cheb_apply_f32(nx, ny, s, r32.ctypes.data, z.ctypes.data)
    if rc:
        raise ValueError("oracle_cheb_apply_f32 rejected the call: %d" % rc)
    return z


def pcg(b, nx, ny, s, tol=1e-8, maxit=2000, x0=None, mode=MODE_SEQUENTIAL, order=None,
        order_rho=None, variant=VARIANT_CLASSIC):
    """CG preconditioned by the s-step Chebyshev polynomial in A: classic
    (variant 0) or pipelined (variant 1, Ghysels and Vanroose's form of
    Algorithm 2).  Canonical mode: classic sums rho = (r, z) in order_rho
    (default: order); every other dot follows order."""
    b = _vec(b, nx, ny)
    x0a = _vec(x0, nx, ny) if x0 is not None else None
    x = np.zeros_like(b)
    res = _Result()
    o = C.byref(order) if order is not None else None
    orho = C.byref(order_rho) if order_rho is not None else None
    rc = _load().oracle_pcg(variant, mode, o, orho, nx, ny, s, _ptr(b), _ptr(x0a), _ptr(x), tol,
                            maxit, C.byref(res))
    if rc < 0:
        raise ValueError("oracle_pcg rejected the call: %d" % rc)
    return x, Result(status=res.status, iterations=res.iterations,
                     outer_iterations=res.outer_iterations,
                     rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)


def refine(b, nx, ny, tol=1e-10, inner_tol=1e-4, maxit=200000, x0=None, precond=0):
    """FP32-inner / FP64-outer iterative refinement (see oracle_refine); precond
    = s > 0: the inner solve preconditioned by s Chebyshev steps in binary32
    (oracle_refine_pc)."""
    b = _vec(b, nx, ny)
    x0a = _vec(x0, nx, ny) if x0 is not None else None
    x = np.zeros_like(b)
    res = _Result()
    if precond:
        rc = _load().oracle_refine_pc(nx, ny, _ptr(b), _ptr(x0a), _ptr(x), tol, inner_tol,
                                      maxit, precond, C.byref(res))
    else:
        rc = _load().oracle_refine(nx, ny, _ptr(b), _ptr(x0a), _ptr(x), tol, inner_tol, maxit,
                                   C.byref(res))
    if rc < 0:
        raise ValueError("oracle_refine rejected the call: %d" % rc)
    return x, Result(status=res.status, iterations=res.iterations,
                     outer_iterations=res.outer_iterations,
                     rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)


# -- fixed point (cg_oracle_fixed.c): Q20.30 values as int64 counts of 2^-30 --

FX_FRAC = 30
FX_MAX = (1 << 49) - 1
FX_MIN = -(1 << 49)
FX_ONE = 1 << FX_FRAC


def fx_quantize(v):
    """Round-half-up, saturating quantization of one float to Q20.30 (count)."""
    return _load().oracle_fx_quantize(float(v))


def fx_value(k):
    return _load().oracle_fx_value(int(k))


def fx_mul(a, b):
    return _load().oracle_fx_mul(int(a), int(b))


def fx_axpy(a, x, y):
    """Q(y + a x) of counts."""
    return _load().oracle_fx_axpy(int(a), int(x), int(y))


def fx_axmy(a, x, y):
    """Q(y - a x) of counts."""
    return _load().oracle_fx_axmy(int(a), int(x), int(y))


def fx_div(n, d):
    if d <= 0:
        raise ValueError("fx_div needs d > 0")
    return _load().oracle_fx_div(int(n), int(d))


def _ivec(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.int64)
    if n is not None and a.size != n:
        raise ValueError("vector has %d entries, needs %d" % (a.size, n))
    return a


def fx_dot(a, b):
    a = _ivec(a).ravel()
    b = _ivec(b, a.size).ravel()
    return _load().oracle_fx_dot(a.size, _ptr(a), _ptr(b))


def fx_spmv(u, nx, ny):
    u = _ivec(u, nx * ny).reshape(ny, nx)
    y = np.zeros_like(u)
    rc = _load().oracle_fx_spmv(nx, ny, _ptr(u), _ptr(y))
    if rc:
        raise RuntimeError("oracle_fx_spmv failed: %d" % rc)
    return y


def cg_fixed(b, nx, ny, variant=VARIANT_CLASSIC, tol=1e-6, maxit=2000, x0=None):
    """Algorithm 1 or 2 in Q20.30 (see cg_oracle_fixed.c).  b and x0 are
    float64 and quantized on entry.  Returns (x float64, x counts int64,
    Result)."""
    b = _vec(b, nx, ny)
    x0a = _vec(x0, nx, ny) if x0 is not None else None
    xq = np.zeros((ny, nx), np.int64)
    x = np.zeros_like(b)
    res = _Result()
    rc = _load().oracle_cg_fixed(variant, nx, ny, _ptr(b), _ptr(x0a), _ptr(xq), _ptr(x), tol,
                                 maxit, C.byref(res))
    if rc < 0:
        raise ValueError("oracle_cg_fixed rejected the call: %d" % rc)
    return x, xq, Result(status=res.status, iterations=res.iterations,
                         outer_iterations=res.outer_iterations,
                         rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)
