"""ctypes binding of libcg.so (include/cg.h), same names as the C ABI.

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch supplies device memory (tensors) and the caller's stream; numpy
arrays are passed as host memory.  The library must be built (build.py);
nothing here falls back to another implementation.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcg.so")

CG_VARIANT_CLASSIC, CG_VARIANT_PIPELINED = 0, 1
CG_PREC_FP64, CG_PREC_FP32_REFINED, CG_PREC_FIXED, CG_PREC_AUTO = 0, 1, 2, 3
CG_MEM_HOST, CG_MEM_DEVICE = 0, 1
CG_OK, CG_PENDING, CG_NOT_CONVERGED, CG_BREAKDOWN = 0, 1, 2, 3
CG_E_INVALID, CG_E_NOMEM, CG_E_DEVICE, CG_E_BUSY, CG_E_TICKET = -1, -2, -3, -4, -5


class cg_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("arena", C.c_void_p),
                ("arena_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("tune_cache", C.c_char_p)]


class cg_problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("mem", C.c_int32),
                ("b", C.c_void_p), ("x0", C.c_void_p), ("x", C.c_void_p),
                ("tol", C.c_double), ("maxit", C.c_int32), ("variant", C.c_int32),
                ("precision", C.c_int32), ("inner_tol", C.c_double),
                ("precond", C.c_int32), ("nz", C.c_int32), ("rr_period", C.c_int32),
                ("kx", C.c_void_p), ("ky", C.c_void_p)]


class cg_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32),
                ("outer_iterations", C.c_int32), ("pad_", C.c_int32),
                ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double),
                ("device_seconds", C.c_double), ("latency_seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class cg_plan_info(C.Structure):
    _fields_ = [("path", C.c_int32), ("cols_per_lane", C.c_int32), ("lanes", C.c_int32),
                ("waves", C.c_int32), ("rows", C.c_int32), ("threads2", C.c_int32),
                ("tiles", C.c_int32), ("grid", C.c_int32), ("pitch", C.c_int32),
                ("seg_rows", C.c_int32), ("seg_waves", C.c_int32), ("seg_cols", C.c_int32),
                ("cheb_rows", C.c_int32), ("cheb_tiles", C.c_int32), ("cheb_grid", C.c_int32),
                ("row_stride", C.c_int32), ("walk_alt", C.c_int32), ("walk_z", C.c_int32),
                ("footprint", C.c_size_t)]


class cg_kstat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("seconds", C.c_double),
                ("bytes", C.c_double)]


SYMBOLS = ["cg_create", "cg_destroy", "cg_solve", "cg_solve_batch", "cg_submit", "cg_poll",
           "cg_status_str", "cg_apply", "cg_dot", "cg_plan", "cg_footprint", "cg_validate",
           "cg_tune", "cg_pin_tile", "cg_set_profiling", "cg_kernel_stats", "cg_version",
           "cg_stream_probe", "cg_mul_probe", "cg_solve_batch_small_noalloc"]

_lib = None


def load():
    """Loads libcg.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcg.so is not built: run paper_1803_03797_amd/build.py "
                           "(or __graft_entry__.build())")
    # PyTorch ships its own HIP runtime under the same soname as ROCm's; load it
    # first so that a process using both has exactly one runtime (torch's).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P, I, D = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "cg_create": (C.c_int, [C.POINTER(cg_config), C.POINTER(P)]),
        "cg_destroy": (C.c_int, [P]),
        "cg_solve": (C.c_int, [P, C.POINTER(cg_problem), C.POINTER(cg_result)]),
        "cg_solve_batch": (C.c_int, [P, C.POINTER(cg_problem), I, C.POINTER(cg_result)]),
        "cg_submit": (C.c_int, [P, C.POINTER(cg_problem), C.POINTER(C.c_uint64)]),
        "cg_poll": (C.c_int, [P, C.c_uint64, C.POINTER(cg_result)]),
        "cg_status_str": (C.c_char_p, [C.c_int]),
        "cg_apply": (C.c_int, [P, I, I, I, P, P]),
        "cg_dot": (C.c_int, [P, I, I, I, P, P, C.POINTER(D)]),
        "cg_plan": (C.c_int, [P, C.POINTER(cg_problem), C.POINTER(cg_plan_info)]),
        "cg_footprint": (C.c_int, [C.POINTER(cg_problem), C.POINTER(C.c_size_t)]),
        "cg_validate": (C.c_int, [C.POINTER(cg_problem)]),
        "cg_tune": (C.c_int, [P, I, I, I, I]),
        "cg_pin_tile": (C.c_int, [P, I, I, I, I, I, I]),
        "cg_stream_probe": (C.c_int, [P, I, C.c_size_t, I, C.POINTER(D), C.POINTER(D)]),
        "cg_mul_probe": (C.c_int, [P, I, I, C.POINTER(D), C.POINTER(D)]),
        "cg_set_profiling": (C.c_int, [P, I]),
        "cg_kernel_stats": (C.c_int, [P, C.POINTER(cg_kstat), I, C.POINTER(I), I]),
        "cg_version": (C.c_char_p, []),
        "cg_solve_batch_small_noalloc": (C.c_int, [C.POINTER(cg_problem), I, P,
                                                   C.POINTER(cg_result)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def cg_status_str(code):
    return load().cg_status_str(code).decode()


def cg_solve_batch_small_noalloc(probs, stream=None):
    """Small solves with no device allocation (no context; the current HIP
    device; `stream` a hipStream_t handle or None).  Returns (worst status,
    results)."""
    n = len(probs)
    arr = (cg_problem * n)(*probs)
    res = (cg_result * n)()
    rc = _check("cg_solve_batch_small_noalloc",
                load().cg_solve_batch_small_noalloc(arr, n, stream, res))
    return rc, list(res)


class CGError(RuntimeError):
    def __init__(self, where, code):
        super().__init__("%s: %s (%d)" % (where, cg_status_str(code), code))
        self.code = code


def _check(where, rc):
    if rc < 0:
        raise CGError(where, rc)
    return rc


def _ptr_mem(a):
    """(pointer, memspace) of a torch tensor or numpy array (float64, contiguous)."""
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError("numpy vectors must be C-contiguous float64")
        return a.ctypes.data, CG_MEM_HOST
    import torch
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError("tensors must be contiguous float64")
        return a.data_ptr(), (CG_MEM_DEVICE if a.is_cuda else CG_MEM_HOST)
    raise TypeError("unsupported vector type %r" % type(a))


def _numel(v):
    return v.size if isinstance(v, np.ndarray) else v.numel()


def make_problem(b, x, nx, ny, tol=1e-8, maxit=2000, variant=CG_VARIANT_CLASSIC,
                 precision=CG_PREC_FP64, x0=None, inner_tol=0.0, precond=0, nz=0, kx=None,
                 ky=None, rr_period=0):
    """nz > 1: the 3D 7-point problem on nx x ny x nz (vectors of nx*ny*nz).
    kx, ky: face conductivities of the variable-coefficient operator, ny x
    (nx+1) and (ny+1) x nx, in the memory space of b (the caller keeps them
    alive until the solve returns).  rr_period: residual replacement every
    rr_period iterations of the pipelined variant (0: none)."""
    pb, mb = _ptr_mem(b)
    px, mx = _ptr_mem(x)
    p0, m0 = _ptr_mem(x0)
    pkx, mkx = _ptr_mem(kx)
    pky, mky = _ptr_mem(ky)
    if mb != mx or (m0 is not None and m0 != mb):
        raise ValueError("b, x and x0 must live in the same memory space")
    if (kx is None) != (ky is None):
        raise ValueError("kx and ky come together")
    if kx is not None:
        if mkx != mb or mky != mb:
            raise ValueError("kx and ky must live in the memory space of b")
        if _numel(kx) != ny * (nx + 1) or _numel(ky) != (ny + 1) * nx:
            raise ValueError("kx must hold ny*(nx+1) values and ky (ny+1)*nx")
    n = nx * ny * max(nz, 1)
    for v in (b, x, x0):
        if v is not None and _numel(v) != n:
            raise ValueError("vector size does not match the %dx%dx%d grid" % (nx, ny, max(nz, 1)))
    p = cg_problem(nx, ny, mb, pb, p0, px, float(tol), int(maxit), int(variant),
                   int(precision), float(inner_tol), int(precond), int(nz), int(rr_period), pkx,
                   pky)
    return p


_VC_PLACEHOLDER = C.c_double(1.0)


class Context:
    """Owns one cg_ctx.  `stream` may be a torch.cuda.Stream; `arena` a uint8
    CUDA tensor the library uses for all its workspace."""

    def __init__(self, device=0, stream=None, arena=None, arena_bytes=0, max_slots=0,
                 tune_cache=None):
        lib = load()
        cfg = cg_config()
        cfg.device = device
        cfg.stream = stream.cuda_stream if stream is not None else None
        if arena is not None:
            cfg.arena = arena.data_ptr()
            cfg.arena_bytes = arena.numel() * arena.element_size()
            self._arena = arena
        else:
            cfg.arena = None
            cfg.arena_bytes = arena_bytes
        cfg.max_slots = max_slots
        cfg.tune_cache = tune_cache.encode() if tune_cache else None
        h = C.c_void_p()
        _check("cg_create", lib.cg_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self.lib = lib

    def close(self):
        if self.h:
            self.lib.cg_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- solves --
    def cg_solve(self, prob):
        res = cg_result()
        rc = _check("cg_solve", self.lib.cg_solve(self.h, C.byref(prob), C.byref(res)))
        return rc, res

    def solve(self, b, x, nx, ny, **kw):
        return self.cg_solve(make_problem(b, x, nx, ny, **kw))

    def cg_solve_batch(self, probs):
        n = len(probs)
        arr = (cg_problem * n)(*probs)
        res = (cg_result * n)()
        rc = _check("cg_solve_batch", self.lib.cg_solve_batch(self.h, arr, n, res))
        return rc, list(res)

    def cg_submit(self, prob):
        t = C.c_uint64()
        _check("cg_submit", self.lib.cg_submit(self.h, C.byref(prob), C.byref(t)))
        return t.value

    def cg_poll(self, ticket):
        res = cg_result()
        rc = _check("cg_poll", self.lib.cg_poll(self.h, C.c_uint64(ticket), C.byref(res)))
        return rc, res

    # -- building blocks --
    def cg_apply(self, u, y, nx, ny):
        pu, mu = _ptr_mem(u)
        py, my = _ptr_mem(y)
        if mu != my:
            raise ValueError("u and y must live in the same memory space")
        _check("cg_apply", self.lib.cg_apply(self.h, nx, ny, mu, pu, py))

    def cg_dot(self, a, b, nx, ny):
        pa, ma = _ptr_mem(a)
        pb, mb = _ptr_mem(b)
        if ma != mb:
            raise ValueError("a and b must live in the same memory space")
        out = C.c_double()
        _check("cg_dot", self.lib.cg_dot(self.h, nx, ny, ma, pa, pb, C.byref(out)))
        return out.value

    def cg_plan(self, nx, ny, variant=CG_VARIANT_CLASSIC, precision=CG_PREC_FP64, precond=0,
                nz=0, vc=False, rr_period=0):
        """vc: plan the variable-coefficient operator (the coefficients are not
        read: a placeholder stands for them)."""
        k = C.addressof(_VC_PLACEHOLDER) if vc else None
        p = cg_problem(nx, ny, CG_MEM_DEVICE, None, None, None, 1e-8, 1, variant, precision, 0.0,
                       precond, nz, rr_period, k, k)
        info = cg_plan_info()
        _check("cg_plan", self.lib.cg_plan(self.h, C.byref(p), C.byref(info)))
        return info

    def cg_tune(self, nx, ny, variant=CG_VARIANT_CLASSIC, precision=CG_PREC_FP64):
        return _check("cg_tune", self.lib.cg_tune(self.h, nx, ny, variant, precision))

    def cg_pin_tile(self, nx, ny, rows, grid=0, precision=CG_PREC_FP64, cols_per_lane=0):
        return _check("cg_pin_tile", self.lib.cg_pin_tile(self.h, nx, ny, precision, rows, grid,
                                                          cols_per_lane))

    def cg_stream_probe(self, pattern, elems, reps=5):
        sec, nbytes = C.c_double(), C.c_double()
        _check("cg_stream_probe", self.lib.cg_stream_probe(self.h, pattern, elems, reps,
                                                           C.byref(sec), C.byref(nbytes)))
        return sec.value, nbytes.value

    def cg_mul_probe(self, rounds=4096, reps=3):
        t, n = C.c_double(), C.c_double()
        _check("cg_mul_probe", self.lib.cg_mul_probe(self.h, rounds, reps, C.byref(t), C.byref(n)))
        return t.value, n.value

    def cg_set_profiling(self, on):
        return _check("cg_set_profiling", self.lib.cg_set_profiling(self.h, 1 if on else 0))

    def cg_kernel_stats(self, reset=False):
        n = C.c_int32()
        buf = (cg_kstat * 64)()
        _check("cg_kernel_stats", self.lib.cg_kernel_stats(self.h, buf, 64, C.byref(n),
                                                           1 if reset else 0))
        out = {}
        for i in range(min(n.value, 64)):
            k = buf[i]
            out[k.name.decode()] = dict(launches=k.launches, seconds=k.seconds, bytes=k.bytes)
        return out


def cg_footprint(prob):
    n = C.c_size_t()
    _check("cg_footprint", load().cg_footprint(C.byref(prob), C.byref(n)))
    return n.value


def cg_validate(prob):
    return load().cg_validate(C.byref(prob))


def cg_version():
    return load().cg_version().decode()
