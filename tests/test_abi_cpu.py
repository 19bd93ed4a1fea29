"""CPU-side checks of the C ABI library: it loads, exports every function the
header declares, and its host-only calls (validation, footprint) behave.  No
compute call is made without a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1803_03797_amd import cg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "cg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(cg_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = cg.load()
    names = header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(cg.SYMBOLS) == names


def test_status_strings():
    for code in (0, 1, 2, 3, -1, -2, -3, -4, -5):
        assert cg.cg_status_str(code).startswith("CG_")
    assert cg.cg_status_str(99) == "CG_UNKNOWN"
    assert "gfx950" in cg.cg_version()


def _prob(**kw):
    d = dict(nx=10, ny=7, mem=cg.CG_MEM_HOST, b=1, x0=None, x=2, tol=1e-8, maxit=10,
             variant=0, precision=0, inner_tol=0.0, precond=0, nz=0, kx=None, ky=None,
             rr_period=0)
    d.update(kw)
    return cg.cg_problem(d["nx"], d["ny"], d["mem"], d["b"], d["x0"], d["x"], d["tol"],
                         d["maxit"], d["variant"], d["precision"], d["inner_tol"],
                         d["precond"], d["nz"], d["rr_period"], d["kx"], d["ky"])


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-1), dict(tol=-1e-3), dict(tol=1.0),
                                 dict(tol=float("nan")), dict(maxit=0), dict(b=None),
                                 dict(x=None), dict(mem=7), dict(variant=2), dict(precision=5),
                                 dict(precision=1, inner_tol=1.5), dict(precision=4),
                                 dict(precision=2, nx=101, ny=101),
                                 dict(precision=2, nx=100, ny=101),
                                 dict(precision=2, nx=1, ny=6783),
                                 dict(precision=2, nx=5088, ny=1),
                                 dict(precond=-1), dict(precond=9),
                                 dict(precond=4, precision=2),
                                 dict(nz=-1), dict(nz=3, precond=2), dict(nz=3, precision=1),
                                 dict(nz=3, precision=2), dict(nx=2048, ny=2048, nz=1024),
                                 dict(kx=3), dict(ky=4), dict(kx=3, ky=4, nz=2),
                                 dict(kx=3, ky=4, precond=2), dict(kx=3, ky=4, precision=1),
                                 dict(kx=3, ky=4, precision=2),
                                 # residual replacement: even period, pipelined FP64 2D
                                 dict(rr_period=3, variant=1), dict(rr_period=-2, variant=1),
                                 dict(rr_period=2), dict(rr_period=2, variant=1, precision=1),
                                 dict(rr_period=2, variant=1, precision=2),
                                 dict(rr_period=2, variant=1, precond=1),
                                 dict(rr_period=2, variant=1, nz=3),
                                 # the precision policy: problems FP64 and refined both take
                                 dict(precision=3, nz=3),
                                 dict(precision=3, kx=3, ky=4),
                                 dict(precision=3, variant=1, rr_period=2),
                                 dict(precision=3, inner_tol=1.5, nx=300, ny=300),
                                 # padded row stride times 14 interleaved vectors > int32
                                 dict(nx=300_000_000, ny=7, variant=1),
                                 dict(nx=153_391_617, ny=1)])
def test_validation_rejects(bad):
    assert cg.cg_validate(_prob(**bad)) == cg.CG_E_INVALID


def test_validation_accepts():
    assert cg.cg_validate(_prob()) == cg.CG_OK
    assert cg.cg_validate(_prob(tol=0.0, precision=1, inner_tol=0.0)) == cg.CG_OK
    # fixed point: (nx + 1)(ny + 2) + nx ny <= 20352; inner_tol is ignored
    for nx, ny in ((1, 1), (100, 100), (98, 102), (1, 6782), (5087, 1)):
        assert cg.cg_validate(_prob(nx=nx, ny=ny, precision=2)) == cg.CG_OK
    assert cg.cg_validate(_prob(precision=2, inner_tol=7.0)) == cg.CG_OK
    # widest row whose padded stride times 14 vectors still fits int32
    assert cg.cg_validate(_prob(nx=153_391_360, ny=1, variant=1)) == cg.CG_OK
    # the 3D operator: nz > 1 (nz = 0 or 1 is the 2D problem)
    for nz in (0, 1, 2, 64):
        for v in (0, 1):
            assert cg.cg_validate(_prob(nz=nz, variant=v)) == cg.CG_OK
    # variable coefficients: 2D FP64, either variant (nz = 1 is 2D)
    for v in (0, 1):
        for nz in (0, 1):
            assert cg.cg_validate(_prob(kx=3, ky=4, variant=v, nz=nz)) == cg.CG_OK
    # the precision policy: either variant, any size, with or without the
    # preconditioner
    for nx, ny in ((10, 7), (181, 181), (182, 181), (2048, 2048)):
        for pc in (0, 4):
            assert cg.cg_validate(_prob(nx=nx, ny=ny, precision=3, precond=pc)) == cg.CG_OK
            assert cg.cg_validate(_prob(nx=nx, ny=ny, precision=3, variant=1,
                                        precond=pc)) == cg.CG_OK
    # residual replacement: pipelined, 5-point or variable coefficients
    for rr in (2, 4, 100):
        assert cg.cg_validate(_prob(rr_period=rr, variant=1)) == cg.CG_OK
        assert cg.cg_validate(_prob(rr_period=rr, variant=1, kx=3, ky=4)) == cg.CG_OK
    # Chebyshev preconditioner: 1..8 steps, FP64 of either variant or the
    # FP32 inner solve of the refinement
    for s in range(0, 9):
        assert cg.cg_validate(_prob(precond=s)) == cg.CG_OK
        assert cg.cg_validate(_prob(precond=s, variant=1)) == cg.CG_OK
        assert cg.cg_validate(_prob(precond=s, precision=1)) == cg.CG_OK
        assert cg.cg_validate(_prob(precond=s, precision=1, variant=1)) == cg.CG_OK


def test_auto_precision_footprint_follows_its_choice():
    """Below 20480 unknowns the policy picks FP64, from there FP32 refinement:
    the footprint is that of the precision chosen."""
    for nx, ny, chosen in ((143, 143, 0), (128, 160, 1), (4096, 4096, 1), (100, 100, 0),
                           (181, 181, 1)):
        for pc in (0, 4):
            assert cg.cg_footprint(_prob(nx=nx, ny=ny, precision=3, precond=pc)) == \
                cg.cg_footprint(_prob(nx=nx, ny=ny, precision=chosen, precond=pc))


def test_footprint_per_unknown():
    """Resident bytes per unknown: classic 5 FP64 vectors, pipelined 8, refined
    2 FP64 + 4 FP32, preconditioned classic 6, preconditioned refined 2 FP64 +
    5 FP32, variable coefficients 4 more (plus padding and small
    partial/state buffers)."""
    n = 4096
    for variant, prec, per, pre in ((0, 0, 40, 0), (1, 0, 64, 0), (0, 1, 32, 0), (0, 0, 48, 4),
                                    (0, 1, 36, 4)):
        fp = cg.cg_footprint(_prob(nx=n, ny=n, variant=variant, precision=prec, precond=pre))
        assert per * n * n <= fp <= per * n * n * 1.01 + (1 << 20)
    # variable coefficients: four more FP64 arrays (west, east, south, north)
    for variant, per in ((0, 72), (1, 96)):
        fp = cg.cg_footprint(_prob(nx=n, ny=n, variant=variant, kx=3, ky=4))
        assert per * n * n <= fp <= per * n * n * 1.01 + (1 << 20)


def test_create_without_gpu_fails_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = cg.load()
    h = C.c_void_p()
    cfg = cg.cg_config(0, None, None, 0, 0, None)
    assert lib.cg_create(C.byref(cfg), C.byref(h)) == cg.CG_E_DEVICE
    assert not h.value
    assert lib.cg_destroy(None) == cg.CG_E_INVALID


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets
    the C compiler gives the header's structures."""
    structs = {"cg_config": cg.cg_config, "cg_problem": cg.cg_problem,
               "cg_result": cg.cg_result, "cg_plan_info": cg.cg_plan_info,
               "cg_kstat": cg.cg_kstat}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "cg.h"', 'int main(void) {']
    for name, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for name, py in structs.items():
        assert got[(name, "size")] == C.sizeof(py), name
        for f in py._fields_:
            assert got[(name, f[0])] == getattr(py, f[0]).offset, (name, f[0])


def test_noalloc_rejects_before_any_device_work():
    """cg_solve_batch_small_noalloc validates every problem first: host memory,
    grids too large for the on-chip solver, other precisions, n outside 1..64."""
    lib = cg.load()
    ok = _prob(mem=cg.CG_MEM_DEVICE, nx=20, ny=30)
    bad = [_prob(nx=20, ny=30), _prob(mem=cg.CG_MEM_DEVICE, nx=200, ny=200),
           _prob(mem=cg.CG_MEM_DEVICE, nx=20, ny=30, precision=1),
           _prob(mem=cg.CG_MEM_DEVICE, nx=20, ny=30, precond=2),
           _prob(mem=cg.CG_MEM_DEVICE, nx=20, ny=30, nz=4),
           _prob(mem=cg.CG_MEM_DEVICE, nx=20, ny=30, kx=3, ky=4),
           _prob(mem=cg.CG_MEM_DEVICE, nx=512, ny=20)]
    res = (cg.cg_result * 65)()
    for p in bad:
        arr = (cg.cg_problem * 2)(ok, p)
        assert lib.cg_solve_batch_small_noalloc(arr, 2, None, res) == cg.CG_E_INVALID
    arr = (cg.cg_problem * 65)(*([ok] * 65))
    assert lib.cg_solve_batch_small_noalloc(arr, 65, None, res) == cg.CG_E_INVALID
    assert lib.cg_solve_batch_small_noalloc(arr, 0, None, res) == cg.CG_E_INVALID
