"""CPU oracle for CG on the unscaled 5-point Laplacian, the 7-point one in 3D
and the variable-coefficient 5-point operator (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  The GPU library never imports, links or executes it.
"""
from .oracle import (  # noqa: F401
    MODE_CANONICAL, MODE_SEQUENTIAL, VARIANT_CLASSIC, VARIANT_PIPELINED,
    OR_OK, OR_NOT_CONVERGED, OR_BREAKDOWN, OR_E_INVALID,
    Order, csr, spmv, dot, cg, refine, lib_path, cg_fixed, cheb_coeffs, cheb_apply, pcg,
    csr3, spmv3, cg3, csr_vc, spmv_vc, cg_vc, cg_timed, cheb_apply_f32, last_solve_seconds,
)
