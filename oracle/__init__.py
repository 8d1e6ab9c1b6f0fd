"""CPU FP64 oracle for the PSD-cone projection by composite polynomial filtering.

ORACLE — test infrastructure only. Only tests/, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it. It shares no code with the
HIP library (``paper_2507_09165_amd``), and the library never imports it.
"""
from .psd import (  # noqa: F401
    deflation_pairs,
    efloat,
    efloat_rows,
    filter_stage,
    final_combine,
    g_scalar,
    gemm_count,
    jacobi_eig,
    lanczos_bound,
    lanczos_run,
    newton_schulz_stage,
    NS_ITERS,
    project_exact,
    project_exact_eigh,
    project_deflated,
    project_poly,
    project_spectral,
    spectral_bound,
    stage_rows,
    start_vector,
    sym_from_upper,
)
from . import admm, tables  # noqa: F401
