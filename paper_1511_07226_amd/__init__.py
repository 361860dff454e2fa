"""pfk: pipelined flexible Krylov solvers on AMD Instinct MI355X (gfx950).

Thin Python binding over the C ABI of ``libpfk.so`` (declared in
``include/pfk.h``).  Every step of a solve runs in the library's HIP kernels;
this package only marshals arguments.  PyTorch provides device memory and
streams.  The library must have been built (``python -m
paper_1511_07226_amd.build``); importing the binding without it raises.
"""
from .binding import (  # noqa: F401
    FCG, PIPEFCG, GCR, PIPEGCR, FGMRES, PIPEFGMRES, PIPEGCR_W, PIPEFCG_NAIVE, METHODS,
    PC_NONE, PC_JACOBI, PC_JACOBI_PCG, PC_JACOBI_GMRES, PC_BLOCK_JACOBI_PCG, PC_NOISY, PC_KINDS,
    FP64, FP32_BF16COEF,
    PfkError, Operator, Precond, Session, SolveInfo, SolveOpts, Batch, Tuning, Server,
    solve, solve_noalloc, solve_batched, workspace_bytes, estimate_sigma, lib, lib_path, EXPORTED,
)
