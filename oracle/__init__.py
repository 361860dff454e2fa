"""FP64 CPU oracle for the pipelined flexible Krylov solvers.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the GPU
path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package
(``paper_1511_07226_amd``) never does, and this package never imports the
product package.  The two share no code: only the seeded input generators in
``gen/`` serve both.

Everything here is numpy in float64, written from the paper
(Sanan, Schnepp, May, "Pipelined, Flexible Krylov Subspace Methods"):

* ``stencil``  -- the variable-coefficient diffusion / upwind convection-
  diffusion operators of the synthetic sinker workloads (their plain
  definition) and their diagonal;
* ``precond``  -- Jacobi, k-step Jacobi-PCG and k-step right-Jacobi GMRES
  inner solves (the flexible, nonlinear preconditioners B), plus the noisy
  preconditioner of the section 2.2.1 toy study;
* ``noise``    -- the counter-based Gaussian generator (Philox4x64-10 and
  Box-Muller) behind the seeded noisy preconditioner that a GPU solve can
  reproduce draw for draw;
* ``krylov``   -- FCG (Alg. 2), PCG (Alg. 3), naive PIPEFCG (Alg. 7),
  PIPEFCG (Alg. 8), GCR (Alg. 9), PIPEGCR (Alg. 11), PIPEGCR_w (Alg. 12),
  FGMRES (Alg. 13) and PIPEFGMRES (Alg. 15), with the truncation rules and
  breakdown restarts of section 5, and Givens least squares.

Parity status of every function is stated in its docstring; functions with
no independent pin say "parity unpinned".
"""
from .stencil import StencilOperator, harmonic_face  # noqa: F401
from .precond import (  # noqa: F401
    identity_pc, jacobi_pc, jacobi_pcg, jacobi_gmres, block_jacobi_pcg, block_operator,
    noisy_pc, make_pc,
)
from .noise import philox4x64, box_muller, gauss, CounterNoisyPC  # noqa: F401
from .krylov import (  # noqa: F401
    Result, truncation_nu, givens_lstsq, solve, estimate_sigma, METHODS,
)
