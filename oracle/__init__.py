"""Plain FP64 CPU oracle of the TAPS slab solve (test infrastructure only).

This package is the checker, not the product: only ``tests/``, the smoke check
and the CPU-baseline leg of the benchmark may import it.  It shares no code
with the HIP path; both sides take their inputs from ``taps_workloads``.

Every function follows one passage of the paper (Guo et al., "Tensor-
decomposition-based A Priori Surrogate (TAPS) modeling for ultra large-scale
simulations") and is written for reading, not speed: dense or scipy-sparse
matrices, library primitives (matmul, LAPACK solves) for single steps, no
blocking or fusion.

Modules
-------
quadrature   Gauss-Legendre rule on each element (Sec. 2.1, MLP vs C-HiDeNN table)
basis        1D C-HiDeNN shape functions and derivatives (Sec. 2.1; Sec. 2.5)
assemble     1D mass / stiffness / time-derivative / weighted-mass matrices and
             load vectors (Sec. 2.5, spatial/parametric/temporal integrals)
separated    separated operator, Grams, Hadamard couplings, force, dim system,
             projected residual (Sec. 2.5, coefficient matrices; Sec. 2.6)
als          subspace iteration, Algorithm 1 (Sec. 2.6)
reconstruct  TD interpolation of the rank-M field (Sec. 2.3)
fulltensor   full-tensor Galerkin solve on tiny grids (the C-HiDeNN solution
             without decomposition, Sec. 2.7)
problems     term tables and separated loads of the paper's PDEs (Sec. 2.4)
"""
