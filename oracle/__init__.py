"""Plain FP64 CPU oracle for the PAW-FE R-ChFSI filter path (TEST INFRASTRUCTURE).

This package is the reference the GPU library is checked against.  It is
written from the paper's definitions and shares no code with the HIP path:
its own Gauss-Lobatto-Legendre and Gauss tables (NumPy's Legendre routines),
element matrices built by direct 3-D quadrature loops, global operators
assembled with scipy.sparse, Algorithm 2 taken step by step, and a dense
generalized eigensolve for the Rayleigh-Ritz step.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path never calls into it.

Modules
  fe      mesh (uniform or graded two-level), DOF map, colouring,
          reference element, local operators with the optional GGA term
          (FE discretization section; cell-level H/M entries)
  paw     projectors, projector matrix C^a, PAW H/S, approximate inverse
          overlap (FE non-local contribution; Sinv approximation)
  chfsi   Algorithm 1 steps 2-6 and Algorithm 2 (residual-based filter),
          the standard scaled Chebyshev filter, Rayleigh-Ritz (also with the
          mixed-precision subspace rotation), residual norms, k-step Lanczos
          bounds, the outer loop to a residual tolerance
  grad    band energy E = sum_n x_n^H H x_n and its gradient with respect to
          V_eff at quadrature points and Delta_H

Every function is pinned by tests/test_oracle_*.py.  The oracle has no
emulation of the FP32 / bf16x3 filter: the library's mixed paths are
checked against the FP64 oracle directly (filter output within the FP32
error, eigenvalues after an FP64 Rayleigh-Ritz within 1e-6 Ha).
"""
