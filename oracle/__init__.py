"""ORACLE -- plain FP64 CPU implementation of the VMS Newton-Schur method.

This package is TEST INFRASTRUCTURE.  Only tests/, the smoke check
(__graft_entry__.smoke) and the CPU-baseline leg of bench.py may import,
call, link or execute anything in it.  The GPU library never uses it, and
it shares no code with the GPU library: the only common dependency is the
seeded input generator package `workloads`, which holds no method
arithmetic.

Modules:
  quadrature  conical-product Gauss-Jacobi rule on the tet (Golub-Welsch)
  element.c   element residual and pointwise-linearised tangent (quadrature)
  element     ctypes wrapper and gcc build of element.c
  vms         condensation, assembly, Dirichlet elimination, GMRES, Newton,
              brute-force uncondensed Newton
  learned_pc  features, MLP forward/backward, loss, Adam (learned block-Jacobi)
  errors      L2 errors against closed-form fields
Every function is pinned by tests in tests/test_oracle_*.py; see the
docstrings there for what fixes each result.
"""
