"""Plain FP64 CPU oracle for the nested-grid multigrid Poisson solver
(Wang & Yen, arXiv:2001.02327).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of the benchmark.  The product library never imports it.

  oracle.core   -- ctypes wrapper of the C implementation (nested_oracle.c):
                   the method's schedule step by step (Sec. 2.2-2.4)
  oracle.dense  -- direct sparse solve of the nested discrete system, the
                   plain definition of the fixed point the iteration reaches
  oracle.norms  -- composite error norms of Sec. 3
"""
