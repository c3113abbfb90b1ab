"""CPU oracle for the PMCHWT (Omit) proxy fast direct solver (arXiv 2603.09381).

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path imports, calls
or links this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It is plain, slow FP64 numpy/scipy
written from the paper, sharing no code with the HIP path.

Modules
  layer     boundary quantities, Hankel kernels (Sec. 2.1), Kress/Maue Nystrom
            blocks for the diagonal (Sec. 2.2 with Kress quadrature)
  dense     the full PMCHWT (Omit) system, plane-wave right-hand side, partial
            pivoted LU solve (Sec. 2.2, Sec. 4), far field
  analytic  single-disk Mie series and multi-disk multipole (T-matrix) solutions
  fast      the proxy + interpolative-decomposition recursive solver, written
            step by step in the order of Sec. 3, for step-level comparison
"""
