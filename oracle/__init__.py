"""Plain, slow, CPU-only reference ("oracle") for the element-local
space-time predictor of ADER-DG for Biot poroelasticity
(Wolf et al., arXiv 2108.10565).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything under this directory: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
use it.  It shares no code, header, table or helper with the HIP library
in ``paper_2108_10565_amd/``; the only module both sides use is the
seeded input generator ``paper_2108_10565_amd/workload.py``, which holds
no arithmetic of the method.

What it computes (the plain definition, no blocking or fusion):

* ``oracle.basis``   -- the temporal Legendre basis and its matrices
  S, W, w, K^tau (section "Space-Time predictor", definitions after
  eq:stp), and the spatial Dubiner basis with its mass and stiffness
  matrices M and K^alpha, all in exact rational arithmetic.
* ``oracle.stp``     -- assembly of the full space-time system
  Y Q = r of eq:stp-lineq / eq:linear_system as a dense matrix, and its
  solution by dense LU with partial pivoting in float64.
* ``oracle.brute``   -- an independent route to Y for tiny degrees, by
  direct space-time quadrature of the integrals of eq:stp (used only to
  pin ``oracle.stp``).

Parity status: every function here is pinned by ``-m "not gpu"`` tests
(see ``tests/test_oracle_*.py``); none is "parity unpinned".
"""
