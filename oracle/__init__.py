"""CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 implementation of what the interior-point hot path
computes, written from the paper (arXiv 2508.16094) and independent of the
HIP library: it shares no code, header, table or helper with
``paper_2508_16094_amd`` and never imports it.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or run anything here.

Modules
  model     f, grad f, g, J and the Lagrangian Hessian (Section 1, problem (1);
            Section 4 derivative templates)
  symbolic  fill-reducing ordering, elimination tree, column counts and
            supernodes (Section 2, LDL^T with a fill-reducing permutation)
  cholesky  dense and simple (column, left-looking) sparse Cholesky in C
  kkt       condensed KKT matrix (Section 3, primal condensed system) and the
            full regularised KKT system (Section 3, eq. kkt_system)
  ipm       predictor-corrector interior-point iteration (Section 3)
  checker   scaled primal/dual infeasibility and complementarity
  mlp       FP64 MLP forward/backward for the learned warm start
"""
