"""FP64 CPU oracle for the tensor-train grid-based filter.

TEST INFRASTRUCTURE.  This package is the checker, not the product: only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run it.  It shares no code with the HIP library
(``paper_2501_07942_amd``), and neither imports the other; the only common
module is the seeded input generator ``paper_2501_07942_amd.workload``, whose
outputs (specifications, truths, measurements) both sides consume.

Contents
  tt       naive TT toolkit: TT-SVD, rounding, Hadamard, sum/dot, convolution,
           Alg. 1 Einstein summation
  model    grid, prior, transition kernel, likelihood, moments
  filters  TT point-mass filter, dense point-mass filter, Kalman filter
  grad     log-likelihood gradients: replayed-rank differences, complex step
  adjoint  reverse-mode log-likelihood gradient at fixed ranks
  redesign grid re-design (Alg. 4) and TT interpolation onto a new grid
  cross    deterministic TT-cross (maxvol pivots) of point-wise functions
  linear   the filter for linear dynamics on re-designed grids (Alg. 3, 4)
"""
from . import tt, model, filters  # noqa: F401
