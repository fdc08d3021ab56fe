"""FP64 CPU oracle for generalized Nystrom (GN) low-rank approximation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
use it.  It shares no code with the GPU path: the Philox counter-based generator,
the SRHT construction and every GN step are written here from their definitions,
independently of the HIP sources.

Paper: Y. Nakatsukasa, "Fast and stable randomized low-rank matrix
approximation" (arXiv:2009.11392).

Modules
  philox  -- Philox4x32-10 words, Box-Muller Gaussians, SRHT signs and samples.
  gn      -- the GN / stabilized GN pipeline (Algorithm 2.1 and Section 5.1),
             plus the comparison formulas used as pins (HMT, Tropp17, SVD
             epsilon-pseudoinverse, Nystrom, CUR) and the theorem bounds.
  exact   -- exact rational GN on tiny integer inputs (brute-force pin).
  grad    -- reverse mode of the approximant with the kept rank held fixed
             (dL/dA for L = <Gbar, A_hat>), pinned by finite differences and by
             torch's FP64 autograd through an independent forward.
  update  -- the Section 6 updates of the sketch products (resampling r -> r+dr,
             appended rows / columns, A -> A + E), pinned against fresh passes.
  stabilize -- the other Section 5.1.1 stabilizations (SVD epsilon-pseudoinverse,
             perturbations (a), (b), (c)) and the Section 5.1.2 power-method check
             of plain GN, pinned by closed forms on designed cores.

Parity status of each function is stated in its module header.
"""
