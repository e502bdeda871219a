"""FP64 CPU oracle for preconditioned conjugate gradients on kernel matrices.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The library under ``paper_1602_06693_amd`` never imports it, and this package
imports nothing from the library: the two share no code.

Everything here is plain NumPy/SciPy in float64, written for a reader to check
against the paper ("Preconditioning Kernel Matrices", Cutajar, Osborne,
Cunningham and Filippone, ICML 2016) by eye:

  kernel    ARD-RBF Gram blocks and (K + lambda I) V             -- Eq. (1)
  direct    Cholesky solve and log-marginal likelihood         -- Section 2.1
  pcg       preconditioned CG, Algorithm 1 (textbook reading)  -- Section 2.1
  precond   Nystrom, FITC and Phi Phi^T + lambda I through the
            matrix inversion lemma                             -- Sections 3.1, 3.2
  gradient  exact gradient, Eq. (2), and its stochastic
            (Hutchinson) estimate                              -- Section 2.1
  mlp       the learned low-rank factor network, loss, manual
            backward and Adam (not in the paper; a low-rank
            factor of the Section 3.2 form learned from data)
  adagrad   ADAGRAD ascent on log-hyperparameters              -- Section 5
  rng       counter-based SplitMix64 Rademacher probes (the
            published generator, for the Section 2.1 estimate)

Parity status per function is stated in each module header.
"""
