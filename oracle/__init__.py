"""CPU oracle for the adjusted DCT/DST transforms -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct FP64 / int64 implementation of
what the GPU path computes.  It exists to check the GPU path; only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it.  The
product path never imports, links or executes anything in here, and this
package shares no code with the HIP library (the seeded input generators live
in the separate ``synth`` module, which holds no transform arithmetic).

Modules
  transforms  exact orthonormal DCT-2/DCT-3/DST-2/DST-3/DST-7/DCT-8 matrices,
              reversal R and sign S (section 2.1, eq. 3)
  adjust      Givens-band and sub-block adjustments, adjusted transforms
              H = C B A (eq. 1), the weighted least-squares criterion (eq. 2),
              its gradient and the parameter fit
  fixed       integer tables and the fixed-point separable 2-D forward/inverse
  fp          FP64 separable 2-D forward/inverse (H_v X H_h^T)
  refit       the differentiable refit objective and its analytic gradient
  design      the adjustment design study of Fig. 1: sparsity objective over
              all orthogonal adjustments, its gradient and an Adam search
  stats       statistics of quantised coefficients: per-position level
              histograms, entropy, energy, distortion, coding gain (a proxy
              for the coding results of Tables 2 and 3)
  fit_params  script that fits and freezes the adjustment parameters

Pins (what fixes each function independently of itself) are listed in the
docstring of each module.  Functions without such a pin say "parity unpinned".
"""
