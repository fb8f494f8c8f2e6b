"""Plain float64 CPU oracle of the exact Khatri-Rao leverage-score sampler
and of the sketched CP-ALS it feeds.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
benchmark's CPU baseline leg use it.  It shares no code with the GPU path:
it is written from the paper (Bharadwaj, Malik, Murray, Grigori, Buluc,
Demmel, "Fast Exact Leverage Score Sampling from Khatri-Rao Products with
Applications to Tensor Decomposition", NeurIPS 2023) with NumPy in float64.

Two levels:

* :mod:`oracle.definition` -- the plain definitions (materialised
  Khatri-Rao product, leverage scores by QR / SVD / the pseudo-inverse
  formula, the conditional distribution of Theorem 3.1).  Only for tiny
  inputs.
* :mod:`oracle.sampler` -- the method step by step (segment trees of
  partial Gram matrices, Algorithms 1-4 with the two-stage draw of
  Section 3.2), batched over independent samples.
* :mod:`oracle.cp` -- the sketched least-squares solve, CP-ALS
  (Algorithm 6 with the sampled solve of Section 3.3), the exact ALS step
  (sparse MTTKRP) and the fit.
* :mod:`oracle.sketch` -- the counter-based generator (Philox4x64-10) of
  in-kernel uniforms and of the range finder's Gaussian sketch.
* :mod:`oracle.accuracy` -- residual error and distortion of a sketch of a
  Khatri-Rao least-squares problem (Section 4.2, Appendix A.12).
"""
from . import definition, sampler, cp, sketch, accuracy  # noqa: F401
