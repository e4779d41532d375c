"""FP64 CPU oracle for the CONCORD / PseudoNet proximal-gradient iteration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
GPU product path never calls it and shares no code with it.

Contents
--------
``concord``   the iteration itself (paper Section 2, Algorithm 1; Section 3,
              Algorithms 2 (Cov) and 3 (Obs)), plain NumPy/SciPy in FP64.
``brute``     exact minimiser for p <= 3 by sign-pattern enumeration and Newton.
``checks``    closed forms, KKT residuals and the lambda1_max bound.

Readings of the paper that the oracle takes where the text is silent, garbled
or at odds with itself (objective scaling, the unthresholded diagonal, where
1/n sits in Obs, the stopping rule, the domain guard, ties at the threshold)
are stated in the docstrings where they apply.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(closed forms, brute force, KKT, Cov/Obs identity, finite differences,
metamorphic scaling/permutation).  Per-step values at large p have no pin
other than these properties, since the paper prints no worked example.
"""
from .concord import (  # noqa: F401
    soft_threshold, prox_step, sample_covariance, smooth_objective, gradient,
    penalty, test_difference_terms, solve, SolveResult, IterRecord,
    smooth_value_and_grads, smooth_value_and_sampled_grads,
)
