"""FP64 CPU oracle for the sparse-covariance exact GP (test infrastructure).

This package is test infrastructure.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the HIP product
path never calls into it and shares no code with it.

It is a plain, slow, obviously-correct restatement of what the paper
defines, in float64 throughout:

* ``kernel``     - the support predicate, bump features, Wendland part and
                   the entries of K = C_core C_sparse + Delta (Sec. 2.1, Eq.
                   bumpFcn, sumOfBumps, C_sparse, compSupp; Sec. 3.1, Eq. Zcov:
                   Delta = a nugget plus optional per-point error variances),
                   as a dense brute-force matrix or a KD-tree-built sparse one.
* ``core``       - the core kernel C_core of C_y = C_core x C_sparse (Eq.
                   sparseCov): stationary Matern and the parametric
                   nonstationary kernel of Eq. PScov (Appendix B).
* ``likelihood`` - the Gaussian log-likelihood (Sec. 3.1 Eq. Zmarg, Sec. 3.3)
                   by dense Cholesky, by sparse LU, and by the split
                   K = A + F F^T with the determinant lemma / Woodbury identity
                   (A factored by SuperLU, or, for space-time data, by a dense
                   block Cholesky over the day blocks).
* ``minres``     - preconditioned MINRES (Paige and Saunders; Sec. 3.3).
* ``slq``        - stochastic Lanczos quadrature for log det (Sec. 3.3, the
                   Lanczos log-determinant) with Rademacher probes from a
                   counter-indexed SplitMix64 sequence.
* ``predict``    - the kriging mean m = C_{y,z} C_z^{-1} (z - W beta) and the
                   posterior variance diag C_{y|z} (Sec. 3.2).
* ``mcmc``       - the Bayesian training chain of Appendix C (adaptive
                   random-walk blocks, Bernoulli amplitudes, Gibbs step for pi).

Every function states the passage it follows.  Readings of passages that
are silent or ambiguous are listed in each module's docstring.

Parity status: every function here is pinned by the ``-m "not gpu"``
tests in ``tests/test_oracle_*.py`` (closed forms, invariants, brute force,
independent algorithms).  Absolute values printed in the paper do not
exist (it shows figures only), so no pin compares against a printed number.
"""
