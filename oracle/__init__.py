"""FP64 CPU oracle for the rapid Kriging predictor (Li, Fasshauer & Nychka).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the GPU library computes.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it;
the GPU library never calls it and shares no code with it.

Modules
-------
matern  -- the Matern covariance of eq. (Matern1), closed forms for nu in
           {1/2, 3/2, 5/2} and the general Bessel form.
exact   -- exact Kriging: GLS-free coefficients c = (K + tau^2 I)^{-1} y
           (eq. findc) and the dense prediction sum (eq. predictionh).
rapid   -- the paper's rapid approximation, Section 2.2, Steps 1-7, with the
           final convolution done as a direct sum (eq. ApproxPrediction2) and,
           for large grids, a test-only FP64 FFT variant.
grad    -- adjoint of the rapid predictor w.r.t. the data y and the lag image.
csim    -- circulant-embedding unconditional simulation and conditional
           simulation built on the rapid predictor (Section 1, steps (1)-(2)).
philox  -- the Philox-4x32-10 counter-based generator (Salmon et al. 2011)
           and Box-Muller normals, used for the conditional-simulation noise.

Every public function states the passage of the paper it follows.  Functions
whose output no independent pin constrains say "parity unpinned".
"""
