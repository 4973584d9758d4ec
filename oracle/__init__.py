"""Plain FP64 CPU oracle for the two-level Schwarz FDFD solver (test infrastructure).

This package is the checker, not the product: only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the HIP path.  Everything is written in complex128 with NumPy/SciPy,
one step at a time, in the order the paper states the method:

* ``fdfd``      -- E_z FDFD operator with UPML stretching (Eq. 1, Methods
                   "Training data generation" UPML equations), direct solve.
* ``partition`` -- rectangular overlapping partition, local Robin matrices
                   (Eq. 2), Robin traces, one-level restricted additive Schwarz
                   and the stationary Robin-data sweep (Algorithm 3 loop).
* ``coarse``    -- pseudo-plane-wave coarse space and the two-level
                   correction (Sec. 2.2 coarse space paragraphs, Algorithm 3
                   pre-compute block, coarse normal equations).
* ``fgmres``    -- flexible GMRES (Algorithm 1 recurrence), used both as the
                   outer Krylov method and as the inner NN-preconditioned
                   subdomain solver.
* ``fno``       -- NumPy forward pass of the subdomain Fourier neural
                   operator (Fig. 2 architecture).

Pins: every function is checked in ``tests/test_oracle_*.py`` against closed
forms, invariants and independent library routines.  ``fno.fno_forward``'s
trained-weight behaviour (how good a preconditioner it is) is "parity
unpinned": the paper prints no values for it.
"""
