"""FP64 CPU oracle for the joint initial-pressure / sound-speed reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, tables, constants or pre/post-processing); the only
thing both sides consume is the seeded input description (grid sizes, sensor
positions, phantoms), which holds none of the method's arithmetic.

Contents
--------
``kspace``   forward map of eq. (2) (k-space pseudospectral solution of eq. (1)),
             data misfit of eq. (4) and its exact discrete adjoint gradient
             (eqs. (5)-(9), taken as the gradient of the discrete objective).
``sensors``  point-sensor sampling operator of Sec. 2.2 and its transpose.
``prior``    Ornstein-Uhlenbeck prior terms of eq. (4) (Sec. 4.1.2): dense
             exponential correlation over the reconstruction pixels, Cholesky.
``optim``    bound projection (eq. (11)), L-BFGS two-loop recursion (Alg. 1),
             projected quasi-Newton step with backtracking (eq. (10)),
             multigrid prolongation (Sec. 3.1) and data time resampling
             (Sec. 4.1.2), relative error (eq. (12)).
``unet``     the learned fine-level start of the sound speed (replacing the
             Sec. 3.1 interpolation): 3x3 convolutions, ReLU, pooling,
             upsampling, masked squared loss and Adam, forward and backward
             written from their definitions.

Parity pins: every function is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants or brute force (see the module docstrings).  The full
multigrid reconstruction has no such pin: parity unpinned.
"""
