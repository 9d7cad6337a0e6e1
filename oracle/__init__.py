"""CPU FP64 oracle for the CROM latent step (test infrastructure only).

This package is a plain, slow, obviously correct NumPy implementation of what
the HIP library computes.  It exists to check the GPU path: only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.
The product path (the C-ABI library and its Python binding) never imports,
calls or links anything here, and this package imports nothing from the
product path.  The two share only the seeded input generators in
``workloads``, which hold none of the method's arithmetic.

Modules
-------
mlp        decoder g(x, q) and its exact derivatives by forward-mode chain rule
heat       heat-equation update at samples, FD full-order solvers, closed forms
inversion  Cholesky, Gauss-Newton with backtracking, linearised inversion
step       the three-stage latent step and rollouts
elastic    neo-Hookean stress, its derivative and the explicit elastic update
fem        corotated stress, tetrahedron forces on the samples' one-ring, FE update
train      encoder/decoder reverse-mode gradients, MSE loss, Adam, the
           standardization of the training data and its fold into the networks
pod        proper orthogonal decomposition baseline (linear basis, same step)
sampling   robust greedy selection of the integration samples

Parity status of each function is stated in its docstring; every function
here is pinned by tests under ``tests/`` that do not call the GPU.
"""
