"""FP64 CPU oracle for the DELIMIT layers -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy float64 implementations of what the
Signal2SH, SH2Signal and local spherical convolution (LSC) layers compute,
following Koppers & Merhof, "DELIMIT PyTorch - An extension for Deep
Learning in Diffusion Imaging" (arXiv:1808.01517):

* ``oracle.sh``    -- real even-order SH basis, shell grouping, the
                      Laplace-Beltrami regularised fit (Signal2SH, Sec. 2.2)
                      and evaluation (SH2Signal, Sec. 2.2), with adjoints.
* ``oracle.lsc``   -- cyclic-kernel geometry, neighbourhood resampling by SH
                      interpolation, the m x (n+1) neighbourhood matrix, the
                      row-wise kernel dot and the refit (Sec. 2.3, incl. the
                      multi-b-value extension), with adjoints.
* ``oracle.stack`` -- layer stacks, the q-space MSE loss and full
                      forward + backward passes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP product path never imports,
links or executes it, and this package imports nothing from the product.

Pins (tests/test_oracle_*.py, run with ``-m "not gpu"``) tie every function
to something other than itself: quadrature orthonormality, the addition
theorem, textbook values, scipy's complex harmonics, exact recovery,
closed-form regularisation bias, Funk-Hecke filtering, permutation
equivariance, brute-force loops, adjoint identities and finite differences.
Parity unpinned: anisotropic LSC kernels beyond the brute-force loops and
permutation test (the paper fixes no frame convention for the kernel
points), and the trained learned-form network (stochastic).
"""
