"""Plain FP64 CPU oracle of the randomized functional sparse Tucker hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the C-ABI
library and its Python binding) never calls into it, and it shares no code with that
path: no kernels, headers, helpers or constant tables.

Every function here follows the paper (Rai, Kolla, Cannada, Gorodetsky, "Randomized
functional sparse Tucker tensor for compression and fast visualization of scientific
data", arXiv 1907.05884) step by step, in float64, without blocking or fusion beyond
batching over points:

* ``basis``       reference coordinates and the orthonormal Legendre basis (Sec. 2, Sec. 4.2)
* ``sampler``     SplitMix64 and the partial Fisher-Yates draw used for every random subset
* ``interp``      equispaced grid and inverse-distance interpolation onto it (Sec. 4.1)
* ``sthosvd``     sequentially truncated HOSVD at fixed ranks (Sec. 4.1)
* ``sparsefit``   sparse Legendre fit of each singular vector, OMP + leave-one-out (Sec. 3, 4.2)
* ``model``       the functional sparse Tucker model, eq. (1)-(2), and its storage count
* ``lsq``         core re-estimation by sampled least squares, eq. (6) and Algorithm 2
* ``reconstruct`` evaluation of eq. (1) at points of interest (Sec. 6)
* ``mlp``         FP64 reference of the small residual-corrector network
* ``pipeline``    Algorithm 1 followed by Algorithm 2

Parity pins (tests/test_oracle_*.py) tie each function to something other than itself:
closed forms, quadrature identities, exact recovery of planted structure, brute force.
"""
