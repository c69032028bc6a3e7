"""CPU FP64 checker for deflated multigrid multilevel Monte Carlo (tr(D^-1), 2D Wilson-Schwinger).

TEST INFRASTRUCTURE ONLY.  Nothing in the library calls, imports or links this package;
only the test suite, the smoke check and the benchmark's CPU-baseline leg use it.

It is a plain, slow, obviously-correct restatement of what the method computes, written
from the paper (Frommer & Ramirez-Hidalgo, Lattice 2022) and the readings listed in the
design notes, with numpy/scipy as the only primitives (sparse matrices, LU, dense eigh):

* ``wilson``     -- the operator D, Gamma5, free-field closed forms      (Sec. 2, Sec. 3.1)
* ``noise``      -- SplitMix64 counter hash, Z2 sample noise, Z4 start vectors (Sec. 2, eq. 2)
* ``multigrid``  -- test vectors, aggregation interpolator P, Galerkin R D P, Gamma5 relations
                    (Sec. 3.1, eq. 8; Sec. 4.2, eq. 14)
* ``deflation``  -- exact deflation from the eigenpairs of Gamma5 D           (eqs. 4-7)
* ``mlmc``       -- sample values, telescoping sum, estimator, stopping rule  (eqs. 1, 2, 5, 11)
* ``mass``       -- the bare-mass rule sigma_min(D) ~ 1e-2                    (workload recipe)

Every function is pinned by the tests in ``tests/test_oracle_*.py`` against closed forms,
invariants, brute force or library routines, except the test-vector setup procedure,
which the paper does not define (it cites its construction): that piece is
"parity unpinned" beyond the invariants P^H P = I and the Gamma5 relations.
"""
