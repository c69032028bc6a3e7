"""Deflated multigrid multilevel Monte Carlo for tr(D^-1) of the 2D Wilson-Schwinger
operator, as a HIP library for gfx950 (Frommer & Ramirez-Hidalgo, "Deflated Multigrid
Multilevel Monte Carlo", Lattice 2022).

The package is split so that importing it loads nothing:

* ``inputs``  -- seeded synthetic inputs (gauge-link angles, workload table); no method
  arithmetic, shared by the tests, the benchmark and the CPU checker.
* ``dmlmc``   -- ctypes binding of the C-ABI library ``libdmlmc.so`` (argument
  marshalling only; every step of the computation runs in the HIP kernels).
* ``build``   -- compiles ``csrc/`` with hipcc for gfx950 into ``libdmlmc.so``.
"""
