"""libprcg: predict-and-recompute conjugate gradient solvers for one MI355X.

The solver itself is the HIP library ``libprcg.so`` (C ABI declared in
``include/prcg.h``); :mod:`paper_1905_01549_amd.prcg` is its thin ctypes
binding.  :mod:`paper_1905_01549_amd.problems` holds the seeded input
generators.  Importing the package does not load the GPU library.
"""
