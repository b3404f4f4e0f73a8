"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU implementation (float64 / complex128)
of what the ParaDiag hot path computes, written from Gander & Palitta, "A new
ParaDiag time-parallel time integration method" (arXiv 2304.12597).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.
The product path (``paper_2304_12597_amd``) never does, and this package
shares no code with it: the only common dependency is the seeded input
generator ``paper_2304_12597_amd.workloads``, which holds none of the
method's arithmetic.

Modules
-------
spatial     sparse M and K for 1D / 2D problems (problem assembly)
allatonce   the all-at-once system: right-hand side G, residual, dense
            Kronecker matrix and its LU solve (O2), sequential backward-Euler
            stepping (O1; C code for 1D, banded Cholesky for 2D)
modal       exact per-sine-mode recurrences for sine-series data (O3)
paradiag    the objects of Algorithm 1 / 3, each from its own definition (the
            spectrum of G, blockwise shifted solves, the alpha-circulant
            solution U_1 by stepping, b, x = J^{-1} b), the capacitance
            matrix J_ell, explicit SMW with Kronecker products (O4), plain
            GMRES and the Galerkin projection of Section 3
dst         the orthonormal DST-I sine matrix
"""
