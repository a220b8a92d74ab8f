"""Plain FP64 CPU oracle for the SU(3) adjoint-Laplacian hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, helpers, tables or constant generators); the
only thing both sides have in common is the seeded input generator module.

What it computes, each piece written from the paper's definitions (section 2,
Eq. 3 and Eq. 4; section 3, Eq. 5 and Eq. 6) in numpy float64, with the
readings listed in the design doc:

* ``su3``       su(3) basis T^a = lambda^a/2, components, structure constants.
* ``lattice``   periodic 4D lattice, x0 fastest; shifts x -> x +- mu.
* ``laplacian`` the adjoint covariant Laplacian Delta = -nabla^2_G (Eq. 3) as
                literal 3x3 matrix products, and its link derivative.
* ``chebyshev`` window indicator coefficients, Jackson damping, the three-term
                recursion, moments, the bandpass power spectrum (Eq. 4) and the
                vector filter.
* ``rational``  Eq. 6 quadratic terms -> real poles, the kappa-shape pole sets,
                per-shift plain CG, R(Delta) x and the kinetic energy (Eq. 5).
* ``force``     d K / d omega, the mass-term force of section 3, in commutator form.
* ``dense``     dense matrices for tiny lattices, for eigen-decomposition pins.

Every function is pinned by ``tests/test_oracle_*.py`` to something other than
itself (closed forms, invariants, brute force, dense eigen-decompositions).
"""
