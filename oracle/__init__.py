"""FP64 CPU oracle for the spline geometric Maxwell leapfrog (schemes 2 and 1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (``paper_2302_04979_amd``) never imports it and shares no code with
it: the two sides meet only through the seeded input generators in
``workloads``.

The oracle is written plainly from the paper, in FP64 with NumPy/SciPy
primitives (matrix products, dense LU), with no blocking or fusion:

* ``splines``   - knot vectors (uniform or with given breakpoints), B-spline and
                  Curry-Schoenberg bases, Gauss rules,
                  1D incidence matrices, 1D pairing matrices G^ and M^
                  (Section 2.3; Section 4.1).
* ``geometry``  - maps F of the unit cube (identity, the deformed cube, the
                  quarter coax of Section 5 as a degree-2 NURBS map) and the
                  2-form and 1-form metric factors DF^T DF / det DF and
                  det DF (DF^T DF)^{-1} (Section 2.3 pullbacks).
* ``assembly``  - level 0, the plain definitions: 3D pairing matrices K1, K~1
                  by 3D quadrature, mass matrices by element loops, sparse curls
                  (Sections 2.4, 3.4).
* ``scheme``    - level 1, the structured method: per-axis Kronecker solves
                  (eq. (4.4), (4.5)), sum-factorised mass applies, the explicit
                  leapfrog of (3.10)-(3.13) in its (e, h) Petrov-Galerkin form,
                  energies, CFL, projections, point sources and probes;
                  symmetric triple-jump compositions of the leapfrog.
* ``scheme1``   - the first scheme (Section 3.3): 1-form mass matrices with
                  the covariant factor det DF (DF^T DF)^{-1}, conjugate-gradient
                  mass solves, the (e, h) leapfrog with the transposed pairings,
                  its energies and CFL.
* ``adjoint``   - the discrete adjoint of the scheme-2 leapfrog.
* ``tensor``    - the scheme with a degree, a knot vector and an element count
                  per direction (Section 4.1, per-direction factors of (4.2),
                  (4.3)), with level-0 counterparts of its pairings and masses.
* ``lifting``   - non-homogeneous tangential data for E (Section 3.5): the
                  whole primal spaces, the least-squares trace fit of the
                  lifting, the lifted leapfrog with separable-in-time data
                  (the coaxial cable's TEM mode, Section 5.1.2).

Every function is pinned by the CPU tests ``tests/test_oracle_*.py`` against
closed forms, invariants, dense level-0 assembly and brute force on tiny
meshes.
"""
