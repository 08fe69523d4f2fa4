"""FP64 CPU oracle for the SIPG-DG diffusion solve and its displacement
covariance (test infrastructure only).

This package is the checker, not the product.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP path (no kernels, headers, helpers, tables or
constant generators); the only common input is the seeded generator in
``workloads``, which draws disk packings and start points and holds none of
the method's arithmetic.

What it computes, and where the paper defines it:

* ``mesh``      -- pixel grid split into two triangles per cell along the
                   main diagonal (section 3.3), cells whose centroid lies in a
                   disk removed (the axons of section 2.1 / 2.2), interior
                   faces between active triangles, connected components.
* ``poly``      -- exact integrals of bivariate polynomials over triangles and
                   along edges (the integrals of the weak form, eq. (7)).
* ``sipg``      -- modal (monomial) local basis and symmetric interior-penalty
                   assembly of M and A, replacing the paper's mixed form
                   (eq. (6)-(7)) and its fluxes (section 3.2) by the primal
                   form; zero flux on walls (eq. (3)).
* ``initial``   -- L2 projection of a Gaussian pulse, scaled to unit mass
                   (section 4.1: normalised densities).
* ``timeint``   -- SSP-RK3 with the Delta-landing schedule, and a Chebyshev
                   expansion of exp(-t M^-1 A) for long runs.
* ``moments``   -- exact zeroth, first and second moments about the start
                   point and the covariance readings (section 4.1).
* ``bounds``    -- largest eigenvalue of M^-1 A and the time-step rule.
* ``solve``     -- the whole pipeline for one geometry and many start points.
* ``surrogate`` -- FP64 forward/backward of the occupancy-image network.

Every function states the passage it follows.  Where the paper is silent
or garbled, the reading taken is named in the docstring.
"""
