"""CPU FP64 oracle for the H2-compressed boundary double-layer operator.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised NumPy implementation of what the GPU library computes.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the library never does, and it shares no code with the library.

Contents, with the passage of Hertel, Christophersen & Boerm (arXiv:1811.05731)
each part follows:

* ``geometry``   -- mesh checks, triangle normals and areas, the solid angle
                    Psi(xi_i) and the diagonal D_ii = Psi_i/(4 pi) - 1
                    (Section 3, eq. matrix_definition; Section 2, eq. mainInt).
* ``lindholm``   -- closed-form integrals of a linear hat function against the
                    double-layer kernel over a flat triangle (the analytic forms
                    the paper cites in Section 3).
* ``quadrature`` -- a collapsed Gauss-Legendre triangle rule (used for the
                    column basis, exact for polynomials).
* ``dense``      -- the dense collocation matrix M = K + D (Section 3, eq. denseMat).
* ``h2``         -- the H2 approximation built by tensor Chebyshev
                    interpolation on a bounding-box cluster tree with
                    eta-admissibility, and its matrix-vector product (Section 4).
* ``energy``     -- the demagnetising energy of a uniformly magnetised body from
                    boundary data (Section 6.2).

Every function that has no independent pin states "parity unpinned" in its
docstring; all others are pinned by tests under ``tests/`` (marker ``not gpu``).
"""
