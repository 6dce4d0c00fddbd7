"""Plain, slow, FP64 CPU oracle for the MLSDC-SH hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
package: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code, tables or constants with the HIP library.

Every function follows a passage of Hamon, Schreiber & Minion, "Multi-Level
Spectral Deferred Corrections Scheme for the Shallow Water Equations on the
Rotating Sphere" (arXiv:1805.07923), cited by section and equation label.
Where the paper defers to other work (spectral right-hand side, implicit
solver, LU-trick weights) the reading used is stated where it is implemented.

Modules
    quadrature  Gauss-Legendre latitudes, SDC nodes and matrices (mpmath)
    sht         normalised associated Legendre functions and the SH pair
    swe         shallow-water tendencies F_I, F_E and the implicit solve
    sdc         IMEX SDC sweep, two-level MLSDC step, collocation residual
    mixed       CPU emulation of reduced-precision Legendre contractions
"""
