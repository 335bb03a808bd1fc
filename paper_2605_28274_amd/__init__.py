"""MI355X (gfx950) factorized Krylov solver for A X + X B = C1 C2^T with a low-rank right-hand side.

The solver is the HIP library ``libsylv.so`` behind the C ABI in ``include/sylv.h``;
:mod:`paper_2605_28274_amd.sylv` is its thin Python binding (importing it raises if the library
has not been built).
"""
