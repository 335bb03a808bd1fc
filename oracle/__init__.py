"""CPU FP64 oracle for the factorized Krylov methods for ``A X + X B = C1 C2^T``.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything in this package. The GPU library and its Python binding never
import it, and this package imports nothing from them: the two share no code; only the seeded
input generators in ``workloads`` serve both.

Modules
-------
``matrix_oriented``  Algorithm 2.1 (matrix-oriented CG) and Algorithm 2.2 (matrix-oriented
                     BiCGSTAB) on the full n x m iterate.
``factored``         Algorithm 4.1 (factorized CG), Algorithm 4.2 (factorized BiCGSTAB) and the
                     Lyapunov case (Section 4.3), with block Lanczos / block Arnoldi bases
                     satisfying eq. (3.8).
``direct``           Dense solves of the Kronecker form eq. (1.2) and Bartels-Stewart
                     (Section 1) for tiny sizes.
``residual``         ``||A X + X B - C1 C2^T||_F`` computed densely or from the factors, and the
                     sketch ``X @ Omega`` used to compare two factored solutions.

Every function is pinned by the CPU tests in ``tests/test_oracle_*.py``.
"""
