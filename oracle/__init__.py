"""FP64 CPU oracle for modal time stepping of strings and plates.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything in this package.  The
product (the HIP library and its Python binding) never imports, links or runs
it, and this package imports nothing from the product.  The two share only the
seeded parameter draws in ``workloads``.

Everything here is plain, slow and written to be checked against the paper by
eye: modes and eigenvalues (Sec. 3, eigenvalue problem), the in-plane (Airy)
eigenpairs, the coupling tensor H by quadrature (coupling-coefficient
equations), the modal ODE coefficients, the Stormer-Verlet and
transfer-function recursions (Sec. 3.2), the tension-modulated and von Karman
modal forces (Sec. 3.1), and the reverse-mode gradient of the time loop.

Functions whose values no test pins independently are marked
"parity unpinned" in their docstrings.
"""
