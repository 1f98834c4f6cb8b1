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
modal forces (Sec. 3.1), the reverse-mode gradient of the time loop, and the
spectral loss, its hand-written gradient and the log-mel features (Sec. 4.3).

Every function is pinned by a CPU test against something other than itself
(textbook frequencies and decay rates, forces computed in physical space,
closed forms, brute force, complex-step and difference derivatives, direct
DFT sums).  A function without such a pin would say "parity unpinned" in its
docstring; none does.
"""
