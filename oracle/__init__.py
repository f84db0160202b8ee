"""CPU FP64 oracle for the element-wise DoGIP operator (test infrastructure only).

This package is the plain, slow, obviously correct reference that the HIP path
is checked against.  It is test infrastructure: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product library never imports, links or calls it, and it shares
no code with the product (it reads only the seeded inputs of ``workloads``).

Modules
-------
reference  reference simplex, Lagrange bases from exact Vandermonde solves,
           interpolation tensors B^ (Theorems 2 and 4) and W-basis weights.
fem        dof numbering, boundary, collapsed Gauss quadrature and the
           quadrature-assembled standard FEM matrices (eq. linsys_gp / linsys_se).
dogip      D construction (Theorems 2 and 4, Corollary for isotropic M) and the
           element loop of Algorithm 1.
solve      Jacobi-PCG and direct solves, Dirichlet handling.
adjoint    gradient of J = 0.5 |u - u_obs|^2 with respect to per-element
           log-coefficients.
counts     the memory and operation counts of Section 3 (CSR memory model,
           eq. memory_eff and eq. comp_eff).

Parity status of each function is stated in its module header.
"""
