"""FP64 CPU oracle of the hybrid-mesh DG discretisation (test infrastructure).

This package is a plain, slow, deliberately unoptimised reference
implementation of the method of Chan, Wang, Modave, Remacle and Warburton,
"GPU-accelerated discontinuous Galerkin methods on hybrid meshes"
(arXiv:1507.02557).  It exists only to check the GPU library: the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product code path never does.  It shares no code with the HIP library.

Every reference operator is built from its definition by direct quadrature
(dense matrices, element loops or batched ``einsum``), in float64.

Modules
-------
quad     1D Jacobi polynomials, Gauss rules and Lagrange polynomials.
refel    the four reference elements (bases, nodes, cubature, faces, vertex maps).
mesh     face matching, canonical face frames, geometric factors.
solver   right-hand side, energy, stable time step, LSERK4 and MRAB3 steppers.
tables   constants printed in the paper (trace-inequality table).
"""
