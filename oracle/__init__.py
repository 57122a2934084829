"""Reference (oracle) implementation of the entropy-stable modal DSEM residual.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, dense FP64 CPU
implementation written from the paper (Montoya & Zingg, "Efficient
entropy-stable discontinuous spectral-element methods using tensor-product
summation-by-parts operators on triangles and tetrahedra").  It exists to check
the HIP library; only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it.  The product path never calls into it.

Everything is computed from the dense definitions: dense operator matrices
D, Q, E, S, R, V, an all-pairs Hadamard sum for the volume term and a dense
facet-correction matrix, the weight-adjusted inverse written with M explicitly.
The vector-Jacobian product is torch autograd of this dense residual.

Modules:
  poly1d    -- orthonormal Jacobi polynomials, Gauss rules, Lagrange bases (Sec. 2.4)
  refelem   -- collapsed-coordinate tensor-product SBP operators and PKD basis (Sec. 3, 4.3)
  geometry  -- split meshes, orientation, isoparametric maps, metrics, connectivity (Sec. 4.1-4.2, 7.3)
  physics   -- Euler fluxes, entropy variables, EC two-point fluxes, interface flux (Sec. 7.1-7.2)
  residual  -- the flux-differencing residual and its hybridized equivalent (Sec. 4.4-4.6, 6)
"""
