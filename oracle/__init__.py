"""CPU FP64 oracle for the interpolation-and-lookup multiscale stiffness assembly
(Hirschler, Antolin, Buffa: Fast and multiscale formation of isogeometric matrices
of microstructured geometric models).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library;
the two meet only through the seeded input generators in ``workloads``.

Every routine is a plain, slow, direct transcription of the definitions in the
paper (section / equation cited in each docstring), in float64, using NumPy /
SciPy primitives (matmul, solve, eigh) as single steps.

Parity status of each part (what pins it, see tests/test_oracle_*.py):
  basis      -- pinned against scipy.interpolate.BSpline and Bernstein identities
  geometry   -- pinned by affine reproduction and closed-form maps
  macro_field-- paper's curvilinear route (eq. 79-97) pinned against the closed
                form of the cube (eq. 98-99) and an independent Cartesian form
  projection -- pinned by polynomial reproduction (Section 3.1.2)
  tables     -- pinned by partition-of-unity row sums, Bernstein sum and degree
                elevation identities, and separable 1-D integrals (identity tile)
  assembly   -- pinned by K^pi == K (standard Gauss) for affine macro maps,
                rigid-body modes, patch test and definiteness
  standard   -- independent B-matrix assembly; pinned by the same invariants
  adjoint    -- pinned by central finite differences of u^T K u and of the
                compliance with a direct solve
  learned    -- POD pinned by orthonormality and the Eckart-Young identity; MLP
                backward pinned by finite differences
"""
