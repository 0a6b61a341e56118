"""FP64 CPU oracle for subdomain CheFSI — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct NumPy implementation of what the HIP
library computes.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does.  It shares
no code with the HIP path (no kernels, headers, helpers or tables).  Both
sides receive the same arrays from the seeded workload generator.

Modules
  grid        FD weights, Laplacian, core mask and local->global map
  projectors  Kleinman-Bylander projector support, values, reverse CSR
  hamiltonian H = -1/2 Lap + V + V_nl applied to a block
  chefsi      Lanczos bounds, scaled Chebyshev filter, Rayleigh-Ritz,
              residuals, the CheFSI iteration
  density     Fermi-Dirac occupations, core density, interior weights,
              band / entropy energies, DOS
  bf16        bit-exact emulation of the FP32 -> (hi, lo) bfloat16 split
  mlp         features, FP64 MLP forward / backward / Adam

Parity status of every function is recorded in its module header; every
function is pinned by a closed form, an invariant or brute force in
tests/test_oracle_*.py unless it says "parity unpinned".
"""
from . import grid, projectors, hamiltonian, chefsi, density, bf16, mlp  # noqa: F401
