"""CPU reference ("oracle") for the spectral-Galerkin hot path.  TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct numpy code, written from the paper's
definitions: naive O(N^2) discrete Fourier sums with exactly reduced phase
indices, direct evaluation of T_k at the Gauss-Chebyshev points, Galerkin
matrices assembled by Gauss quadrature, and dense LU with partial pivoting
(plus extended-precision iterative refinement) for every linear system.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library and
imports nothing from it.

Function-by-function pins live in tests/test_oracle_*.py.  Parity-unpinned
functions: none (every public function is pinned by at least one closed
form, invariant or brute-force check).
"""
from . import fourier, chebyshev, linalg, tensor, gl, fno, derivative, legendre  # noqa: F401
