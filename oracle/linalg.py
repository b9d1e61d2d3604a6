"""Dense direct solves for the oracle (test infrastructure only).

Every Galerkin system is solved as a dense matrix: LU with partial pivoting
(LAPACK getrf/getrs through scipy, in float64), followed by iterative
refinement whose residual b - A x is formed in x87 extended precision
(numpy.longdouble) from an extended-precision copy of A.  The paper solves
these systems with O(N) special-purpose algorithms "if available" and a
general sparse solver otherwise (Sec. 3.2); a dense LU is the plain
definition of "solve A x = b".
"""
import numpy as np
import scipy.linalg as sla

LD = np.longdouble


def solve_refined(A, b, iters=3):
    """Solve A x = b for real A (n x n, longdouble or float64) and real or
    complex b (n or n x k).  Returns x as float64/complex128."""
    A_ld = np.asarray(A, dtype=LD)
    lu = sla.lu_factor(A_ld.astype(np.float64))
    b = np.asarray(b)
    if np.iscomplexobj(b):
        return solve_refined(A_ld, b.real, iters) + 1j * solve_refined(A_ld, b.imag, iters)
    b_ld = b.astype(LD)
    x = sla.lu_solve(lu, b.astype(np.float64)).astype(LD)
    for _ in range(iters):
        r = b_ld - A_ld @ x
        x = x + sla.lu_solve(lu, r.astype(np.float64)).astype(LD)
    return x.astype(np.float64)
