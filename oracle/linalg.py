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


def householder_qr(A):
    """Dense Householder QR of a real m x n (m >= n) matrix in extended precision.

    Returns (V, R): V holds the n reflector vectors v_i (unit norm, zero
    above row i), R the n x n upper triangle, with A = Q R and
    Q^T = H_{n-1} ... H_0, H_i = I - 2 v_i v_i^T."""
    A = np.array(A, dtype=LD, copy=True)
    m, n = A.shape
    V = np.zeros((m, n), dtype=LD)
    for i in range(n):
        x = A[i:, i].copy()
        alpha = -np.sign(x[0]) * np.sqrt((x * x).sum()) if x[0] != 0 else -np.sqrt((x * x).sum())
        v = x
        v[0] = v[0] - alpha
        nv = np.sqrt((v * v).sum())
        if nv == 0:
            continue
        v = v / nv
        V[i:, i] = v
        A[i:, i:] -= 2 * np.outer(v, v @ A[i:, i:])
    return V, np.triu(A[:n, :n])


def lstsq_qr(V, R, b):
    """min ||A x - b||_2 for the factorisation returned by householder_qr;
    b is real (m or m x k) and is kept in extended precision throughout."""
    y = np.array(b, dtype=LD, copy=True)
    vec = y.ndim == 1
    if vec:
        y = y[:, None]
    m, n = V.shape
    for i in range(n):
        v = V[i:, i]
        y[i:] -= 2 * np.outer(v, v @ y[i:])
    z = y[:n]
    x = np.zeros_like(z)
    for i in range(n - 1, -1, -1):
        x[i] = (z[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x[:, 0] if vec else x
