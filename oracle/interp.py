"""Column interpolative decomposition of one block (oracle, test infrastructure).

The butterfly factorization needs a low-rank factorization of every block and
leaves its kind open (Sec. 2, Alg. "Butterfly factorization": SVD, QR or an
interpolative decomposition all serve).  The factor sets here use column IDs
from a column-pivoted QR with Businger-Golub pivoting (at each step the
remaining column whose part orthogonal to the chosen columns is longest):

  A Pi = Q [R11 R12; 0 R22],   k = #{i : |R_ii| > tol |R_11|},
  J = Pi(1..k),   P(:, Pi) = [I  R11^-1 R12],   so A ~ A(:, J) P.

Reading of the tolerance: relative to the first pivot, per block (the paper
states a relative ID tolerance and nothing finer).  A block that keeps all its
columns is the identity, with J in column order and no P; an empty or all-zero
block keeps none.  The pivoted QR is the library's (LAPACK's dgeqp3 through
SciPy), a step the definition names; the rest is written out.

Parity status: pinned in tests/test_oracle_interp.py (exact-rank blocks, the
least-squares meaning of R11^-1 R12, the residual bound sqrt(K-k) tol |A|, and
the pivot order against a pure-Python greedy Gram-Schmidt selection).
"""
import numpy as np
import scipy.linalg as sla


def column_id(A, tol):
    """Return (J, P, ident) with A ~ A[:, J] @ P.

    J: int64 column indices (pivot order, or 0..K-1 when ident);
    P: float64 k x K (None when ident); ident: True when k == K.
    """
    A = np.asarray(A, dtype=np.float64)
    M, K = A.shape
    if K == 0:
        return np.zeros(0, np.int64), None, True
    if M == 0:
        return np.zeros(0, np.int64), np.zeros((0, K)), False
    R, piv = sla.qr(A, mode="r", pivoting=True, check_finite=False)
    d = np.abs(np.diag(R))
    if d[0] == 0.0:
        return np.zeros(0, np.int64), np.zeros((0, K)), False
    k = int(np.count_nonzero(d > tol * d[0]))
    if k == K:
        return np.arange(K, dtype=np.int64), None, True
    T = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False, check_finite=False)
    P = np.zeros((k, K))
    P[:, piv[:k]] = np.eye(k)
    P[:, piv[k:]] = T
    return piv[:k].astype(np.int64), P, False
