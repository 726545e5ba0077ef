"""Column interpolative decomposition by pivoted QR (host, FP64).

The paper leaves the low-rank factorization free (SVD, QR, interpolative
decomposition, Sec. 2) and mentions interpolative decompositions for the
factorization step; the factor set here uses column IDs, A ~ A(:, J) P, because
then every column basis is a plain submatrix of Phi and only Phi entries are
ever evaluated.

Reading of the tolerance: the rank k is the number of diagonal entries of the
column-pivoted R with |R_ii| > tol * |R_11| (relative, per block).  A block that
keeps all its columns is flagged as the identity and stores nothing, with J in
concatenation order.
"""
import numpy as np
import scipy.linalg as sla


def column_id(A, tol):
    """Return (J, P, ident) with A ~ A[:, J] @ P.

    J: int64 indices into A's columns (skeleton, in pivot order unless ident);
    P: k x ncols float64 (None when ident); ident: True when k == ncols.
    """
    A = np.asarray(A, dtype=np.float64)
    rows, cols = A.shape
    if cols == 0:
        return np.zeros(0, np.int64), None, True
    if rows == 0:
        return np.zeros(0, np.int64), np.zeros((0, cols)), False
    B = A
    if rows > 2 * cols:
        # R of an unpivoted QR has the same column geometry as A; pivot on it.
        B = sla.qr(A, mode="r", check_finite=False)[0][:cols]
    R, piv = sla.qr(B, mode="r", pivoting=True, check_finite=False)
    d = np.abs(np.diag(R))
    if d.size == 0 or d[0] == 0.0:
        return np.zeros(0, np.int64), np.zeros((0, cols)), False
    k = int(np.count_nonzero(d > tol * d[0]))
    if k == cols:
        return np.arange(cols, dtype=np.int64), None, True
    R11 = R[:k, :k]
    R12 = R[:k, k:]
    T = sla.solve_triangular(R11, R12, lower=False, check_finite=False)
    P = np.zeros((k, cols), dtype=np.float64)
    P[:, piv[:k]] = np.eye(k)
    P[:, piv[k:]] = T
    return piv[:k].astype(np.int64), P, False
