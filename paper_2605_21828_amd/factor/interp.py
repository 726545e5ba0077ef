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

Every diagonal entry of any QR factor of A satisfies |R_ii| >= sigma_min(A), and
|R_11| <= sigma_max(A).  So when sigma_min / sigma_max is well above tol the
pivoted QR would keep every column, and the block is the identity without it.
The ratio is bounded from below through the Gram matrix A^T A (a matrix product,
much faster than a pivoted QR of a tall block), allowing for the rounding of the
product and of its eigenvalues; only blocks that pass with a wide margin take
this shortcut, so it never changes a result.  It is tried on tall blocks only
(rows >= 4 cols), where the QR it saves costs far more than the test.
"""
import numpy as np
import scipy.linalg as sla


def surely_full_rank(A, tol):
    """True when sigma_min(A) > 10 tol sigma_max(A) is certain from the
    eigenvalues of the computed Gram matrix: each eigenvalue is within
    (rows + 2) cols eps lambda_max of the exact one (the product's rounding, at
    most rows eps |A|^T |A| elementwise with || |A|^T |A| || <= cols lambda_max, plus
    the symmetric eigensolver's backward error)."""
    rows, cols = A.shape
    if rows < cols or cols == 0:
        return False
    w = np.linalg.eigvalsh(A.T @ A)
    if not w[-1] > 0.0:
        return False
    slack = 1.01 * (rows + 2) * cols * np.finfo(np.float64).eps * w[-1]
    return w[0] - slack > (10.0 * tol) ** 2 * (w[-1] + slack)


def column_id(A, tol, gram_check=True):
    """Return (J, P, ident) with A ~ A[:, J] @ P.

    J: int64 indices into A's columns (skeleton, in pivot order unless ident);
    P: k x ncols float64 (None when ident); ident: True when k == ncols.
    gram_check=False always runs the pivoted QR (same result, slower).
    """
    A = np.asarray(A, dtype=np.float64)
    rows, cols = A.shape
    if cols == 0:
        return np.zeros(0, np.int64), None, True
    if rows == 0:
        return np.zeros(0, np.int64), np.zeros((0, cols)), False
    if gram_check and rows >= 4 * cols and surely_full_rank(A, tol):
        return np.arange(cols, dtype=np.int64), None, True
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
