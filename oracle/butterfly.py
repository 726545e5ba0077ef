"""O2: CPU FP64 apply of a stored row-wise butterfly factor set (oracle, test infrastructure).

The factor set is the return value of the butterfly factorization (Sec. 2,
Alg. "Butterfly factorization"): a basis block per frequency leaf at level 0,
a transfer block per (space node, frequency node) pair at levels 1..L, and a
dense column basis per space leaf.  With column interpolative decompositions
(the paper allows any low-rank factorization, Sec. 2) the blocks read as:

  level 0:      Phi(:, nu_j)          ~ Phi(:, J_0j) P_0j
  level l>=1:   Phi(tau_i, [J_{l-1,p,2j}, J_{l-1,p,2j+1}]) ~ Phi(tau_i, J_lij) P_lij,
                p = parent of tau_i (Sec. 2, the recursion for Phi(tau, nu) in
                terms of the previous level's factors)
  final:        U_i = Phi(tau_i, J_Li0)

so the synthesis is y_0j = P_0j c[nu_j], then y_lij = P_lij [y_{l-1,p,2j}; y_{l-1,p,2j+1}]
for l = 1..L, then f[tau_i] = U_i y_Li0.  The paper's prose lists the apply
steps in the adjoint's order; this follows the algebra of the recursion.  The
analysis is the exact transpose of those steps.

Factor-set fields (plain dict of NumPy arrays, the factor-file schema):
  n, m, L        sizes; both trees are complete binary trees of depth L
  perm_x  [n]    tree position -> original point index
  xoff    [2^L+1] space-leaf offsets into tree positions
  koff    [2^L+1] frequency-leaf offsets into the eigenvalue-sorted columns
  rank    [L+1, 2^L] r_{l,q}, block q = i * 2^(L-l) + j (space node i at depth l,
                 frequency node j at depth L-l)
  ident   [L+1, 2^L] 1 where the block's P is the identity (not stored)
  P, P_off       row-major r_lq x r_in blocks, offset -1 for identity blocks
  U, U_off       row-major |tau_i| x r_{L,i} blocks
"""
import numpy as np


def _children(L, lvl, i, j):
    """Previous-level block ids of the two inputs of block (lvl, i, j).

    The parent p of space node i and the children 2j, 2j+1 of frequency node j
    (Sec. 2, local labels p, c1, c2), as space-major ids at level lvl - 1.
    """
    nf_prev = 1 << (L - lvl + 1)
    p = i >> 1
    return p * nf_prev + 2 * j, p * nf_prev + 2 * j + 1


def _block_in_rows(fs, lvl, q):
    """Number of input rows of block q at level lvl."""
    L = int(fs["L"])
    if lvl == 0:
        return int(fs["koff"][q + 1] - fs["koff"][q])
    i, j = divmod(q, 1 << (L - lvl))
    q1, q2 = _children(L, lvl, i, j)
    return int(fs["rank"][lvl - 1][q1] + fs["rank"][lvl - 1][q2])


def _P(fs, lvl, q):
    r = int(fs["rank"][lvl][q])
    k = _block_in_rows(fs, lvl, q)
    if fs["ident"][lvl][q]:
        return np.eye(r, k)
    o = int(fs["P_off"][lvl][q])
    return np.asarray(fs["P"][o:o + r * k], dtype=np.float64).reshape(r, k)


def _U(fs, i):
    L = int(fs["L"])
    rows = int(fs["xoff"][i + 1] - fs["xoff"][i])
    r = int(fs["rank"][L][i])
    o = int(fs["U_off"][i])
    return np.asarray(fs["U"][o:o + rows * r], dtype=np.float64).reshape(rows, r)


def apply(fs, c):
    """f = Phi~ c.  c: (m,) or (m, b) float64.  Returns (n,) or (n, b)."""
    c = np.asarray(c, dtype=np.float64)
    squeeze = c.ndim == 1
    if squeeze:
        c = c[:, None]
    L, n = int(fs["L"]), int(fs["n"])
    nb = 1 << L
    koff, xoff, perm = fs["koff"], fs["xoff"], fs["perm_x"]
    # level 0: one block per frequency leaf
    y = [_P(fs, 0, j) @ c[koff[j]:koff[j + 1]] for j in range(nb)]
    for lvl in range(1, L + 1):
        nf = 1 << (L - lvl)
        ynew = []
        for i in range(1 << lvl):
            for j in range(nf):
                q1, q2 = _children(L, lvl, i, j)
                x = np.vstack([y[q1], y[q2]])
                ynew.append(_P(fs, lvl, i * nf + j) @ x)
        y = ynew
    f = np.zeros((n, c.shape[1]), dtype=np.float64)
    for i in range(nb):
        f[perm[xoff[i]:xoff[i + 1]]] = _U(fs, i) @ y[i]
    return f[:, 0] if squeeze else f


def apply_transpose(fs, f):
    """g = Phi~^T f.  f: (n,) or (n, b) float64.  Returns (m,) or (m, b)."""
    f = np.asarray(f, dtype=np.float64)
    squeeze = f.ndim == 1
    if squeeze:
        f = f[:, None]
    L, m = int(fs["L"]), int(fs["m"])
    nb = 1 << L
    b = f.shape[1]
    koff, xoff, perm = fs["koff"], fs["xoff"], fs["perm_x"]
    z = [_U(fs, i).T @ f[perm[xoff[i]:xoff[i + 1]]] for i in range(nb)]
    for lvl in range(L, 0, -1):
        nf = 1 << (L - lvl)
        zprev = [np.zeros((int(fs["rank"][lvl - 1][q]), b)) for q in range(nb)]
        for i in range(1 << lvl):
            for j in range(nf):
                q1, q2 = _children(L, lvl, i, j)
                w = _P(fs, lvl, i * nf + j).T @ z[i * nf + j]
                r1 = zprev[q1].shape[0]
                zprev[q1] += w[:r1]
                zprev[q2] += w[r1:]
        z = zprev
    g = np.zeros((m, b), dtype=np.float64)
    for j in range(nb):
        g[koff[j]:koff[j + 1]] = _P(fs, 0, j).T @ z[j]
    return g[:, 0] if squeeze else g


def stored_entries(fs):
    """F: number of stored factor entries (identity blocks store nothing)."""
    L = int(fs["L"])
    tot = 0
    for lvl in range(L + 1):
        for q in range(1 << L):
            if not fs["ident"][lvl][q]:
                tot += int(fs["rank"][lvl][q]) * _block_in_rows(fs, lvl, q)
    for i in range(1 << L):
        tot += int(fs["xoff"][i + 1] - fs["xoff"][i]) * int(fs["rank"][L][i])
    return tot
