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

The same recursion holds for k-ary trees (Sec. 2: the construction generalizes
to k-ary trees, quadtrees in two dimensions; Sec. 5 analyses the quadtree in
space with a 4-ary tree on the eigenvalue range): a node's k children
c_1 .. c_k replace the pair, so y_lij = P_lij [y_{l-1,p,kj}; ...; y_{l-1,p,kj+k-1}]
with p the parent of tau_i.  A factor set states its k as "arity" (2 if absent).

Factor-set fields (plain dict of NumPy arrays, the factor-file schema):
  n, m, L        sizes; both trees are complete k-ary trees of depth L
  arity          k (optional, default 2); below, 2^ stands for k^
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


def arity(fs):
    """Children per tree node (k of a k-ary tree; 2 when the set does not say)."""
    return int(fs["arity"]) if "arity" in fs else 2


def _children(L, lvl, i, j, k=2):
    """Previous-level block ids of the k inputs of block (lvl, i, j).

    The parent p of space node i and the children k j, ..., k j + k - 1 of
    frequency node j (Sec. 2, local labels p, c1, c2 for k = 2), as space-major
    ids at level lvl - 1.
    """
    nf_prev = k ** (L - lvl + 1)
    p = i // k
    return [p * nf_prev + k * j + t for t in range(k)]


def _block_in_rows(fs, lvl, q):
    """Number of input rows of block q at level lvl."""
    L, k = int(fs["L"]), arity(fs)
    if lvl == 0:
        return int(fs["koff"][q + 1] - fs["koff"][q])
    i, j = divmod(q, k ** (L - lvl))
    return int(sum(fs["rank"][lvl - 1][c] for c in _children(L, lvl, i, j, k)))


def _P(fs, lvl, q):
    r = int(fs["rank"][lvl][q])
    k = _block_in_rows(fs, lvl, q)
    if fs["ident"][lvl][q]:
        return np.eye(r, k)
    o = int(fs["P_off"][lvl][q])
    return np.asarray(fs["P"][o:o + r * k], dtype=np.float64).reshape(r, k)


def _U(fs, i):
    L = int(fs["L"])  # leaf i of the space tree
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
    L, n, k = int(fs["L"]), int(fs["n"]), arity(fs)
    nb = k ** L
    koff, xoff, perm = fs["koff"], fs["xoff"], fs["perm_x"]
    # level 0: one block per frequency leaf
    y = [_P(fs, 0, j) @ c[koff[j]:koff[j + 1]] for j in range(nb)]
    for lvl in range(1, L + 1):
        nf = k ** (L - lvl)
        ynew = []
        for i in range(k ** lvl):
            for j in range(nf):
                x = np.vstack([y[q] for q in _children(L, lvl, i, j, k)])
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
    L, m, k = int(fs["L"]), int(fs["m"]), arity(fs)
    nb = k ** L
    b = f.shape[1]
    koff, xoff, perm = fs["koff"], fs["xoff"], fs["perm_x"]
    z = [_U(fs, i).T @ f[perm[xoff[i]:xoff[i + 1]]] for i in range(nb)]
    for lvl in range(L, 0, -1):
        nf = k ** (L - lvl)
        zprev = [np.zeros((int(fs["rank"][lvl - 1][q]), b)) for q in range(nb)]
        for i in range(k ** lvl):
            for j in range(nf):
                w = _P(fs, lvl, i * nf + j).T @ z[i * nf + j]
                s = 0
                for q in _children(L, lvl, i, j, k):   # split the stacked rows back to the children
                    r = zprev[q].shape[0]
                    zprev[q] += w[s:s + r]
                    s += r
        z = zprev
    g = np.zeros((m, b), dtype=np.float64)
    for j in range(nb):
        g[koff[j]:koff[j + 1]] = _P(fs, 0, j).T @ z[j]
    return g[:, 0] if squeeze else g


def stored_entries(fs):
    """F: number of stored factor entries (identity blocks store nothing)."""
    L, k = int(fs["L"]), arity(fs)
    tot = 0
    for lvl in range(L + 1):
        for q in range(k ** L):
            if not fs["ident"][lvl][q]:
                tot += int(fs["rank"][lvl][q]) * _block_in_rows(fs, lvl, q)
    for i in range(k ** L):
        tot += int(fs["xoff"][i + 1] - fs["xoff"][i]) * int(fs["rank"][L][i])
    return tot
