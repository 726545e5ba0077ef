"""The butterfly factor set multiplied out as a product of block-sparse matrices.

The paper remarks that the butterfly factorization can equally be written as a
product of O(log m) sparse matrices, one per level, each holding that level's
transfer blocks (Sec. 2, Remark after Alg. "Butterfly factorization").  This
module assembles those matrices densely (tiny sizes only) and multiplies them:

  Phi~ = B_final B_L ... B_1 B_0,

where B_0 maps coefficients to the stacked level-0 vector, B_l maps the stacked
level-(l-1) vector to the stacked level-l vector, and B_final scatters the leaf
bases U_i into the point rows.  It is a second, independent formulation of what
the butterfly apply computes, used to pin the recursive apply.  Factor sets of k-ary trees ("arity" k, 2 if absent) are
assembled the same way, each block reading its k children.
"""
import numpy as np


def _offsets(ranks):
    return np.concatenate([[0], np.cumsum(np.asarray(ranks, dtype=np.int64))])


def dense_operator(fs):
    """The explicit n x m matrix Phi~ represented by the factor set (tiny sizes)."""
    L, n, m = int(fs["L"]), int(fs["n"]), int(fs["m"])
    k = int(fs["arity"]) if "arity" in fs else 2
    nb = k ** L
    rank = np.asarray(fs["rank"])
    ident = np.asarray(fs["ident"])
    koff = np.asarray(fs["koff"])
    mats = []
    # B_0: block diagonal over frequency leaves
    off0 = _offsets(rank[0])
    B = np.zeros((off0[-1], m))
    for j in range(nb):
        r, k0, k1 = rank[0][j], koff[j], koff[j + 1]
        if ident[0][j]:
            blk = np.eye(r, k1 - k0)
        else:
            o = fs["P_off"][0][j]
            blk = np.asarray(fs["P"][o:o + r * (k1 - k0)]).reshape(r, k1 - k0)
        B[off0[j]:off0[j] + r, k0:k1] = blk
    mats.append(B)
    prev_off = off0
    for lvl in range(1, L + 1):
        nf = k ** (L - lvl)
        cur_off = _offsets(rank[lvl])
        B = np.zeros((cur_off[-1], prev_off[-1]))
        for i in range(k ** lvl):
            for j in range(nf):
                q = i * nf + j
                c1 = (i // k) * (k * nf) + k * j   # first child block at the previous level
                cols = []
                for c in range(c1, c1 + k):
                    cols += list(range(prev_off[c], prev_off[c + 1]))
                r = rank[lvl][q]
                if ident[lvl][q]:
                    blk = np.eye(r, len(cols))
                else:
                    o = fs["P_off"][lvl][q]
                    blk = np.asarray(fs["P"][o:o + r * len(cols)]).reshape(r, len(cols))
                B[cur_off[q]:cur_off[q] + r][:, cols] = blk
        mats.append(B)
        prev_off = cur_off
    # final: leaf bases scattered to the original point rows
    Bf = np.zeros((n, prev_off[-1]))
    xoff, perm = np.asarray(fs["xoff"]), np.asarray(fs["perm_x"])
    for i in range(nb):
        rows = perm[xoff[i]:xoff[i + 1]]
        r = rank[L][i]
        o = fs["U_off"][i]
        blk = np.asarray(fs["U"][o:o + len(rows) * r]).reshape(len(rows), r)
        Bf[np.ix_(rows, np.arange(prev_off[i], prev_off[i] + r))] = blk
    out = Bf
    for B in reversed(mats):
        out = out @ B
    return out
