"""Seeded random factor sets for tests (an input generator: no transform arithmetic).

A random factor set has the structure of a butterfly factor set (complete
trees of depth L, ranks bounded by input rows, identity blocks, possibly empty
leaves) with random numbers as factor entries, so both the oracle and the GPU
path can be exercised on uneven shapes that a real factorization rarely makes.
"""
import numpy as np


def _partition(rng, total, parts, allow_empty=True):
    if parts == 1:
        return np.array([0, total], dtype=np.int64)
    if allow_empty:
        cuts = np.sort(rng.integers(0, total + 1, size=parts - 1))
    else:
        cuts = np.sort(rng.choice(np.arange(1, total), size=parts - 1, replace=False))
    return np.concatenate([[0], cuts, [total]]).astype(np.int64)


def random_factor_set(seed, n, m, L, max_rank=None, p_ident=0.25, allow_empty=True, identity_values=False,
                      p_id_form=0.0, ident_levels=0, arity=2, full_rank_leaves=False):
    """Random factor set.  identity_values=True makes every P the identity and
    every U_i a 0/1 selection so that the apply is an exact permutation.
    p_id_form: probability that a non-identity block with 0 < rank < inputs has
    the column-ID form P = [I T] Pi^T (r random columns hold e_1 .. e_r).
    ident_levels: levels 0 .. ident_levels-1 hold identity blocks only.
    arity: children per tree node (k-ary trees); a block's inputs are the k
    children of its frequency node under the parent of its space node.
    full_rank_leaves: a non-identity block of the last level takes rank
    min(inputs, leaf rows), as in factorizations whose leaves are smaller than
    their blocks' numerical rank (max_rank does not apply there)."""
    rng = np.random.default_rng(seed)
    nb = arity ** L
    perm = rng.permutation(n).astype(np.int32)
    xoff = _partition(rng, n, nb, allow_empty)
    koff = _partition(rng, m, nb, allow_empty)
    rank = np.zeros((L + 1, nb), np.int32)
    ident = np.zeros((L + 1, nb), np.uint8)
    P_off = np.full((L + 1, nb), -1, np.int64)
    chunks, off = [], 0
    for lvl in range(L + 1):
        nf = arity ** (L - lvl)
        for q in range(nb):
            if lvl == 0:
                rin = int(koff[q + 1] - koff[q])
            else:
                i, j = divmod(q, nf)
                q1 = (i // arity) * arity * nf + arity * j
                rin = int(rank[lvl - 1, q1:q1 + arity].sum())
            if identity_values or lvl < ident_levels or (rng.random() < p_ident and (max_rank is None or rin <= max_rank)):
                rank[lvl, q] = rin
                ident[lvl, q] = 1
                continue
            hi = rin if max_rank is None else min(rin, max_rank)
            r = int(rng.integers(0, hi + 1))
            if full_rank_leaves and lvl == L:
                r = min(rin, int(xoff[q + 1] - xoff[q]))
            rank[lvl, q] = r
            P_off[lvl, q] = off
            blk = rng.standard_normal((r, rin)) / np.sqrt(max(rin, 1))
            if p_id_form > 0 and 0 < r < rin and rng.random() < p_id_form:
                skel = rng.choice(rin, size=r, replace=False)
                blk[:, skel] = np.eye(r)
            chunks.append(blk.ravel())
            off += blk.size
    U_off = np.zeros(nb, np.int64)
    uch, uo = [], 0
    for i in range(nb):
        rows = int(xoff[i + 1] - xoff[i])
        r = int(rank[L, i])
        if identity_values:
            # with identity transfers y_L,i is all of c, so selecting column
            # xoff[i] + t makes f[perm_x[s]] = c[s] when m == n
            blk = np.zeros((rows, r))
            for t in range(rows):
                if xoff[i] + t < r:
                    blk[t, xoff[i] + t] = 1.0
        else:
            blk = rng.standard_normal((rows, r)) / np.sqrt(max(r, 1))
        U_off[i] = uo
        uch.append(blk.ravel())
        uo += blk.size
    return dict(n=np.int64(n), m=np.int64(m), L=np.int64(L), tol=np.float64(0.0), arity=np.int64(arity),
                perm_x=perm, xoff=xoff, koff=koff, rank=rank, ident=ident,
                P=np.concatenate(chunks) if chunks else np.zeros(0), P_off=P_off,
                U=np.concatenate(uch) if uch else np.zeros(0), U_off=U_off)
