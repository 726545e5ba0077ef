"""The butterfly factorization of a dense Phi with column IDs (oracle, test infrastructure).

Follows Alg. "Butterfly factorization" of Sec. 2 in the order its levels are
defined, on an explicit dense matrix (tiny sizes only):

  level 0:   for every frequency leaf nu_j, a column ID of Phi(:, nu_j);
  level l:   for every space node tau_i at depth l and frequency node nu_j at
             depth L - l, a column ID of [U_{p c_1}(tau_i, :) ... U_{p c_k}(tau_i, :)],
             p the parent of tau_i and c_1 .. c_k the children of nu_j.  With
             column IDs U_{p c}(tau, :) is Phi(tau, J_{p c}), so the block is
             Phi(tau_i, [J_{p c_1}, ..., J_{p c_k}]);
  final:     U_i = Phi(tau_i, J_{L,i}) for every space leaf.

Sec. 4's streaming variant visits the frequency nodes in post-order instead;
every block depends only on the blocks of its children, so the two orders
compute the same blocks, and this one keeps the levels apart for reading.

The trees are inputs (perm_x, xoff, koff as in the factor-set schema); the
factor set returned has the schema `oracle.butterfly` reads, with block
q = i * k^(L-l) + j at level l.

Parity status: pinned in tests/test_oracle_interp.py (the factor set applied by
O2 reproduces Phi within the bound the per-block IDs allow, exactly for a
matrix of exact low rank, and each block equals the column ID of its block of
Phi).
"""
import numpy as np

from .interp import column_id


def butterfly_factorization(Phi, perm_x, xoff, koff, L, tol, arity=2):
    Phi = np.asarray(Phi, dtype=np.float64)
    n, m = Phi.shape
    k = int(arity)
    nb = k ** L
    perm_x = np.asarray(perm_x)
    rank = np.zeros((L + 1, nb), np.int32)
    ident = np.zeros((L + 1, nb), np.uint8)
    P_off = np.full((L + 1, nb), -1, np.int64)
    P_parts, off = [], 0
    J = [None] * nb
    for lvl in range(L + 1):
        nf = k ** (L - lvl)            # frequency nodes at depth L - lvl
        w = k ** (L - lvl)             # space leaves under a space node at depth lvl
        Jnew = [None] * nb
        for i in range(k ** lvl):
            rows = perm_x[xoff[i * w]:xoff[(i + 1) * w]]
            for j in range(nf):
                q = i * nf + j
                if lvl == 0:
                    cols = np.arange(koff[j], koff[j + 1])
                else:
                    p = i // k
                    first = p * (k * nf) + k * j     # block (p, c_1) at level lvl - 1
                    cols = np.concatenate([J[first + t] for t in range(k)])
                Jl, P, idf = column_id(Phi[np.ix_(rows, cols)], tol)
                Jnew[q] = cols[Jl]
                rank[lvl, q] = len(Jl)
                ident[lvl, q] = 1 if idf else 0
                if not idf:
                    P_off[lvl, q] = off
                    P_parts.append(P.ravel())
                    off += P.size
        J = Jnew
    U_off = np.zeros(nb, np.int64)
    U_parts, uo = [], 0
    for i in range(nb):
        rows = perm_x[xoff[i]:xoff[i + 1]]
        U = Phi[np.ix_(rows, J[i])]
        U_off[i] = uo
        U_parts.append(U.ravel())
        uo += U.size
    cat = lambda parts: np.concatenate(parts) if parts else np.zeros(0)
    return dict(n=np.int64(n), m=np.int64(m), L=np.int64(L), tol=np.float64(tol), arity=np.int64(k),
                perm_x=np.asarray(perm_x, np.int32), xoff=np.asarray(xoff, np.int64),
                koff=np.asarray(koff, np.int64), rank=rank, ident=ident,
                P=cat(P_parts), P_off=P_off, U=cat(U_parts), U_off=U_off,
                skel_L=np.concatenate([J[i] for i in range(nb)]).astype(np.int64))
