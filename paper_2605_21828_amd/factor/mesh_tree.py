"""Neumann Fiedler tree on a triangulated surface (host, FP64).

The space tree of the butterfly factorization on a manifold is a Fiedler tree
(Sec. 3, Alg. "Construct Fiedler tree"): split a region by the sign of the
second eigenfunction of its Laplace-Beltrami operator with homogeneous Neumann
conditions (Sec. 3, eq. neumann-eigenproblem), recurse.  On a mesh given by
its vertices, the mesh-free rule of the paper applies: vertices with
phi_2(x_j) <= 0 form the first part.

Discrete Neumann problem on a vertex subset S: the stiffness matrix keeps the
cotangent weights of edges inside S, its diagonal is minus the row sum of
those (edges leaving S are dropped, which is the natural boundary condition),
and the mass is the lumped mass restricted to S.  Readings taken where the
paper is silent: the eigenvector's sign is fixed so its largest-magnitude
entry is positive (deterministic trees); if one side comes out empty the
subset is cut at the mass-weighted median of phi_2; the depth is fixed at L so
both trees have equal depth.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def fiedler_vector(Kraw, Ms, dense_max=64):
    """Second Neumann eigenvector of a vertex subset (sign: largest entry positive).

    Kraw is the stiffness matrix restricted to the subset (rows and columns),
    Ms its lumped masses."""
    n = Kraw.shape[0]
    if n < 2:
        return np.zeros(n)
    off = Kraw - sp.diags(Kraw.diagonal())
    Ks = (off - sp.diags(np.asarray(off.sum(axis=1)).ravel())).tocsr()
    if n <= dense_max:
        d = 1.0 / np.sqrt(Ms)
        A = (Ks.toarray() * d[:, None]) * d[None, :]
        w, U = sla.eigh(A, subset_by_index=[0, 1])
        phi = U[:, 1] * d
    else:
        scale = abs(Ks.diagonal()).max() / Ms.max()
        w, U = spla.eigsh(Ks, k=2, M=sp.diags(Ms).tocsc(), sigma=-1e-6 * scale, which="LM", tol=1e-10)
        phi = U[:, np.argsort(w)[1]]
    if phi[np.argmax(np.abs(phi))] < 0:
        phi = -phi
    return phi


def split_mask(Kraw, Ms):
    """Boolean mask of the first part by the sign rule, else the mass-weighted median."""
    phi = fiedler_vector(Kraw, Ms)
    first = phi <= 0
    if first.all() or not first.any():
        order = np.argsort(phi, kind="stable")
        cm = np.cumsum(Ms[order])
        cut = int(np.searchsorted(cm, 0.5 * cm[-1])) + 1
        first = np.zeros(len(Ms), dtype=bool)
        first[order[:cut]] = True
    return first


def mesh_fiedler_tree(K, M, L, log=None):
    """Fixed-depth Neumann Fiedler tree.  Returns (perm_x int32[n], xoff int64[2^L + 1])."""
    n = K.shape[0]
    K = sp.csr_matrix(K)
    M = np.asarray(M, dtype=np.float64)
    # each node carries its vertex ids and the stiffness restricted to them
    nodes = [(np.arange(n, dtype=np.int64), K)]
    for d in range(L):
        nxt = []
        for S, Kr in nodes:
            if len(S) < 2:
                nxt += [(S, Kr), (S[:0], Kr[:0][:, :0])]
                continue
            first = split_mask(Kr, M[S])
            a, b = np.nonzero(first)[0], np.nonzero(~first)[0]
            nxt += [(S[a], Kr[a][:, a].tocsr()), (S[b], Kr[b][:, b].tocsr())]
        nodes = nxt
        if log:
            sz = [len(s) for s, _ in nodes]
            log(dict(depth=d + 1, nodes=len(nodes), min=min(sz), max=max(sz)))
    perm = np.concatenate([s for s, _ in nodes]).astype(np.int32)
    xoff = np.concatenate([[0], np.cumsum([len(s) for s, _ in nodes])]).astype(np.int64)
    return perm, xoff
