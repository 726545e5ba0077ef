"""Space and frequency trees for the row-wise butterfly (host, FP64).

Both trees are complete binary trees of one common depth L: the butterfly moves
one level down the space tree while moving one level up the frequency tree, so
every level pairs space depth l with frequency depth L - l (Sec. 2, the level
recursion and Fig. "BF-levels").  Nodes may be empty; an empty node simply
yields rank-zero blocks.

Space tree.  The paper builds a Fiedler tree: split a region by the sign of its
second Neumann eigenfunction, recurse (Sec. 3, Alg. "Construct Fiedler tree" and
the Neumann eigenproblem).  On an axis-aligned box [lo, hi] the second Neumann
eigenfunction is -cos(pi (x_a - lo_a) / (hi_a - lo_a)) along the longer side a,
whose sign splits the box at its midpoint; the mesh-free rule (points with
phi_2 <= 0 go to the first part) then puts x_a <= mid in the first child.  On
the flat periodic square the Fiedler vector itself is degenerate (cos x1, sin x1,
cos x2, sin x2 share one eigenvalue), so the box form is used there: the root box
is the points' bounding box, child boxes are the geometric halves, ties in side
length go to x1.  Mesh surfaces use `mesh_fiedler_tree` in `mesh_tree.py`.

Frequency tree.  A binary tree on the eigenvalue-sorted column range (Sec. 3,
first paragraph: a tree on [0, lambda_m]); by index rather than by eigenvalue
value so that degenerate eigenvalue shells cannot unbalance it.  A range [a, b)
splits at a + ceil((b - a) / 2).
"""
import numpy as np


def depth_for(n, leaf, arity=2):
    """L = ceil(log_arity(n / leaf)), at least 0."""
    L = 0
    while -(-n // arity ** L) > leaf:
        L += 1
    return L


def box_bisection_tree(points, L):
    """Neumann-box Fiedler tree of fixed depth L on 2-D points.

    Returns (perm_x int32[n], xoff int64[2^L + 1]): tree position -> point
    index, and the leaf offsets in tree positions.  Leaves are in left-first
    order; inside a node points keep ascending original index.
    """
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    lo = pts.min(axis=0) if n else np.zeros(2)
    hi = pts.max(axis=0) if n else np.zeros(2)
    nodes = [(np.arange(n, dtype=np.int64), lo.copy(), hi.copy())]
    for _ in range(L):
        nxt = []
        for idx, blo, bhi in nodes:
            ext = bhi - blo
            a = 0 if ext[0] >= ext[1] else 1
            mid = 0.5 * (blo[a] + bhi[a])
            first = pts[idx, a] <= mid
            lo1, hi1 = blo.copy(), bhi.copy()
            hi1[a] = mid
            lo2, hi2 = blo.copy(), bhi.copy()
            lo2[a] = mid
            nxt.append((idx[first], lo1, hi1))
            nxt.append((idx[~first], lo2, hi2))
        nodes = nxt
    perm = np.concatenate([nd[0] for nd in nodes]) if nodes else np.zeros(0, np.int64)
    sizes = np.array([len(nd[0]) for nd in nodes], dtype=np.int64)
    xoff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return perm.astype(np.int32), xoff


def quadtree(points, L):
    """Quadtree of fixed depth L on 2-D points (Sec. 2: the construction
    generalizes to quadtrees; Sec. 5 uses one on [-pi, pi]^2).  A box's four
    children are its quadrants, split at the midpoints of both sides, in the
    order (x1 low, x2 low), (x1 low, x2 high), (x1 high, x2 low), (x1 high, x2
    high); a coordinate equal to the midpoint goes low, as in the binary
    Neumann-box tree.  The root box is the points' bounding box.

    Returns (perm_x int32[n], xoff int64[4^L + 1]) like box_bisection_tree.
    """
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    lo = pts.min(axis=0) if n else np.zeros(2)
    hi = pts.max(axis=0) if n else np.zeros(2)
    nodes = [(np.arange(n, dtype=np.int64), lo.copy(), hi.copy())]
    for _ in range(L):
        nxt = []
        for idx, blo, bhi in nodes:
            mid = 0.5 * (blo + bhi)
            low1 = pts[idx, 0] <= mid[0]
            low2 = pts[idx, 1] <= mid[1]
            for h1 in (0, 1):
                for h2 in (0, 1):
                    sel = (low1 != bool(h1)) & (low2 != bool(h2))
                    clo, chi = blo.copy(), bhi.copy()
                    if h1:
                        clo[0] = mid[0]
                    else:
                        chi[0] = mid[0]
                    if h2:
                        clo[1] = mid[1]
                    else:
                        chi[1] = mid[1]
                    nxt.append((idx[sel], clo, chi))
        nodes = nxt
    perm = np.concatenate([nd[0] for nd in nodes]) if nodes else np.zeros(0, np.int64)
    sizes = np.array([len(nd[0]) for nd in nodes], dtype=np.int64)
    xoff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return perm.astype(np.int32), xoff


def frequency_tree(m, L, arity=2):
    """Leaf offsets int64[arity^L + 1] of the index-splitting tree on [0, m).
    A node's range [a, b) is halved at a + ceil((b - a) / 2); a 4-ary node
    halves twice, so its four children are the binary tree's grandchildren."""
    if arity not in (2, 4):
        raise ValueError("arity must be 2 or 4")
    L = L * (1 if arity == 2 else 2)
    ranges = [(0, m)]
    for _ in range(L):
        nxt = []
        for a, b in ranges:
            s = a + (b - a + 1) // 2
            nxt.append((a, s))
            nxt.append((s, b))
        ranges = nxt
    return np.array([r[0] for r in ranges] + [m], dtype=np.int64)


def node_range(off, L, depth, idx, arity=2):
    """[start, end) of node idx at the given depth, from leaf offsets of a depth-L tree."""
    w = arity ** (L - depth)
    return int(off[idx * w]), int(off[(idx + 1) * w])
