"""Linear finite elements on a triangle mesh, element by element (oracle, test infrastructure).

The discrete Laplace-Beltrami eigenproblem of Sec. 1 (eq. eigenproblem), with
piecewise-linear hat functions: the stiffness entry K[a, b] sums, over the
triangles containing both vertices, area * grad(phi_a) . grad(phi_b); the
lumped mass gives each vertex a third of the area of every triangle around it.
Here the gradients are built explicitly from each triangle's geometry (the
gradient of the hat function of vertex a is the in-plane normal of the
opposite edge divided by twice the area), a formulation independent of the
cotangent formula used by the workload generator.  Dense output, small meshes only.
"""
import numpy as np


def stiffness_and_mass(v, f):
    n = len(v)
    K = np.zeros((n, n))
    Md = np.zeros(n)
    for tri in f:
        P = v[tri]                       # 3 x 3, rows are the corners
        nrm = np.cross(P[1] - P[0], P[2] - P[0])
        area2 = np.linalg.norm(nrm)
        unit = nrm / area2
        grads = []
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            e = P[c] - P[b]              # edge opposite corner a
            g = np.cross(unit, e) / area2
            # orient toward corner a: the hat function grows from the edge to the corner
            if np.dot(g, P[a] - P[b]) < 0:
                g = -g
            grads.append(g)
        area = 0.5 * area2
        for a in range(3):
            Md[tri[a]] += area / 3.0
            for b in range(3):
                K[tri[a], tri[b]] += area * np.dot(grads[a], grads[b])
    return K, Md
