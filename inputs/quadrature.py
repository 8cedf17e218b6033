"""Quadrature rules on [0,1], triangles and tetrahedra (collapsed-coordinate
Gauss rules: Gauss-Jacobi in the collapsed directions, Gauss-Legendre in the
last).  A rule built for degree d integrates every polynomial of total
degree <= d exactly."""
import numpy as np
from scipy.special import roots_jacobi


def gauss_legendre01(n):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def gauss_jacobi01(n, beta):
    """Nodes/weights on [0,1] for the weight x**beta."""
    t, w = roots_jacobi(n, 0.0, float(beta))
    return 0.5 * (t + 1.0), w / 2.0 ** (beta + 1)


def gauss_lobatto_interior01(k):
    """The k-1 interior nodes of the (k+1)-point Gauss-Lobatto rule on [0,1]
    (the edge points of the degree-k space)."""
    if k < 2:
        return np.zeros(0)
    # interior Lobatto nodes are the roots of P'_k
    c = np.zeros(k + 1)
    c[k] = 1.0
    dc = np.polynomial.legendre.legder(c)
    r = np.sort(np.polynomial.legendre.legroots(dc).real)
    return 0.5 * (r + 1.0)


def lobatto_weights01(nodes):
    """Weights of the interpolatory rule on the given nodes of [0,1]."""
    n = len(nodes)
    V = np.vander(nodes, n, increasing=True).T
    mom = 1.0 / np.arange(1, n + 1)
    return np.linalg.solve(V, mom)


def triangle_rule(d):
    """Barycentric coordinates (q,3) and weights (q,) summing to 1 (area
    fraction) for the reference triangle; exact to degree d."""
    n = max(1, (d + 2) // 2)
    u, wu = gauss_jacobi01(n, 1)
    v, wv = gauss_legendre01(n)
    U, Vv = np.meshgrid(u, v, indexing="ij")
    W = np.outer(wu, wv) * 2.0  # area of reference triangle is 1/2 -> fractions
    lam = np.stack([1 - U, U * (1 - Vv), U * Vv], axis=-1).reshape(-1, 3)
    return lam, W.reshape(-1)


def tet_rule(d):
    """Barycentric coordinates (q,4) and weights (q,) summing to 1 (volume
    fraction) for the reference tetrahedron; exact to degree d."""
    n = max(1, (d + 2) // 2)
    u, wu = gauss_jacobi01(n, 2)
    v, wv = gauss_jacobi01(n, 1)
    w, ww = gauss_legendre01(n)
    U, Vv, Ww = np.meshgrid(u, v, w, indexing="ij")
    W = np.einsum("i,j,k->ijk", wu, wv, ww) * 6.0
    lam = np.stack([1 - U, U * (1 - Vv), U * Vv * (1 - Ww), U * Vv * Ww], axis=-1)
    return lam.reshape(-1, 4), W.reshape(-1)
