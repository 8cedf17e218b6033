"""Scaled monomial bases and the coefficient-space operators (gradient,
Laplacian, x-wedge) used by the virtual element projections.

3D monomials are m_a(x) = ((x - x_K)/h_K)^a, ordered by total degree; 2D face
monomials use the face frame (t1, t2) and the face diameter.  All operators
below act on coefficient vectors in the scaled variable xh = (x - x_K)/h_K.
"""
import numpy as np
from functools import lru_cache


@lru_cache(None)
def mono3(n):
    out = []
    for d in range(n + 1):
        for a in range(d, -1, -1):
            for b in range(d - a, -1, -1):
                out.append((a, b, d - a - b))
    return tuple(out)


@lru_cache(None)
def mono2(n):
    out = []
    for d in range(n + 1):
        for a in range(d, -1, -1):
            out.append((a, d - a))
    return tuple(out)


def dim3(n):
    return 0 if n < 0 else (n + 1) * (n + 2) * (n + 3) // 6


def dim2(n):
    return 0 if n < 0 else (n + 1) * (n + 2) // 2


@lru_cache(None)
def index3(n):
    return {e: i for i, e in enumerate(mono3(n))}


@lru_cache(None)
def index2(n):
    return {e: i for i, e in enumerate(mono2(n))}


def eval3(Xh, n):
    """Monomials of degree <= n at scaled points Xh (...,3) -> (..., dim3(n))."""
    P = [np.ones(Xh.shape[:-1] + (n + 1,)) for _ in range(3)]
    for d in range(3):
        for p in range(1, n + 1):
            P[d][..., p] = P[d][..., p - 1] * Xh[..., d]
    ex = np.array(mono3(n))
    return P[0][..., ex[:, 0]] * P[1][..., ex[:, 1]] * P[2][..., ex[:, 2]]


def eval2(Xi, n):
    P = [np.ones(Xi.shape[:-1] + (n + 1,)) for _ in range(2)]
    for d in range(2):
        for p in range(1, n + 1):
            P[d][..., p] = P[d][..., p - 1] * Xi[..., d]
    ex = np.array(mono2(n))
    return P[0][..., ex[:, 0]] * P[1][..., ex[:, 1]]


def grad2_eval(Xi, n):
    """d/dxi_d of 2D monomials -> (..., dim2(n), 2) (in the xi variable)."""
    ex = np.array(mono2(n))
    out = np.zeros(Xi.shape[:-1] + (len(ex), 2))
    P = [np.ones(Xi.shape[:-1] + (n + 1,)) for _ in range(2)]
    for d in range(2):
        for p in range(1, n + 1):
            P[d][..., p] = P[d][..., p - 1] * Xi[..., d]
    for i, (a, b) in enumerate(ex):
        if a > 0:
            out[..., i, 0] = a * P[0][..., a - 1] * P[1][..., b]
        if b > 0:
            out[..., i, 1] = b * P[0][..., a] * P[1][..., b - 1]
    return out


@lru_cache(None)
def grad3_coef(n):
    """G[d] (dim3(n) x dim3(n)): d/dxh_d m_a = sum_b G[d][a,b] m_b."""
    idx = index3(n)
    G = np.zeros((3, dim3(n), dim3(n)))
    for i, e in enumerate(mono3(n)):
        for d in range(3):
            if e[d] > 0:
                f = list(e)
                f[d] -= 1
                G[d, i, idx[tuple(f)]] = e[d]
    return G


@lru_cache(None)
def lap3_coef(n):
    idx = index3(n)
    L = np.zeros((dim3(n), dim3(n)))
    for i, e in enumerate(mono3(n)):
        for d in range(3):
            if e[d] > 1:
                f = list(e)
                f[d] -= 2
                L[i, idx[tuple(f)]] += e[d] * (e[d] - 1)
    return L


@lru_cache(None)
def lap2_coef(n):
    idx = index2(n)
    L = np.zeros((dim2(n), dim2(n)))
    for i, e in enumerate(mono2(n)):
        for d in range(2):
            if e[d] > 1:
                f = list(e)
                f[d] -= 2
                L[i, idx[tuple(f)]] += e[d] * (e[d] - 1)
    return L


_EPS = np.zeros((3, 3, 3))
_EPS[0, 1, 2] = _EPS[1, 2, 0] = _EPS[2, 0, 1] = 1
_EPS[0, 2, 1] = _EPS[2, 1, 0] = _EPS[1, 0, 2] = -1


def wedge_coef(n):
    """W[k, g] -> (3, dim3(n+1)) coefficients of xh ^ (e_k m_g) for m_g of
    degree <= n: component i = sum_j eps_ijk xh_j m_g."""
    idx = index3(n + 1)
    W = np.zeros((3, dim3(n), 3, dim3(n + 1)))
    for g, e in enumerate(mono3(n)):
        for kk in range(3):
            for i in range(3):
                for j in range(3):
                    if _EPS[i, j, kk] != 0:
                        f = list(e)
                        f[j] += 1
                        W[kk, g, i, idx[tuple(f)]] += _EPS[i, j, kk]
    return W


@lru_cache(None)
def helmholtz_tables(jmax):
    """Decomposition of homogeneous vector monomials e_c m_g (|g| = j) as
    grad(q) + xh ^ r with q homogeneous of degree j+1 and r of degree j-1
    (all in the scaled variable).  Returns, for every j <= jmax, arrays
    Q[j] (3, dim3(j), dim3(j+1)) and R[j] (3, dim3(j), 3, dim3(max(j-1,0)))
    indexed by full-degree monomial positions."""
    Q, R = {}, {}
    for j in range(jmax + 1):
        nq = dim3(j + 1)
        nr = dim3(j - 1) if j >= 1 else 0
        G = grad3_coef(j + 1)
        ex = mono3(j + 1)
        hq = [i for i, e in enumerate(ex) if sum(e) == j + 1]
        tgt = [i for i, e in enumerate(mono3(j)) if sum(e) == j]
        ncol_q = len(hq)
        if j >= 1:
            W = wedge_coef(j - 1)
            hr = [i for i, e in enumerate(mono3(j - 1)) if sum(e) == j - 1]
        else:
            hr = []
        # columns: grad of homogeneous q, then xh^(e_k m_r)
        cols = []
        for i in hq:
            v = np.zeros((3, dim3(j)))
            for d in range(3):
                v[d] = G[d, i, : dim3(j)]
            cols.append(v.ravel())
        for kk in range(3):
            for g in hr:
                v = W[kk, g][:, : dim3(j)]
                cols.append(v.ravel())
        Mat = np.array(cols).T  # (3*dim3(j), ncols)
        Qj = np.zeros((3, dim3(j), nq))
        Rj = np.zeros((3, dim3(j), 3, max(nr, 1)))
        for c in range(3):
            for g in tgt:
                b = np.zeros((3, dim3(j)))
                b[c, g] = 1.0
                sol, *_ = np.linalg.lstsq(Mat, b.ravel(), rcond=None)
                assert np.allclose(Mat @ sol, b.ravel(), atol=1e-12)
                for t, i in enumerate(hq):
                    Qj[c, g, i] = sol[t]
                off = ncol_q
                for kk in range(3):
                    for t, gg in enumerate(hr):
                        Rj[c, g, kk, gg] = sol[off + kk * len(hr) + t]
        Q[j] = Qj
        R[j] = Rj
    return Q, R
