"""Preconditioned conjugate gradients with a Lanczos condition estimate.

Test infrastructure only (the CPU oracle).

The interface system S_hat u = g_hat (eq. globInt) is solved by CG
preconditioned with M^-1 (eq. BDDCprec), from x0 = 0, stopping when the
recursive residual satisfies ||r||_2 <= tol ||g_hat||_2 (Sec. 7: a 1e-8
reduction of the l2 norm of the residual; the unpreconditioned residual is
used).  The CG coefficients give the Lanczos tridiagonal matrix of
M^-1 S_hat, whose extreme eigenvalues estimate lambda_min (>= 1 by Theorem
teoEst) and lambda_max, hence the k_2 reported in Sec. 7.
"""
import numpy as np


def pcg(apply_A, apply_M, b, tol=1e-8, maxit=1000, x0=None, fixed_iters=None):
    """Returns (x, info) with info = dict(iters, alphas, betas, resid)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    z = apply_M(r)
    p = z.copy()
    rz = r @ z
    alphas, betas, res = [], [], [np.linalg.norm(r) / nb]
    it = 0
    while True:
        if fixed_iters is None and (res[-1] <= tol or it >= maxit):
            break
        if fixed_iters is not None and it >= fixed_iters:
            break
        q = apply_A(p)
        pq = p @ q
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        alphas.append(alpha)
        res.append(np.linalg.norm(r) / nb)
        if fixed_iters is None and res[-1] <= tol:
            break
        z = apply_M(r)
        rz_new = r @ z
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
    return x, {"iters": it, "alphas": np.array(alphas), "betas": np.array(betas),
               "resid": np.array(res)}


def lanczos_extremes(alphas, betas):
    """Extreme eigenvalues of the CG-Lanczos tridiagonal matrix:
    T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_{j,j+1} = sqrt(b_j)/a_j."""
    m = len(alphas)
    if m == 0:
        return np.nan, np.nan
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return ev[0], ev[-1]
