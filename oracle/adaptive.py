"""Adaptive face constraints (Sec. 6): the generalized eigenproblems that
enrich the primal space.  Test infrastructure (FP64 CPU oracle).

For a face F shared by subdomains i and j, in the coordinates of the
current change of basis (Sec. 4.3):

* A^(k)  = the principal minor of S_Gamma^(k) (transformed) on the dual
  coordinates F_Delta of F (the matrix deluxe scaling uses);
* At^(k) = the Schur complement of the transformed S_Gamma^(k) onto F_Delta,
  eliminating every other coordinate of Gamma_k (primal ones included);
* the parallel sum X:Y = (X^-1 + Y^-1)^-1, evaluated as X (X+Y)^+ Y so that
  singular X or Y (floating subdomains) are allowed;
* the pencil (At^(i):At^(j)) psi = lambda (A^(i):A^(j)) psi; the
  eigenvectors with lambda < 1/theta give the new primal functionals
  (A^(i):A^(j)) Psi on the dual coordinates of F.

One pass over the faces, with the bases of the minimal primal space; the
caller then rebuilds the change of basis with the appended rows.
"""
import numpy as np
import scipy.linalg as sla

PINV_RTOL = 1e-12


def parallel_sum(X, Y, rtol=PINV_RTOL):
    """X:Y = X (X+Y)^+ Y, symmetrised (X, Y symmetric PSD)."""
    P = X @ sla.pinvh(X + Y, rtol=rtol) @ Y
    return 0.5 * (P + P.T)


def schur_onto(S, keep, rtol=PINV_RTOL):
    """Schur complement of symmetric S onto the index set `keep`,
    eliminating all other indices (pseudo-inverse of the eliminated block)."""
    keep = np.asarray(keep)
    other = np.setdiff1d(np.arange(S.shape[0]), keep)
    if len(other) == 0:
        return S[np.ix_(keep, keep)].copy()
    Skk = S[np.ix_(keep, keep)]
    Sok = S[np.ix_(other, keep)]
    Soo = S[np.ix_(other, other)]
    R = Skk - Sok.T @ sla.pinvh(Soo, rtol=rtol) @ Sok
    return 0.5 * (R + R.T)


def schur_onto_cholesky(S, keep):
    """The same Schur complement with the eliminated block factored by
    Cholesky (it is positive definite whenever the rigid-mode traces on
    `keep` are independent): a second FP64 evaluation of the formula."""
    keep = np.asarray(keep)
    other = np.setdiff1d(np.arange(S.shape[0]), keep)
    c = sla.cho_factor(S[np.ix_(other, other)])
    R = S[np.ix_(keep, keep)] - S[np.ix_(other, keep)].T @ sla.cho_solve(c, S[np.ix_(other, keep)])
    return 0.5 * (R + R.T)


def face_pencil(bddc, e, cholesky=False):
    """(At_par, A_par, subs) for face entity e in the current basis."""
    dual = bddc.de_idx[e]
    subs = bddc.ent_subs[e]
    At, A = [], []
    for k in subs:
        L = bddc.loc[k]
        pos = np.array([np.nonzero(L.gid == d)[0][0] for d in dual], dtype=np.int64)
        A.append(L.St[np.ix_(pos, pos)])
        At.append(schur_onto_cholesky(L.St, pos) if cholesky else schur_onto(L.St, pos))
    return parallel_sum(At[0], At[1]), parallel_sum(A[0], A[1]), subs


def adaptive_rows(bddc, theta):
    """Append the adaptive rows of every face to bddc.extra_rows (original
    coordinates of the face DoFs) and return per-face information."""
    info = []
    for e, E in enumerate(bddc.ents):
        if E["kind"] != 2 or len(bddc.ent_subs[e]) != 2 or len(bddc.de_idx[e]) == 0:
            continue
        Atp, Ap, subs = face_pencil(bddc, e)
        lam, Psi = sla.eigh(Atp, Ap)
        sel = lam < 1.0 / theta
        rows_dual = Ap @ Psi[:, sel]                    # functionals on F_Delta
        Qd = bddc.Q[e][:, bddc.npi[e]:]                 # dual basis (original coordinates)
        rows = (Qd @ rows_dual).T                        # m x n_F
        # unit rows: the span is what matters, and the rank test of the
        # change of basis is relative to the largest singular value
        rows = rows / np.maximum(np.linalg.norm(rows, axis=1, keepdims=True), 1e-300)
        if rows.shape[0]:
            bddc.extra_rows[e] = rows
        info.append({"entity": e, "subs": tuple(subs), "n_dual": len(bddc.de_idx[e]),
                     "eigenvalues": lam, "n_selected": int(sel.sum())})
    return info
