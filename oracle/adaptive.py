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

Edges (an extension, not in the paper's text): the same pencil on the dual
coordinates of an edge, with the parallel sums taken over every subdomain
sharing it, (At^(1) : ... : At^(n)) psi = lambda (A^(1) : ... : A^(n)) psi
(the parallel sum is associative).  Faces alone leave kappa_2 above 4 at
k = 4 however many face constraints are added; with edges the paper's flat
kappa_2 of about 1.5 at nu_tol = 2 across k = 2, 3, 4 is approached.
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
    """(At_par, A_par, subs) for entity e in the current basis: the parallel
    sums over the subdomains sharing it (two for a face), folded left."""
    dual = bddc.de_idx[e]
    subs = bddc.ent_subs[e]
    At, A = [], []
    for k in subs:
        L = bddc.loc[k]
        pos = np.array([np.nonzero(L.gid == d)[0][0] for d in dual], dtype=np.int64)
        A.append(L.St[np.ix_(pos, pos)])
        At.append(schur_onto_cholesky(L.St, pos) if cholesky else schur_onto(L.St, pos))
    Atp, Ap = At[0], A[0]
    for q in range(1, len(subs)):
        Atp, Ap = parallel_sum(Atp, At[q]), parallel_sum(Ap, A[q])
    return Atp, Ap, subs


def adaptive_rows(bddc, theta, edges=False):
    """Append the adaptive rows of every face (and with edges=True every
    edge shared by two or more subdomains) to bddc.extra_rows (original
    coordinates of the entity's DoFs) and return per-entity information."""
    info = []
    for e, E in enumerate(bddc.ents):
        if len(bddc.de_idx[e]) == 0:
            continue
        if not ((E["kind"] == 2 and len(bddc.ent_subs[e]) == 2)
                or (edges and E["kind"] == 1 and len(bddc.ent_subs[e]) >= 2)):
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
