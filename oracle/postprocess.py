"""Discretisation errors for the manufactured solutions (test use only).

|u - Pi^nabla_k u_h|_{1,h} and ||p - p_h||_0 by element quadrature, with the
element projections of the virtual element space (Sec. 3).  The theorem of
Sec. 3.2 (eq. teoConv) predicts O(h^k) for both on smooth solutions.
"""
import numpy as np
from inputs.vem import element_matrices, element_quadrature
from inputs.poly import eval3, grad3_coef, dim3


def errors(pb, ufull, pfull, grad_u, p_exact):
    m, k, L = pb.mesh, pb.k, pb.L
    eu2 = 0.0
    ep2 = 0.0
    chunk = 256
    for s in range(0, m.nK, chunk):
        el = np.arange(s, min(m.nK, s + chunk))
        out = element_matrices(m, k, el, 1.0, keep=True)
        d = ufull[pb.gmap[el]]
        pin = np.einsum("ecbn,en->ecb", out["PiN"], d)
        P, W = element_quadrature(m, el, 2 * k + 4)
        xK, hK = m.elem_centroid[el], m.elem_diam[el]
        Xh = (P - xK[:, None]) / hK[:, None, None]
        M = eval3(Xh, k)
        G3 = grad3_coef(k)
        dM = np.einsum("dab,eqb->eqad", G3, M) / hK[:, None, None, None]
        gh = np.einsum("ecb,eqbd->eqcd", pin, dM)
        eu2 += np.einsum("eq,eqcd->", W, (grad_u(P) - gh) ** 2)
        Mp = eval3(Xh, k - 1)
        ph = np.einsum("eqa,ea->eq", Mp, pfull[L.nP * el[:, None] + np.arange(L.nP)[None, :]])
        ep2 += np.einsum("eq,eq->", W, (p_exact(P) - ph) ** 2)
    return np.sqrt(eu2), np.sqrt(ep2)
