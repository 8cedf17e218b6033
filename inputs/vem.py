"""Divergence-free virtual elements of degree k on hexahedra (Sec. 3).

Local degrees of freedom of an element K (Sec. 3, D1-D5), in this order:

* D1: the three components at each of the 8 vertices;
* D2: the three components at the k-1 interior Gauss-Lobatto points of
  each of the 12 edges (the paper only asks for k-1 distinct points);
* D3: per face f and scaled face monomial m of degree <= k-2,
  (1/|f|) int_f (v.n_f) m, (1/|f|) int_f (v.t1_f) m, (1/|f|) int_f (v.t2_f) m,
  with the face frame (t1_f, t2_f, n_f) fixed globally per face (n_f points
  toward +axis), so the tangential moments recover v_tau;
* D4: (1/|K|) int_K v.(xh ^ (e_c m_g)) for the scaled monomials m_g of
  degree <= k-3 (k = 3: the 3 constants), leaving out the pairs (c = z, m_g
  = z q): xh ^ (e_x x q) + xh ^ (e_y y q) + xh ^ (e_z z q) = xh ^ (xh q) = 0,
  so x ^ [P_{k-3}]^3 has dimension 3 dim P_{k-3} - dim P_{k-4} (k = 4: 11);
* D5: (h_K/|K|) int_K div(v) m for the non-constant scaled monomials of
  degree <= k-1.

Moments are normalised by measure so that every DoF of an O(1) field is O(1).

From these, every quantity the discrete forms need is computed:

* the face H1 projection Pi^{nabla,f}_k and, through the enhancement
  condition (iii) of the face space, the face moments up to degree k+1;
* div v in P_{k-1}(K) (condition (iii) of the element space);
* volume moments of v against [P_n]^3 via the splitting
  [P_n]^3 = grad P_{n+1} + x ^ [P_{n-1}]^3, integrating the gradient part by
  parts and taking the x-wedge part from D4 (low degrees) or from the
  super-enhancement of the velocity space (degrees k-2 and k-1);
* Pi^{nabla,K}_k (boundary-mean constant), Pi^0_{k-1} grad v, Pi^0_k v.

The local stiffness is a_h^K of eq. (discreteA) with nu_K on both terms and
a diagonal "D-recipe" stabilisation sigma_i = max(h_K, (consistency)_ii).
The divergence rows are exact (computed from D1-D3 and D5).
"""
import numpy as np
from .quadrature import (gauss_legendre01, gauss_lobatto_interior01, triangle_rule,
                         tet_rule)
from .poly import (mono3, mono2, dim3, dim2, index3, eval3, eval2, grad2_eval, grad3_coef,
                   lap3_coef, lap2_coef, wedge_coef, helmholtz_tables)
from .mesh import LOCAL_VERTS, LOCAL_EDGES, LOCAL_FACES


def ein(*args):
    return np.einsum(*args, optimize=True)


class DofLayout:
    """Element-local DoF numbering for degree k."""

    def __init__(self, k):
        assert k in (2, 3, 4), "degrees 2, 3 and 4 are supported"
        self.k = k
        self.nf2 = dim2(k - 2)  # face moment monomials per kind
        ex = mono3(k - 3) if k >= 3 else ()
        self.d4_pairs = [(c, g) for c in range(3) for g, e in enumerate(ex)
                         if not (c == 2 and e[2] >= 1)]
        self._d4_pos = {pr: i for i, pr in enumerate(self.d4_pairs)}
        self.nD4 = len(self.d4_pairs)
        self.nD5 = dim3(k - 1) - 1
        self.nP = dim3(k - 1)  # pressure monomials per element
        self.off2 = 24
        self.off3 = 24 + 36 * (k - 1)
        self.off4 = self.off3 + 18 * self.nf2
        self.off5 = self.off4 + self.nD4
        self.N = self.off5 + self.nD5
        self.nI = self.nD4 + self.nD5  # element-internal velocity dofs

    def d1(self, lv, c):
        return 3 * lv + c

    def d2(self, le, j, c):
        return self.off2 + 3 * ((self.k - 1) * le + j) + c

    def d3(self, lf, b, kind):
        return self.off3 + 3 * (self.nf2 * lf + b) + kind

    def d4(self, i):
        return self.off4 + i

    def d5(self, a):  # a = 0 .. nD5-1  (monomial index a+1)
        return self.off5 + a

    def d4_terms(self, c, g):
        """(coefficient, DoF) pairs giving (1/|K|) int_K v.(xh ^ (e_c m_g)) for
        any m_g of degree <= k-3: the DoF itself, or for a left-out pair
        (c = z, m_g = z q) minus the x q and y q moments."""
        if (c, g) in self._d4_pos:
            return [(1.0, self.d4(self._d4_pos[(c, g)]))]
        e = mono3(self.k - 3)[g]
        idx = index3(self.k - 3)
        gx = idx[(e[0] + 1, e[1], e[2] - 1)]
        gy = idx[(e[0], e[1] + 1, e[2] - 1)]
        return [(-1.0, self.d4(self._d4_pos[(0, gx)])), (-1.0, self.d4(self._d4_pos[(1, gy)]))]


def _edge_nodes(k):
    return np.concatenate([[0.0], gauss_lobatto_interior01(k), [1.0]])


def _lagrange(nodes, s):
    """Lagrange basis on nodes evaluated at s -> (len(s), len(nodes))."""
    n = len(nodes)
    L = np.ones((len(s), n))
    for i in range(n):
        for j in range(n):
            if i != j:
                L[:, i] *= (s - nodes[j]) / (nodes[i] - nodes[j])
    return L


def element_quadrature(mesh, elems, deg):
    """Volume quadrature: cones from the vertex average over the two
    triangles of each planar face.  -> points (E,Q,3), weights (E,Q)."""
    X8 = mesh.verts[mesh.elem_verts[elems]]
    xb = mesh.elem_xbar[elems]
    lam, w = tet_rule(deg)
    pts, wts = [], []
    for (a, s, vs, es) in LOCAL_FACES:
        for tri in [(vs[0], vs[1], vs[2]), (vs[0], vs[2], vs[3])]:
            A, B, C = X8[:, tri[0]], X8[:, tri[1]], X8[:, tri[2]]
            vol = np.abs(ein("ij,ij->i", A - xb, np.cross(B - xb, C - xb))) / 6.0
            P = (lam[None, :, 0, None] * xb[:, None] + lam[None, :, 1, None] * A[:, None]
                 + lam[None, :, 2, None] * B[:, None] + lam[None, :, 3, None] * C[:, None])
            pts.append(P)
            wts.append(vol[:, None] * w[None, :])
    return np.concatenate(pts, 1), np.concatenate(wts, 1)


def face_quadrature(mesh, elems, lf, deg):
    """Quadrature on local face lf of each element -> (E,Q,3), (E,Q)."""
    X8 = mesh.verts[mesh.elem_verts[elems]]
    a, s, vs, es = LOCAL_FACES[lf]
    lam, w = triangle_rule(deg)
    pts, wts = [], []
    for tri in [(vs[0], vs[1], vs[2]), (vs[0], vs[2], vs[3])]:
        A, B, C = X8[:, tri[0]], X8[:, tri[1]], X8[:, tri[2]]
        ar = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
        P = lam[None, :, 0, None] * A[:, None] + lam[None, :, 1, None] * B[:, None] + lam[None, :, 2, None] * C[:, None]
        pts.append(P)
        wts.append(ar[:, None] * w[None, :])
    return np.concatenate(pts, 1), np.concatenate(wts, 1)


def _face_frame(mesh, elems, lf):
    gf = mesh.elem_faces[elems, lf]
    return (mesh.face_normal[gf], mesh.face_t1[gf], mesh.face_t2[gf],
            mesh.face_centroid[gf], mesh.face_diam[gf], mesh.face_area[gf])


def element_matrices(mesh, k, elems, nu, force=None, keep=False):
    """Local matrices of the elements ``elems``.

    Returns dict with
      A  (E,N,N)   nu_K * (consistency + stabilisation)
      B  (E,nP,N)  rows b(v, m_a) for the pressure monomials m_a (a=0: constant)
      F  (E,N)     load (f_h, phi_i)_K = int f . Pi^0_k phi_i  (if force given)
      and, if keep, the projection matrices PiN (E,3,dim3(k),N) (Pi^nabla_k)
      and P0 (E,3,dim3(k),N) (Pi^0_k).
    """
    L = DofLayout(k)
    N = L.N
    E = len(elems)
    X8 = mesh.verts[mesh.elem_verts[elems]]
    xK = mesh.elem_centroid[elems]
    hK = mesh.elem_diam[elems]
    vK = mesh.elem_vol[elems]
    nuK = np.asarray(nu, float)[elems] if np.ndim(nu) else np.full(E, float(nu))
    qdeg = 2 * k + 1
    eye = np.eye(N)

    # ---------------- face level: moments of v_c up to degree k+1
    n1 = dim2(k + 1)
    nk2 = dim2(k)
    nlo = dim2(k - 2)
    enodes = _edge_nodes(k)
    sg, wg = gauss_legendre01(k + 1)
    Lg = _lagrange(enodes, sg)  # (Qe, k+1)
    FM = np.zeros((E, 6, 3, n1, N))
    Rf = np.zeros((E, 6, n1, dim3(k + 1)))  # restriction of 3D monomials to faces
    FMass_all = []
    lap2 = lap2_coef(k)
    for lf, (ax, s, vs, es) in enumerate(LOCAL_FACES):
        nf, t1, t2, xf, hf, af = _face_frame(mesh, elems, lf)
        P, W = face_quadrature(mesh, elems, lf, 2 * k + 3)
        Xi = np.stack([ein("eqi,ei->eq", P - xf[:, None], t1),
                       ein("eqi,ei->eq", P - xf[:, None], t2)], -1) / hf[:, None, None]
        Mf = eval2(Xi, k + 1)  # (E,Q,n1)
        FMass = ein("eq,eqa,eqb->eab", W, Mf, Mf)
        FMass_all.append(FMass)
        dM = grad2_eval(Xi, k) / hf[:, None, None, None]  # gradient in x, face coords
        Kst = ein("eq,eqad,eqbd->eab", W, dM, dM)
        # restriction of 3D monomials (degree <= k+1) to this face
        M3 = eval3((P - xK[:, None]) / hK[:, None, None], k + 1)
        Rf[:, lf] = np.linalg.solve(FMass, ein("eq,eqa,eqb->eab", W, Mf, M3))
        # DoF moments of degree <= k-2: int_f v_c m_b = |f| (n_c Dn + t1_c Dt1 + t2_c Dt2)
        DM = np.zeros((E, 3, nlo, N))
        for b in range(nlo):
            for kind, vec in enumerate((nf, t1, t2)):
                DM[:, :, b, L.d3(lf, b, kind)] = af[:, None] * vec
        # boundary of the face: 4 edges
        Kb0 = np.zeros((E, nk2))
        rhs_b = np.zeros((E, 3, nk2, N))  # edge terms for rows >= 1 and row 0
        for le in es:
            ea, v0, v1, st = LOCAL_EDGES[le]
            A0, A1 = X8[:, v0], X8[:, v1]
            ev = A1 - A0
            le_len = np.linalg.norm(ev, axis=1)
            ne = np.cross(ev, nf)
            ne /= np.linalg.norm(ne, axis=1)[:, None]
            mid = 0.5 * (A0 + A1)
            sgn = np.sign(ein("ei,ei->e", mid - xf, ne))
            ne *= sgn[:, None]
            Xq = A0[:, None] + sg[None, :, None] * ev[:, None]  # (E,Qe,3)
            Xiq = np.stack([ein("eqi,ei->eq", Xq - xf[:, None], t1),
                            ein("eqi,ei->eq", Xq - xf[:, None], t2)], -1) / hf[:, None, None]
            mq = eval2(Xiq, k)  # (E,Qe,nk2)
            gq = grad2_eval(Xiq, k)  # d/dxi
            dn = (gq[..., 0] * ein("ei,ei->e", t1, ne)[:, None, None]
                  + gq[..., 1] * ein("ei,ei->e", t2, ne)[:, None, None]) / hf[:, None, None]
            wl = wg[None, :] * le_len[:, None]  # (E,Qe)
            Kb0 += ein("eq,eqa->ea", wl, mq)
            # node dof indices along the edge
            for c in range(3):
                idx = [L.d1(v0, c)] + [L.d2(le, j, c) for j in range(k - 1)] + [L.d1(v1, c)]
                # v_c(s_q) = sum_i Lg[q,i] dof_i
                for i, di in enumerate(idx):
                    rhs_b[:, c, 1:, di] += ein("eq,eqa->ea", wl * Lg[None, :, i], dn[:, :, 1:])
                    rhs_b[:, c, 0, di] += ein("eq->e", wl * Lg[None, :, i])
        Ksys = Kst[:, :nk2, :nk2].copy()
        Ksys[:, 0, :] = Kb0
        for c in range(3):
            rhs = rhs_b[:, c].copy()
            # - int_f v_c Lap(m_b), Lap m_b in P_{k-2}
            rhs[:, 1:] -= ein("ab,eb...->ea...", lap2[1:, :nlo], DM[:, c]) / (hf ** 2)[:, None, None]
            a_c = np.linalg.solve(Ksys, rhs)  # (E,nk2,N)
            FM[:, lf, c, :nlo] = DM[:, c]
            FM[:, lf, c, nlo:] = ein("egb,egn->ebn", FMass[:, :nk2, nlo:], a_c)

    # ---------------- volume level
    Pv, Wv = element_quadrature(mesh, elems, qdeg)
    Xh = (Pv - xK[:, None]) / hK[:, None, None]
    M = eval3(Xh, k + 1)  # (E,Q,n3)
    n3 = dim3(k + 1)
    Mass = ein("eq,eqa,eqb->eab", Wv, M, M)  # (E,n3,n3)
    nk = dim3(k)
    nkm1 = dim3(k - 1)
    nkm2 = dim3(k - 2)
    sig = np.array([-1.0 if s == 0 else 1.0 for (a, s, vs, es) in LOCAL_FACES])
    normals = np.stack([_face_frame(mesh, elems, lf)[0] for lf in range(6)], 1)  # (E,6,3)
    areas = np.stack([_face_frame(mesh, elems, lf)[5] for lf in range(6)], 1)
    # BV[c,d,a] = int_dK v_c m_a n_d ; BP[c,a] = int_dK v_c m_a
    RFM = np.matmul(Rf.transpose(0, 1, 3, 2)[:, :, None], FM)  # (E,6,3,n3,N)
    BV = ein("f,efd,efcan->ecdan", sig, normals, RFM)
    BP = RFM.sum(1)
    BN = ein("eccan->ean", BV)  # int_dK (v.n) m_a
    # div v in P_{k-1}
    mu = np.zeros((E, nkm1, N))
    for lf in range(6):
        mu[:, 0, L.d3(lf, 0, 0)] = sig[lf] * areas[:, lf]
    for a in range(1, nkm1):
        mu[:, a, L.d5(a - 1)] = vK / hK
    dcoef = np.linalg.solve(Mass[:, :nkm1, :nkm1], mu)  # (E,nkm1,N)
    # int_K div v q for q monomial (deg <= k+1): DQ[a] = sum_b d_b Mass[b,a]
    DQ = ein("ebn,eba->ean", dcoef, Mass[:, :nkm1, :])  # (E,n3,N)
    GRADQ = -DQ + BN  # int_K v . grad_x q  (q = m_a, gradient in x)
    Qt, Rt = helmholtz_tables(k)
    # moments of v against e_c m_g for |g| <= k-2  (VM)
    VM = np.zeros((E, 3, max(nkm2, 1), N))
    ex3 = mono3(k + 1)
    for g in range(nkm2):
        j = sum(ex3[g])
        for c in range(3):
            q = Qt[j][c, g]  # over dim3(j+1)
            val = hK[:, None] * ein("a,ean->en", q, GRADQ[:, : len(q)])
            if j >= 1:
                r = Rt[j][c, g]  # (3, dim3(j-1)), homogeneous of degree j-1 <= k-3
                # int_K v.(xh ^ r) from the D4 moments
                for kk in range(3):
                    for gg in range(r.shape[1]):
                        if r[kk, gg] != 0.0:
                            for coef, dof in L.d4_terms(kk, gg):
                                val[:, dof] += coef * r[kk, gg] * vK
            VM[:, c, g] = val
    # Pi^nabla_k
    G3 = grad3_coef(k + 1)
    dMv = ein("dab,eqb->eqad", G3[:, :nk, :], M) / hK[:, None, None, None]
    KK = ein("eq,eqad,eqbd->eab", Wv, dMv, dMv)
    Pb = np.zeros((E, nk))
    for lf in range(6):
        P, W = face_quadrature(mesh, elems, lf, 2 * k + 1)
        Pb += ein("eq,eqa->ea", W, eval3((P - xK[:, None]) / hK[:, None, None], k))
    Ksys = KK.copy()
    Ksys[:, 0, :] = Pb
    lap3 = lap3_coef(k)
    bcoef = np.zeros((E, 3, nk, N))
    for c in range(3):
        rhs = np.zeros((E, nk, N))
        if nkm2 > 0:
            rhs -= ein("ab,ebn->ean", lap3[:, :nkm2], VM[:, c, :nkm2]) / (hK ** 2)[:, None, None]
        rhs += ein("dab,edbn->ean", G3[:, :nk, :], BV[:, c]) / hK[:, None, None]
        rhs[:, 0] = BP[:, c, 0]
        bcoef[:, c] = np.linalg.solve(Ksys, rhs)
    # Pi^0_{k-1} grad v : Gc[c,d] coefficients over P_{k-1}
    Gmom = np.zeros((E, 3, 3, nkm1, N))
    for c in range(3):
        for d in range(3):
            Gmom[:, c, d] = BV[:, c, d, :nkm1]
            if nkm2 > 0:
                Gmom[:, c, d] -= ein("ab,ebn->ean", G3[d, :nkm1, :nkm2], VM[:, c, :nkm2]) / hK[:, None, None]
    Minv1 = np.linalg.inv(Mass[:, :nkm1, :nkm1])
    Gc = np.matmul(Minv1[:, None, None], Gmom)
    # Pi^0_k v
    VMk = np.zeros((E, 3, nk, N))
    if nkm2 > 0:
        VMk[:, :, :nkm2] = VM[:, :, :nkm2]
    for g in range(nkm2, nk):
        j = sum(ex3[g])
        for c in range(3):
            q = Qt[j][c, g]
            val = hK[:, None] * ein("a,ean->en", q, GRADQ[:, : len(q)])
            r = Rt[j][c, g]  # (3, dim3(j-1)), degree j-1 in {k-2, k-1}
            # xh ^ r as polynomial of degree j (over dim3(j) monomials)
            W = wedge_coef(j - 1)  # (3, dim3(j-1), 3, dim3(j))
            wr = ein("kg,kgip->ip", r, W)  # (3 comps, dim3(j))
            # int Pi^nabla v . (xh^r) = sum_{c',b} bcoef[c',b] int m_b wr[c']
            T = ein("ip,ebp->eib", wr, Mass[:, :nk, : wr.shape[1]])
            val += ein("eibn,eib->en", bcoef, T)
            VMk[:, c, g] = val
    Minvk = np.linalg.inv(Mass[:, :nk, :nk])
    P0 = np.matmul(Minvk[:, None], VMk)
    # DoFs of the vector monomials e_c m_b (b over P_k): DOFM (E,N,3,nk)
    DOFM = np.zeros((E, N, 3, nk))
    mv = eval3((X8 - xK[:, None]) / hK[:, None, None], k)  # (E,8,nk)
    for lv in range(8):
        for c in range(3):
            DOFM[:, L.d1(lv, c), c] = mv[:, lv]
    for le, (ea, v0, v1, st) in enumerate(LOCAL_EDGES):
        for j in range(k - 1):
            t = enodes[1 + j]
            Xp = X8[:, v0] + t * (X8[:, v1] - X8[:, v0])
            mp = eval3((Xp - xK) / hK[:, None], k)
            for c in range(3):
                DOFM[:, L.d2(le, j, c), c] = mp
    for lf in range(6):
        nf, t1, t2, xf, hf, af = _face_frame(mesh, elems, lf)
        P, W = face_quadrature(mesh, elems, lf, 2 * k + 1)
        Xi = np.stack([ein("eqi,ei->eq", P - xf[:, None], t1),
                       ein("eqi,ei->eq", P - xf[:, None], t2)], -1) / hf[:, None, None]
        m2 = eval2(Xi, k - 2)
        m3 = eval3((P - xK[:, None]) / hK[:, None, None], k)
        FX = ein("eq,eqa,eqb->eab", W, m2, m3) / af[:, None, None]  # (E,nlo,nk)
        for b in range(nlo):
            for kind, vec in enumerate((nf, t1, t2)):
                DOFM[:, L.d3(lf, b, kind)] = vec[:, :, None] * FX[:, b][:, None, :]
    if L.nD4:
        Wd = wedge_coef(k - 3)  # xh ^ (e_kk m_g) : (3, dim3(k-3), 3, dim3(k-2))
        for i, (kk, gg) in enumerate(L.d4_pairs):
            wr = Wd[kk, gg]  # (3, dim3(k-2))
            for c in range(3):
                DOFM[:, L.d4(i), c] = ein("p,ebp->eb", wr[c], Mass[:, :nk, :dim3(k - 2)]) / vK[:, None]
    # D5 of e_c m_b: (hK/|K|) int (1/hK) d_c m_b m_a = (1/|K|) sum G3[c][b,g] Mass[g,a]
    for a in range(1, nkm1):
        for c in range(3):
            DOFM[:, L.d5(a - 1), c] = ein("bg,eg->eb", G3[c, :nk, :nk], Mass[:, :nk, a]) / vK[:, None]
    DPi = np.matmul(DOFM.reshape(E, N, -1), bcoef.reshape(E, -1, N))
    # consistency and stabilisation
    eps = 0.5 * (Gc + Gc.transpose(0, 2, 1, 3, 4))
    Y = np.matmul(Mass[:, None, None, :nkm1, :nkm1], eps).reshape(E, -1, N)
    Acons = np.matmul(eps.reshape(E, -1, N).transpose(0, 2, 1), Y)
    sigma = np.maximum(hK[:, None], ein("enn->en", Acons))
    IminD = eye[None] - DPi
    Astab = np.matmul(IminD.transpose(0, 2, 1), sigma[:, :, None] * IminD)
    A = nuK[:, None, None] * (Acons + Astab)
    out = {"A": A, "B": mu, "layout": L, "P0": P0}
    if force is not None:
        fq = force(Pv, elems)  # (E,Q,3)
        fm = ein("eq,eqc,eqa->eca", Wv, fq, M[:, :, :nk])
        out["F"] = ein("eca,ecan->en", fm, P0)
    if keep:
        out["PiN"] = bcoef
        out["Gc"] = Gc
        out["div"] = dcoef
        out["DOFM"] = DOFM
    return out


def interpolate(mesh, k, elems, u, divu=None):
    """Element-local DoF vectors (E,N) of a vector field u (callable on
    (...,3) points).  divu (callable) gives div u for D5 (zero if None)."""
    L = DofLayout(k)
    E = len(elems)
    X8 = mesh.verts[mesh.elem_verts[elems]]
    xK = mesh.elem_centroid[elems]
    hK = mesh.elem_diam[elems]
    vK = mesh.elem_vol[elems]
    out = np.zeros((E, L.N))
    uv = u(X8)
    for lv in range(8):
        for c in range(3):
            out[:, L.d1(lv, c)] = uv[:, lv, c]
    enodes = _edge_nodes(k)
    for le, (ea, v0, v1, st) in enumerate(LOCAL_EDGES):
        for j in range(k - 1):
            t = enodes[1 + j]
            up = u(X8[:, v0] + t * (X8[:, v1] - X8[:, v0]))
            for c in range(3):
                out[:, L.d2(le, j, c)] = up[:, c]
    for lf in range(6):
        nf, t1, t2, xf, hf, af = _face_frame(mesh, elems, lf)
        P, W = face_quadrature(mesh, elems, lf, 2 * k + 5)
        Xi = np.stack([ein("eqi,ei->eq", P - xf[:, None], t1),
                       ein("eqi,ei->eq", P - xf[:, None], t2)], -1) / hf[:, None, None]
        m2 = eval2(Xi, k - 2)
        uq = u(P)
        for kind, vec in enumerate((nf, t1, t2)):
            un = ein("eqc,ec->eq", uq, vec)
            mom = ein("eq,eq,eqb->eb", W, un, m2) / af[:, None]
            for b in range(L.nf2):
                out[:, L.d3(lf, b, kind)] = mom[:, b]
    Pv, Wv = element_quadrature(mesh, elems, 2 * k + 5)
    Xh = (Pv - xK[:, None]) / hK[:, None, None]
    if L.nD4:
        uq = u(Pv)
        M4 = eval3(Xh, k - 3)
        for i, (kk, gg) in enumerate(L.d4_pairs):
            ek = np.zeros(3)
            ek[kk] = 1.0
            wq = np.cross(Xh, ek) * M4[:, :, gg, None]
            out[:, L.d4(i)] = ein("eq,eqc,eqc->e", Wv, uq, wq) / vK
    if divu is not None:
        M = eval3(Xh, k - 1)
        dq = divu(Pv)
        for a in range(1, L.nP):
            out[:, L.d5(a - 1)] = hK / vK * ein("eq,eq,eq->e", Wv, dq, M[:, :, a])
    return out
