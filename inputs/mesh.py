"""Hexahedral meshes of the unit cube (the CUBE family of Sec. 7).

Vertices, edges, faces and elements of an n x n x n grid.  The optional
"plane jitter" moves every interior grid plane of each family
(x_a = i*h) to a tilted plane

    x_a = i*h + alpha + beta*(x_b - 1/2) + gamma*(x_c - 1/2),

so that every element stays a convex hexahedron with six planar faces
(assumptions A1-A3 of Sec. 2 need planar, star-shaped faces) and every
vertex moves by at most ``jitter*h`` per coordinate.  Boundary planes stay
fixed.  The draws come from ``numpy.random.default_rng(seed)`` in the order
axis x, y, z and, per axis, alpha, beta, gamma.
"""
import numpy as np

# element-local vertex (ix,iy,iz) -> ix + 2 iy + 4 iz
LOCAL_VERTS = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)])


def _other_axes(a):
    return [b for b in range(3) if b != a]


def _local_edges():
    """12 local edges: (axis, start local vertex, end local vertex)."""
    out = []
    for a in range(3):
        b, c = _other_axes(a)
        for o2 in range(2):
            for o1 in range(2):
                s = np.zeros(3, int)
                s[b] = o1
                s[c] = o2
                e = s.copy()
                e[a] = 1
                lv = lambda v: int(v[0] + 2 * v[1] + 4 * v[2])
                out.append((a, lv(s), lv(e), s.copy()))
    return out


def _local_faces():
    """6 local faces 2a+s: (axis, side s, 4 local vertices in cyclic order
    (b,c) offsets (0,0),(1,0),(1,1),(0,1), 4 local edges)."""
    edges = _local_edges()
    out = []
    for a in range(3):
        b, c = _other_axes(a)
        for s in range(2):
            vs = []
            for (o1, o2) in [(0, 0), (1, 0), (1, 1), (0, 1)]:
                v = np.zeros(3, int)
                v[a] = s
                v[b] = o1
                v[c] = o2
                vs.append(int(v[0] + 2 * v[1] + 4 * v[2]))
            es = []
            for le, (ea, v0, v1, st) in enumerate(edges):
                if ea != a and st[a] == s:
                    es.append(le)
            out.append((a, s, vs, es))
    return out


LOCAL_EDGES = _local_edges()
LOCAL_FACES = _local_faces()


class CubeMesh:
    """Structured hexahedral mesh of [0,1]^3 with n elements per side."""

    def __init__(self, n, jitter=0.0, seed=0):
        self.n = n
        self.h = 1.0 / n
        self.jitter = float(jitter)
        self.seed = seed
        n1 = n + 1
        I, J, K = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
        self.vidx = np.stack([I.ravel(order="F"), J.ravel(order="F"), K.ravel(order="F")], 1)
        # vertex id = i + n1*(j + n1*k): Fortran ravel of (i,j,k)
        self.verts = self._place_vertices()
        self.nV = n1 ** 3
        self.nK = n ** 3
        # edges
        self.edge_off = [0, n * n1 * n1, 2 * n * n1 * n1]
        self.nE = 3 * n * n1 * n1
        # faces
        self.face_off = [0, n1 * n * n, 2 * n1 * n * n]
        self.nF = 3 * n1 * n * n
        self._build_topology()
        self._build_face_geometry()
        self._build_element_geometry()

    # ---------------- ids
    def vid(self, i, j, k):
        n1 = self.n + 1
        return i + n1 * (j + n1 * k)

    def eid(self, a, i, j, k):
        n, n1 = self.n, self.n + 1
        d = [n1, n1, n1]
        d[a] = n
        return self.edge_off[a] + i + d[0] * (j + d[1] * k)

    def fid(self, a, i, j, k):
        n, n1 = self.n, self.n + 1
        d = [n, n, n]
        d[a] = n1
        return self.face_off[a] + i + d[0] * (j + d[1] * k)

    # ---------------- geometry
    def _place_vertices(self):
        n, h = self.n, self.h
        rng = np.random.default_rng(self.seed)
        J = self.jitter
        planes = []
        for a in range(3):
            al = np.zeros(n + 1)
            be = np.zeros(n + 1)
            ga = np.zeros(n + 1)
            if J > 0 and n > 1:
                al[1:n] = rng.uniform(-J / 3 * h, J / 3 * h, n - 1)
                be[1:n] = rng.uniform(-2 * J / 3 * h, 2 * J / 3 * h, n - 1)
                ga[1:n] = rng.uniform(-2 * J / 3 * h, 2 * J / 3 * h, n - 1)
            planes.append((al, be, ga))
        idx = self.vidx
        nv = idx.shape[0]
        M = np.zeros((nv, 3, 3))
        rhs = np.zeros((nv, 3))
        for a in range(3):
            b, c = _other_axes(a)
            al, be, ga = planes[a]
            ia = idx[:, a]
            M[:, a, a] = 1.0
            M[:, a, b] = -be[ia]
            M[:, a, c] = -ga[ia]
            rhs[:, a] = ia * h + al[ia] - 0.5 * be[ia] - 0.5 * ga[ia]
        X = np.linalg.solve(M, rhs[..., None])[..., 0]
        # boundary planes exactly on the cube faces
        X[idx == 0] = 0.0
        X[idx == n] = 1.0
        return X

    def _build_topology(self):
        n = self.n
        I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        ei = np.stack([I.ravel(order="F"), J.ravel(order="F"), K.ravel(order="F")], 1)
        self.eidx = ei  # element (i,j,k), element id = Fortran ravel
        ev = np.zeros((self.nK, 8), np.int64)
        for lv in range(8):
            o = LOCAL_VERTS[lv]
            ev[:, lv] = self.vid(ei[:, 0] + o[0], ei[:, 1] + o[1], ei[:, 2] + o[2])
        self.elem_verts = ev
        ee = np.zeros((self.nK, 12), np.int64)
        for le, (a, v0, v1, st) in enumerate(LOCAL_EDGES):
            o = LOCAL_VERTS[v0]
            ee[:, le] = self.eid(a, ei[:, 0] + o[0], ei[:, 1] + o[1], ei[:, 2] + o[2])
        self.elem_edges = ee
        ef = np.zeros((self.nK, 6), np.int64)
        for lf, (a, s, vs, es) in enumerate(LOCAL_FACES):
            o = LOCAL_VERTS[vs[0]]
            ef[:, lf] = self.fid(a, ei[:, 0] + o[0], ei[:, 1] + o[1], ei[:, 2] + o[2])
        self.elem_faces = ef
        # global edge endpoints and axis, global face vertices and axis
        n1 = n + 1
        ev0 = np.zeros((self.nE, 2), np.int64)
        eax = np.zeros(self.nE, np.int64)
        estart = np.zeros((self.nE, 3), np.int64)
        for a in range(3):
            d = [n1, n1, n1]
            d[a] = n
            A, B, C = np.meshgrid(np.arange(d[0]), np.arange(d[1]), np.arange(d[2]), indexing="ij")
            st = np.stack([A.ravel(order="F"), B.ravel(order="F"), C.ravel(order="F")], 1)
            ids = self.eid(a, st[:, 0], st[:, 1], st[:, 2])
            en = st.copy()
            en[:, a] += 1
            ev0[ids, 0] = self.vid(*st.T)
            ev0[ids, 1] = self.vid(*en.T)
            eax[ids] = a
            estart[ids] = st
        self.edge_verts = ev0
        self.edge_axis = eax
        self.edge_start = estart
        fv = np.zeros((self.nF, 4), np.int64)
        fax = np.zeros(self.nF, np.int64)
        fstart = np.zeros((self.nF, 3), np.int64)
        for a in range(3):
            b, c = _other_axes(a)
            d = [n, n, n]
            d[a] = n1
            A, B, C = np.meshgrid(np.arange(d[0]), np.arange(d[1]), np.arange(d[2]), indexing="ij")
            st = np.stack([A.ravel(order="F"), B.ravel(order="F"), C.ravel(order="F")], 1)
            ids = self.fid(a, st[:, 0], st[:, 1], st[:, 2])
            for q, (o1, o2) in enumerate([(0, 0), (1, 0), (1, 1), (0, 1)]):
                v = st.copy()
                v[:, b] += o1
                v[:, c] += o2
                fv[ids, q] = self.vid(*v.T)
            fax[ids] = a
            fstart[ids] = st
        self.face_verts = fv
        self.face_axis = fax
        self.face_start = fstart
        # boundary flags
        vb = np.any((self.vidx == 0) | (self.vidx == n), axis=1)
        self.vert_bnd = vb
        # an edge is on the boundary iff both its endpoints are on one cube face
        e_on = np.zeros(self.nE, bool)
        for a in range(3):
            for val in (0, n):
                on0 = self.vidx[ev0[:, 0], a] == val
                on1 = self.vidx[ev0[:, 1], a] == val
                e_on |= on0 & on1
        self.edge_bnd = e_on
        f_on = np.zeros(self.nF, bool)
        for a in range(3):
            sel = fax == a
            f_on[sel] = (fstart[sel, a] == 0) | (fstart[sel, a] == n)
        self.face_bnd = f_on

    def _build_face_geometry(self):
        X = self.verts[self.face_verts]  # (nF,4,3)
        P0, P1, P2, P3 = X[:, 0], X[:, 1], X[:, 2], X[:, 3]
        c1 = np.cross(P1 - P0, P2 - P0)
        c2 = np.cross(P2 - P0, P3 - P0)
        a1 = 0.5 * np.linalg.norm(c1, axis=1)
        a2 = 0.5 * np.linalg.norm(c2, axis=1)
        self.face_area = a1 + a2
        self.face_centroid = ((P0 + P1 + P2) / 3 * a1[:, None] + (P0 + P2 + P3) / 3 * a2[:, None]) / self.face_area[:, None]
        nrm = c1 + c2
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        ax = self.face_axis
        sgn = np.sign(nrm[np.arange(self.nF), ax])
        nrm *= sgn[:, None]
        t1 = P1 - P0
        t1 /= np.linalg.norm(t1, axis=1)[:, None]
        t2 = np.cross(nrm, t1)
        self.face_normal = nrm
        self.face_t1 = t1
        self.face_t2 = t2
        d = [np.linalg.norm(X[:, i] - X[:, j], axis=1) for i in range(4) for j in range(i + 1, 4)]
        self.face_diam = np.max(np.stack(d, 1), axis=1)

    def _build_element_geometry(self):
        X = self.verts[self.elem_verts]  # (nK,8,3)
        xb = X.mean(axis=1)
        vol = np.zeros(self.nK)
        cen = np.zeros((self.nK, 3))
        for (a, s, vs, es) in LOCAL_FACES:
            for tri in [(vs[0], vs[1], vs[2]), (vs[0], vs[2], vs[3])]:
                A, B, C = X[:, tri[0]], X[:, tri[1]], X[:, tri[2]]
                v = np.abs(np.einsum("ij,ij->i", A - xb, np.cross(B - xb, C - xb))) / 6.0
                vol += v
                cen += v[:, None] * (xb + A + B + C) / 4.0
        self.elem_vol = vol
        self.elem_centroid = cen / vol[:, None]
        d = [np.linalg.norm(X[:, i] - X[:, j], axis=1) for i in range(8) for j in range(i + 1, 8)]
        self.elem_diam = np.max(np.stack(d, 1), axis=1)
        self.elem_xbar = xb
