"""Box decomposition of a cube mesh into subdomains (Sec. 4.1-4.2).

Subdomains are boxes of elements cut along each axis at element indices
``cuts[a] = [0, c_1, ..., n]``.  An interface DoF is a free (non-Dirichlet)
velocity DoF shared by two or more subdomains.  Interface DoFs are grouped
into macro entities (faces, edges, vertices) by their position relative to
the cut planes; each entity carries the candidate primal functionals of the
recipe of Sec. 5.1:

* vertex: the three velocity components (all vertices are primal);
* edge:   integral averages of each component over the open macro edge;
* face:   integral averages of each component over the open macro face;
* flux:   the normal flux through the open macro face, eq. (primalfacen).

For a VEM function the flux through an element face f equals |f| times its
zeroth normal moment, so the face functionals only involve D3 DoFs.

The per-subdomain output is exactly what the hot path consumes: a CSR matrix
of the reduced local saddle problem, the DoF kinds, the global interface ids,
the element volumes of the pressure DoFs and the lifted right-hand side.
"""
import numpy as np
import scipy.sparse as sp
from .quadrature import gauss_lobatto_interior01, lobatto_weights01

KIND_INTERIOR, KIND_INTERFACE, KIND_PRESSURE = 0, 1, 2
ENT_VERTEX, ENT_EDGE, ENT_FACE = 0, 1, 2


def regular_cuts(n, parts):
    return [np.linspace(0, n, p + 1).round().astype(int) for p in parts]


def random_cuts(n, lo, hi, parts, seed):
    """Uneven cuts: per axis x, y, z draw piece sizes in [lo, hi] until they
    sum to n (numpy.random.default_rng(seed), one generator for all axes)."""
    rng = np.random.default_rng(seed)
    cuts = []
    for a in range(3):
        while True:
            s = rng.integers(lo, hi + 1, size=parts)
            if s.sum() == n:
                break
        cuts.append(np.concatenate([[0], np.cumsum(s)]).astype(int))
    return cuts


class Subdomain:
    def __init__(self):
        self.dofs = None  # global reduced ids
        self.kind = None
        self.gid = None
        self.pweight = None
        self.K = None  # scipy csr (local)
        self.rhs = None
        self.elems = None


class Decomposition:
    def __init__(self, pb, cuts, constraints=("vertex", "edge", "face", "flux")):
        self.pb = pb
        m, k, L = pb.mesh, pb.k, pb.L
        n = m.n
        self.cuts = [np.asarray(c, int) for c in cuts]
        self.parts = [len(c) - 1 for c in self.cuts]
        self.constraints = tuple(constraints)
        px, py, pz = self.parts
        self.nsub = px * py * pz
        # element -> subdomain
        seg = [np.searchsorted(self.cuts[a], m.eidx[:, a], side="right") - 1 for a in range(3)]
        self.elem_sub = seg[0] + px * (seg[1] + py * seg[2])
        # ---------------- owners of every reduced dof
        rm = pb.rmap
        pairs = np.unique(np.stack([rm.ravel(), np.repeat(self.elem_sub, rm.shape[1])], 1), axis=0)
        cnt = np.bincount(pairs[:, 0], minlength=pb.Nr)
        isvel = np.arange(pb.Nr) < pb.Nvr
        iface = isvel & (cnt >= 2) & ~pb.red_dir
        self.iface_red = np.nonzero(iface)[0]
        self.gid_of_red = -np.ones(pb.Nr, np.int64)
        # ---------------- entity keys for interface dofs
        info = self._dof_positions()
        keys = {}
        ent_of = np.zeros(len(self.iface_red), np.int64)
        for t, r in enumerate(self.iface_red):
            key = info[r]
            if key not in keys:
                keys[key] = len(keys)
            ent_of[t] = keys[key]
        klist = list(keys.keys())
        kinds = np.array([3 - sum(1 for ax in kk[1] if ax[0] == "seg") - 1 for kk in klist])
        # kinds: number of 'cut' axes: 1 face, 2 edge, 3 vertex -> ENT_FACE.. mapping
        ncut = np.array([sum(1 for ax in kk[1] if ax[0] == "cut") for kk in klist])
        ekind = np.where(ncut == 3, ENT_VERTEX, np.where(ncut == 2, ENT_EDGE, ENT_FACE))
        # order entities: vertices, edges, faces; within kind by key
        order = sorted(range(len(klist)), key=lambda i: (ekind[i], klist[i][1]))
        rank = np.empty(len(order), np.int64)
        rank[order] = np.arange(len(order))
        ent_of = rank[ent_of]
        self.ent_kind = ekind[order]
        self.ent_key = [klist[i] for i in order]
        # global interface ids: grouped by entity, sorted by reduced id inside
        perm = np.lexsort((self.iface_red, ent_of))
        self.iface_red = self.iface_red[perm]
        ent_of = ent_of[perm]
        self.gid_of_red[self.iface_red] = np.arange(len(self.iface_red))
        self.n_iface = len(self.iface_red)
        self.ent_dofs = [np.nonzero(ent_of == e)[0] for e in range(len(order))]
        self.ent_of_gid = ent_of
        # subdomains sharing each entity
        self.ent_subs = []
        for e in range(len(order)):
            r = self.iface_red[self.ent_dofs[e][0]]
            self.ent_subs.append(np.sort(pairs[pairs[:, 0] == r, 1]))
        self._build_constraints(info)
        self._build_subdomains()

    # ---------------------------------------------------------------------
    def _axis_pos_vertex(self, a, i):
        c = self.cuts[a]
        # a Neumann side of the cube is not a cut: DoFs on it belong to the
        # open faces and edges of the subdomains they touch
        if i == c[0] and 2 * a in self.pb.neumann_sides:
            return ("seg", 0)
        if i == c[-1] and 2 * a + 1 in self.pb.neumann_sides:
            return ("seg", len(c) - 2)
        j = np.searchsorted(c, i)
        if j < len(c) and c[j] == i:
            return ("cut", int(j))
        return ("seg", int(np.searchsorted(c, i, side="right") - 1))

    def _axis_pos_cell(self, a, i):
        c = self.cuts[a]
        return ("seg", int(np.searchsorted(c, i, side="right") - 1))

    def _dof_positions(self):
        """For every interface reduced dof: (type, ((axis pos) x3), extra)."""
        pb, m, L = self.pb, self.pb.mesh, self.pb.L
        info = {}
        for r in self.iface_red:
            full = pb.full_of_red[r]
            if full < pb.offE:
                v = full // 3
                idx = m.vidx[v]
                pos = tuple(self._axis_pos_vertex(a, idx[a]) for a in range(3))
            elif full < pb.offF:
                e = (full - pb.offE) // (3 * (pb.k - 1))
                a0 = m.edge_axis[e]
                st = m.edge_start[e]
                pos = tuple(self._axis_pos_cell(a, st[a]) if a == a0 else self._axis_pos_vertex(a, st[a])
                            for a in range(3))
            else:
                f = (full - pb.offF) // (3 * L.nf2)
                a0 = m.face_axis[f]
                st = m.face_start[f]
                pos = tuple(self._axis_pos_vertex(a, st[a]) if a == a0 else self._axis_pos_cell(a, st[a])
                            for a in range(3))
            info[r] = ("ent", pos)
        return info

    # ---------------------------------------------------------------------
    def _build_constraints(self, info):
        pb, m, L, k = self.pb, self.pb.mesh, self.pb.L, self.pb.k
        nodes = np.concatenate([[0.0], gauss_lobatto_interior01(k), [1.0]])
        wl = lobatto_weights01(nodes)
        self.ent_con = []
        self.ent_con_tag = []
        for e, dofs in enumerate(self.ent_dofs):
            red = self.iface_red[dofs]
            full = pb.full_of_red[red]
            nd = len(dofs)
            rows, tags = [], []
            kind = self.ent_kind[e]
            if kind == ENT_VERTEX:
                if "vertex" in self.constraints:
                    for c in range(3):
                        row = np.zeros(nd)
                        row[full % 3 == c] = 1.0
                        rows.append(row)
                        tags.append("vertex")
            elif kind == ENT_EDGE:
                if "edge" in self.constraints:
                    w = np.zeros(nd)
                    total = 0.0
                    for t, fdof in enumerate(full):
                        if fdof < pb.offE:  # grid vertex inside the macro edge
                            v = fdof // 3
                            # adjacent element edges of the macro edge
                            acc = 0.0
                            for ee in self._edges_of_vertex(v):
                                if self._edge_in_entity(ee, e):
                                    ln = np.linalg.norm(m.verts[m.edge_verts[ee, 1]] - m.verts[m.edge_verts[ee, 0]])
                                    acc += ln * (wl[0] if m.edge_verts[ee, 0] == v else wl[-1])
                            w[t] = acc
                        else:
                            ee = (fdof - pb.offE) // (3 * (k - 1))
                            j = ((fdof - pb.offE) % (3 * (k - 1))) // 3
                            ln = np.linalg.norm(m.verts[m.edge_verts[ee, 1]] - m.verts[m.edge_verts[ee, 0]])
                            w[t] = ln * wl[1 + j]
                    for ee in self._entity_edges(e):
                        total += np.linalg.norm(m.verts[m.edge_verts[ee, 1]] - m.verts[m.edge_verts[ee, 0]])
                    for c in range(3):
                        row = np.where(full % 3 == c, w, 0.0) / total
                        rows.append(row)
                        tags.append("edge")
            else:
                # face dofs of zeroth moment
                fr = full - pb.offF
                isF = full >= pb.offF
                f = np.where(isF, fr // (3 * L.nf2), -1)
                b = np.where(isF, (fr % (3 * L.nf2)) // 3, -1)
                kd = np.where(isF, fr % 3, -1)
                sel = isF & (b == 0)
                fa = np.where(sel, m.face_area[np.maximum(f, 0)], 0.0)
                area = fa[sel & (kd == 0)].sum()
                if "face" in self.constraints:
                    for c in range(3):
                        row = np.zeros(nd)
                        for kind3, vec in enumerate((m.face_normal, m.face_t1, m.face_t2)):
                            s2 = sel & (kd == kind3)
                            row[s2] = fa[s2] * vec[f[s2], c]
                        rows.append(row / area)
                        tags.append("face")
                if "flux" in self.constraints:
                    row = np.zeros(nd)
                    s2 = sel & (kd == 0)
                    row[s2] = fa[s2]
                    rows.append(row / area)
                    tags.append("flux")
            self.ent_con.append(np.array(rows).reshape(len(rows), nd))
            self.ent_con_tag.append(tags)

    def _edges_of_vertex(self, v):
        m = self.pb.mesh
        if not hasattr(self, "_v2e"):
            ev = m.edge_verts
            order = np.argsort(np.concatenate([ev[:, 0], ev[:, 1]]), kind="stable")
            eids = np.concatenate([np.arange(m.nE), np.arange(m.nE)])[order]
            vs = np.concatenate([ev[:, 0], ev[:, 1]])[order]
            ptr = np.searchsorted(vs, np.arange(m.nV + 1))
            self._v2e = (ptr, eids)
        ptr, eids = self._v2e
        return eids[ptr[v]:ptr[v + 1]]

    def _entity_edges(self, e):
        """Element edges lying inside macro edge e."""
        if not hasattr(self, "_eedge_cache"):
            self._eedge_cache = {}
        if e in self._eedge_cache:
            return self._eedge_cache[e]
        m = self.pb.mesh
        key = self.ent_key[e][1]
        ax = [i for i in range(3) if key[i][0] == "seg"][0]
        sel = m.edge_axis == ax
        ok = sel.copy()
        for a in range(3):
            if a == ax:
                s = key[a][1]
                ok &= (m.edge_start[:, a] >= self.cuts[a][s]) & (m.edge_start[:, a] < self.cuts[a][s + 1])
            else:
                ok &= m.edge_start[:, a] == self.cuts[a][key[a][1]]
        res = np.nonzero(ok)[0]
        self._eedge_cache[e] = res
        return res

    def _edge_in_entity(self, ee, e):
        return ee in set(self._entity_edges(e).tolist())

    # ---------------------------------------------------------------------
    def _build_subdomains(self):
        pb = self.pb
        self.subs = []
        for s in range(self.nsub):
            el = np.nonzero(self.elem_sub == s)[0]
            rm = pb.rmap[el]
            d = np.unique(rm.ravel())
            d = d[~pb.red_dir[d]]
            loc = -np.ones(pb.Nr, np.int64)
            loc[d] = np.arange(len(d))
            lr = loc[rm]
            ok = lr >= 0
            nl = pb.nloc
            rows = np.repeat(lr, nl, axis=1)
            cols = np.tile(lr, (1, nl))
            vals = pb.Ke[el]
            msk = (rows >= 0) & (cols >= 0)
            K = sp.coo_matrix((vals.reshape(len(el), -1)[msk.reshape(len(el), -1)],
                               (rows[msk], cols[msk])), shape=(len(d), len(d))).tocsr()
            K.sum_duplicates()
            K.sort_indices()
            rhs = np.zeros(len(d))
            np.add.at(rhs, lr[ok], pb.ge[el][ok])
            kind = np.full(len(d), KIND_INTERIOR, np.int32)
            kind[d >= pb.Nvr] = KIND_PRESSURE
            g = self.gid_of_red[d]
            kind[g >= 0] = KIND_INTERFACE
            pw = np.zeros(len(d))
            pw[d >= pb.Nvr] = pb.mesh.elem_vol[d[d >= pb.Nvr] - pb.Nvr]
            sd = Subdomain()
            sd.dofs, sd.kind, sd.gid, sd.pweight, sd.K, sd.rhs, sd.elems = d, kind, g.astype(np.int64), pw, K, rhs, el
            sd.part = self._sub_boxes(s, el, lr, kind)
            sd.has_p0 = self._sub_has_p0(s)
            self.subs.append(sd)
        self.sub_vol = np.array([pb.mesh.elem_vol[sd.elems].sum() for sd in self.subs])

    def _sub_has_p0(self, s):
        """Whether subdomain s keeps its constant pressure p0 as a global
        unknown: true unless one of its sides lies on a Neumann side of the
        cube.  There the open boundary DoFs carry flux, so the constant
        pressure couples to the subdomain's own interior problem and is
        eliminated with the other element pressures."""
        px, py, pz = self.parts
        seg = (s % px, (s // px) % py, s // (px * py))
        for a in range(3):
            if seg[a] == 0 and 2 * a in self.pb.neumann_sides:
                return False
            if seg[a] == self.parts[a] - 1 and 2 * a + 1 in self.pb.neumann_sides:
                return False
        return True

    def _sub_boxes(self, s, el, lr, kind):
        """Geometric one-level nested dissection of subdomain s: its box of
        elements is halved along every axis with at least two elements,
        giving up to eight sub-boxes.  Per local DoF: the sub-box whose
        elements alone carry it (its interior velocities and element
        pressures), or -1 for the separator DoFs shared by elements of
        several sub-boxes and for the interface DoFs."""
        m = self.pb.mesh
        px, py, pz = self.parts
        seg = (s % px, (s // px) % py, s // (px * py))
        nb, sub = [], np.zeros(len(el), np.int64)
        mult = 1
        for a in range(3):
            c0, c1 = self.cuts[a][seg[a]], self.cuts[a][seg[a] + 1]
            side = c1 - c0
            pieces = 2 if side >= 2 else 1
            half = (m.eidx[el, a] - c0) >= side // 2 if pieces == 2 else np.zeros(len(el), bool)
            sub += mult * half.astype(np.int64)
            mult *= pieces
        ok = lr >= 0
        b = np.broadcast_to(sub[:, None], lr.shape)[ok]
        idx = lr[ok]
        lo = np.full(len(kind), np.iinfo(np.int64).max)
        hi = np.full(len(kind), -1)
        np.minimum.at(lo, idx, b)
        np.maximum.at(hi, idx, b)
        part = np.where(lo == hi, lo, -1).astype(np.int32)
        part[kind == KIND_INTERFACE] = -1
        return part

    # ---------------------------------------------------------------------
    def interface_solution(self, xred):
        """(u_Gamma by interface id, p0 per subdomain that keeps one) of a
        reduced-system vector: p0_i is the volume-weighted mean pressure of
        subdomain i."""
        pb = self.pb
        uG = xred[self.iface_red]
        pK = xred[pb.Nvr:]
        p0 = np.array([np.dot(pb.mesh.elem_vol[sd.elems], pK[sd.elems]) / self.sub_vol[i]
                       for i, sd in enumerate(self.subs) if sd.has_p0])
        return uG, p0

    # ---------------------------------------------------------------------
    def workload(self):
        """Plain-data description of the decomposed problem (what the hot
        path consumes).  Subdomain matrices are local CSR (both triangles)."""
        subs = []
        for sd in self.subs:
            subs.append({"indptr": sd.K.indptr.astype(np.int64), "indices": sd.K.indices.astype(np.int64),
                         "data": sd.K.data.astype(np.float64), "kind": sd.kind.astype(np.int32),
                         "gid": sd.gid.astype(np.int64), "pweight": sd.pweight.astype(np.float64),
                         "rhs": sd.rhs.astype(np.float64), "part": sd.part.astype(np.int32)})
        ents = []
        for e in range(len(self.ent_dofs)):
            ents.append({"kind": int(self.ent_kind[e]), "gids": self.ent_dofs[e].astype(np.int64),
                         "con": np.ascontiguousarray(self.ent_con[e], dtype=np.float64)})
        return {"n_iface": int(self.n_iface), "subs": subs, "ents": ents,
                "pressure_kernel": bool(self.pb.pressure_kernel),
                "has_p0": np.array([int(sd.has_p0) for sd in self.subs], np.int32)}
