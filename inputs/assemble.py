"""Global numbering, assembly, boundary conditions and the reduced scheme.

Global velocity DoFs: 3 per vertex, 3(k-1) per edge, 3*dim P_{k-2}(f) per
face, then the element-internal D4 and D5 moments; pressures: dim P_{k-1}
per element (Sec. 3, Q_h).  Dirichlet DoFs (vertices, edges and faces on the
boundary) are eliminated into the right-hand side.  By default the whole
boundary is no-slip; `neumann_sides` lists sides of the cube (0..5: x = 0,
x = 1, y = 0, y = 1, z = 0, z = 1) that carry the natural condition with zero
traction instead (Sec. 7 solves with Neumann conditions on two faces and
no-slip on the other four): the entities inside such a side stay free, those
on its boundary shared with a no-slip side stay Dirichlet.  With a Neumann
side the constant pressure is no longer a kernel of the problem.

Reduced scheme (the remark closing Sec. 3.2): the constraint rows of the
non-constant pressures force D5(u_h) = 0, and those pressures only appear in
the D5 momentum rows, so deleting the D5 velocity DoFs and the non-constant
pressures leaves a principal submatrix with the same discrete velocity.
The reduced system (velocity D1-D4 + one constant pressure per element) is
what the subdomain solvers receive.
"""
import numpy as np
import scipy.sparse as sp
from .vem import DofLayout, element_matrices, interpolate
from .poly import dim3, eval3
from .quadrature import tet_rule


def dirichlet_entities(m, neumann_sides=()):
    """Vertices, edges and faces of the cube mesh lying on a no-slip side
    (side 2a + t: x_a = 0 for t = 0, x_a = n for t = 1): a vertex on any such
    side, an edge with both endpoints on one, a boundary face on one."""
    n = m.n
    sides = [s for s in range(6) if s not in tuple(neumann_sides)]

    def on(idx, s):
        a, t = divmod(s, 2)
        return idx[..., a] == (0 if t == 0 else n)

    vb = np.zeros(m.nV, bool)
    eb = np.zeros(m.nE, bool)
    fb = np.zeros(m.nF, bool)
    ev = m.edge_verts
    for s in sides:
        vb |= on(m.vidx, s)
        eb |= on(m.vidx[ev[:, 0]], s) & on(m.vidx[ev[:, 1]], s)
        a, t = divmod(s, 2)
        sel = m.face_axis == a
        fb[sel] |= m.face_start[sel, a] == (0 if t == 0 else n)
    return vb, eb, fb


def u_curl(X):
    """u = curl(psi), psi = sin(pi x) sin(pi y) sin(pi z) (1,1,1)."""
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    pi = np.pi
    sx, sy, sz = np.sin(pi * x), np.sin(pi * y), np.sin(pi * z)
    cx, cy, cz = np.cos(pi * x), np.cos(pi * y), np.cos(pi * z)
    dx = pi * cx * sy * sz
    dy = pi * sx * cy * sz
    dz = pi * sx * sy * cz
    return np.stack([dy - dz, dz - dx, dx - dy], -1)


def grad_u_curl(X):
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    pi = np.pi
    s = [np.sin(pi * x), np.sin(pi * y), np.sin(pi * z)]
    c = [np.cos(pi * x), np.cos(pi * y), np.cos(pi * z)]
    # second derivatives of s = prod sin
    H = np.zeros(X.shape[:-1] + (3, 3))
    for i in range(3):
        for j in range(3):
            f = np.ones_like(x) * pi * pi
            for t in range(3):
                if t == i and t == j:
                    f = f * (-s[t])
                elif t == i or t == j:
                    f = f * c[t]
                else:
                    f = f * s[t]
            H[..., i, j] = f
    # u_0 = d_y s - d_z s, u_1 = d_z s - d_x s, u_2 = d_x s - d_y s
    G = np.zeros_like(H)
    G[..., 0, :] = H[..., 1, :] - H[..., 2, :]
    G[..., 1, :] = H[..., 2, :] - H[..., 0, :]
    G[..., 2, :] = H[..., 0, :] - H[..., 1, :]
    return G


def zero_div(X):
    return np.zeros(X.shape[:-1])


def _chunk_matrices(args):
    m, k, el = args
    out = element_matrices(m, k, el, 1.0)
    return out["A"], out["B"], out["P0"]


def load_vector(m, k, el, P0, force):
    """(f_h, phi_i)_K = int_K f . Pi^0_k phi_i, by quadrature of f against the
    scaled monomials of degree <= k."""
    from .vem import element_quadrature
    P, W = element_quadrature(m, el, 2 * k + 1)
    Xh = (P - m.elem_centroid[el][:, None]) / m.elem_diam[el][:, None, None]
    M = eval3(Xh, k)
    fq = force(P, el)
    fm = np.einsum("eq,eqc,eqa->eca", W, fq, M, optimize=True)
    return np.einsum("eca,ecan->en", fm, P0, optimize=True)


class Problem:
    """A VEM Stokes problem on a CubeMesh.

    nu: scalar or per-element array.  force(P (E,Q,3), elems) -> (E,Q,3).
    uD: Dirichlet velocity (callable), divD: its divergence (for D5).
    keep_full: also keep the full (unreduced) element matrices.
    """

    def __init__(self, mesh, k, nu=1.0, force=None, uD=None, divD=None, keep_full=False,
                 chunk=None, workers=None, progress=None, element_data=None, neumann_sides=()):
        self.mesh, self.k = mesh, k
        self.neumann_sides = tuple(sorted(set(int(s) for s in neumann_sides)))
        assert all(0 <= s < 6 for s in self.neumann_sides) and len(self.neumann_sides) < 6
        # the constant pressure is a kernel only with no-slip on the whole boundary
        self.pressure_kernel = len(self.neumann_sides) == 0
        L = DofLayout(k)
        self.L = L
        nuK = np.asarray(nu, float) if np.ndim(nu) else np.full(mesh.nK, float(nu))
        self.nu = nuK
        default_load = force is None
        if force is None:
            force = lambda P, el: 1.5 * np.pi ** 2 * nuK[el][:, None, None] * u_curl(P)
        if uD is None:
            uD, divD = u_curl, zero_div
        self.force = force
        m = mesh
        # ---------------- global numbering (full)
        self.offE = 3 * m.nV
        self.offF = self.offE + 3 * (k - 1) * m.nE
        self.offI = self.offF + 3 * L.nf2 * m.nF
        self.Nv = self.offI + L.nI * m.nK
        self.Np = L.nP * m.nK
        gm = np.zeros((m.nK, L.N), np.int64)
        for lv in range(8):
            for c in range(3):
                gm[:, L.d1(lv, c)] = 3 * m.elem_verts[:, lv] + c
        for le in range(12):
            for j in range(k - 1):
                for c in range(3):
                    gm[:, L.d2(le, j, c)] = self.offE + 3 * ((k - 1) * m.elem_edges[:, le] + j) + c
        for lf in range(6):
            for b in range(L.nf2):
                for kind in range(3):
                    gm[:, L.d3(lf, b, kind)] = self.offF + 3 * (L.nf2 * m.elem_faces[:, lf] + b) + kind
        for i in range(L.nI):
            gm[:, L.off4 + i] = self.offI + L.nI * np.arange(m.nK) + i
        self.gmap = gm
        dir_mask = np.zeros(self.Nv, bool)
        vb, eb, fb = dirichlet_entities(m, self.neumann_sides)
        for c in range(3):
            dir_mask[3 * np.nonzero(vb)[0] + c] = True
        for j in range(3 * (k - 1)):
            dir_mask[self.offE + 3 * (k - 1) * np.nonzero(eb)[0] + j] = True
        for j in range(3 * L.nf2):
            dir_mask[self.offF + 3 * L.nf2 * np.nonzero(fb)[0] + j] = True
        self.dir_mask = dir_mask
        # ---------------- reduced numbering: velocity without D5, element constants
        keep_local = np.ones(L.N, bool)
        keep_local[L.off5:] = False
        self.keep_local = keep_local
        isD5 = np.zeros(self.Nv, bool)
        for i in range(L.nD4, L.nI):
            isD5[self.offI + L.nI * np.arange(m.nK) + i] = True
        vred = np.nonzero(~isD5)[0]
        self.red_of_full = -np.ones(self.Nv, np.int64)
        self.red_of_full[vred] = np.arange(len(vred))
        self.full_of_red = vred
        self.Nvr = len(vred)
        self.Nr = self.Nvr + m.nK  # + one constant pressure per element
        self.red_dir = np.zeros(self.Nr, bool)
        self.red_dir[: self.Nvr] = dir_mask[vred]
        nloc = int(keep_local.sum())
        self.nloc = nloc + 1  # reduced local size incl. the element pressure
        rmap = np.zeros((m.nK, self.nloc), np.int64)
        rmap[:, :nloc] = self.red_of_full[gm[:, keep_local]]
        rmap[:, nloc] = self.Nvr + np.arange(m.nK)
        self.rmap = rmap
        # ---------------- Dirichlet data (full dof values on the boundary)
        self.uD = np.zeros(self.Nv)
        # ---------------- element matrices
        if chunk is None:
            chunk = 512 if k == 2 else 128
        Ke = np.zeros((m.nK, self.nloc, self.nloc))
        Fe = np.zeros((m.nK, self.nloc))
        self.full = {} if keep_full else None
        if keep_full:
            self.full = {"A": np.zeros((m.nK, L.N, L.N)), "B": np.zeros((m.nK, L.nP, L.N)),
                         "F": np.zeros((m.nK, L.N))}
        # element_data: (A, B, F) of every element for nu = 1 and the default
        # load, computed elsewhere (A and F scale with nu_K)
        if element_data is not None:
            assert default_load, "element_data holds the default load"
        uniform = (m.jitter == 0.0) and element_data is None
        if element_data is not None:
            pass
        elif uniform:
            ref = element_matrices(m, k, np.array([0]), 1.0)
        elif workers is None or workers > 1:
            chunks = [np.arange(s, min(m.nK, s + chunk)) for s in range(0, m.nK, chunk)]
            import concurrent.futures as cf
            import os
            nw = workers or min(16, os.cpu_count() or 1)
            results = []
            every = max(1, len(chunks) // 8)
            with cf.ProcessPoolExecutor(nw) as ex:
                for r in ex.map(_chunk_matrices, [(m, k, el) for el in chunks]):
                    results.append(r)
                    if progress and len(results) % every == 0:
                        progress("element matrices: %d of %d chunks" % (len(results), len(chunks)))
        for ci, s in enumerate(range(0, m.nK, chunk)):
            el = np.arange(s, min(m.nK, s + chunk))
            if uniform:
                A = np.broadcast_to(ref["A"], (len(el),) + ref["A"].shape[1:]) * nuK[el][:, None, None]
                B = np.broadcast_to(ref["B"], (len(el),) + ref["B"].shape[1:])
                P0 = np.broadcast_to(ref["P0"], (len(el),) + ref["P0"].shape[1:])
            elif element_data is None:
                if workers is None or workers > 1:
                    A, B, P0 = results[ci]
                else:
                    A, B, P0 = _chunk_matrices((m, k, el))
                A = A * nuK[el][:, None, None]
            if element_data is not None:
                A = element_data[0][el] * nuK[el][:, None, None]
                B = element_data[1][el]
                F = element_data[2][el] * nuK[el][:, None]
            else:
                F = load_vector(m, k, el, P0, force)
            Ke[el, :nloc, :nloc] = A[:, keep_local][:, :, keep_local]
            Ke[el, nloc, :nloc] = B[:, 0, keep_local]
            Ke[el, :nloc, nloc] = B[:, 0, keep_local]
            Fe[el, :nloc] = F[:, keep_local]
            # boundary interpolant: element dofs of uD
            onb = np.any(dir_mask[gm[el]], axis=1)
            if np.any(onb):
                eb = el[onb]
                d = interpolate(m, k, eb, uD, divD)
                g = gm[eb]
                msk = dir_mask[g]
                self.uD[g[msk]] = d[msk]
            if keep_full:
                self.full["A"][el] = A
                self.full["B"][el] = B
                self.full["F"][el] = F
        self.Ke = Ke
        self.Fe = Fe
        # Dirichlet values in reduced numbering
        self.uD_red = np.zeros(self.Nr)
        self.uD_red[: self.Nvr] = self.uD[vred]
        # element-level lifted rhs: g_e = F_e - K_e[:, D] uD
        ud_e = self.uD_red[rmap] * self.red_dir[rmap]
        self.ge = Fe - np.einsum("eij,ej->ei", Ke, ud_e)

    # ---------------------------------------------------------------- global
    def reduced_system(self):
        """Assembled reduced system on the free DoFs: (K csr, g, free index)."""
        rm = self.rmap
        rows = np.repeat(rm, self.nloc, axis=1).ravel()
        cols = np.tile(rm, (1, self.nloc)).ravel()
        K = sp.coo_matrix((self.Ke.ravel(), (rows, cols)), shape=(self.Nr, self.Nr)).tocsr()
        g = np.zeros(self.Nr)
        np.add.at(g, rm.ravel(), self.ge.ravel())
        free = np.nonzero(~self.red_dir)[0]
        return K[free][:, free], g[free], free

    def pressure_mean_row(self):
        """Row w with w . p = int_Omega p for element-constant pressures."""
        return self.mesh.elem_vol.copy()

    def solve_reduced_direct(self):
        """Sparse direct solve of the reduced system, with the mean-zero
        pressure constraint as a Lagrange multiplier when the constant
        pressure is a kernel (no-slip everywhere).  Returns the full reduced
        vector (Dirichlet values included)."""
        K, g, free = self.reduced_system()
        nfree = len(free)
        from scipy.sparse.linalg import spsolve
        if self.pressure_kernel:
            w = np.zeros(nfree)
            pf = free >= self.Nvr
            w[pf] = self.mesh.elem_vol[free[pf] - self.Nvr]
            Kb = sp.bmat([[K, sp.csr_matrix(w[:, None])], [sp.csr_matrix(w[None, :]), None]]).tocsc()
            x = spsolve(Kb, np.concatenate([g, [0.0]]))
        else:
            x = spsolve(K.tocsc(), g)
        out = self.uD_red.copy()
        out[free] = x[:nfree]
        return out

    def full_system_direct(self):
        """Solve the unreduced system (all velocity DoFs incl. D5 and all
        P_{k-1} pressures), mean-zero pressure by a multiplier when the
        constant pressure is a kernel.  Small meshes only (requires
        keep_full).  Returns (u full, p full)."""
        from scipy.sparse.linalg import spsolve
        m, L = self.mesh, self.L
        A, B, F = self.full["A"], self.full["B"], self.full["F"]
        gm = self.gmap
        rows = np.repeat(gm, L.N, axis=1).ravel()
        cols = np.tile(gm, (1, L.N)).ravel()
        Ag = sp.coo_matrix((A.ravel(), (rows, cols)), shape=(self.Nv, self.Nv)).tocsr()
        pm = L.nP * np.arange(m.nK)[:, None] + np.arange(L.nP)[None, :]
        rows = np.repeat(pm, L.N, axis=1).ravel()
        cols = np.tile(gm, (1, L.nP)).ravel()
        Bg = sp.coo_matrix((B.ravel(), (rows, cols)), shape=(self.Np, self.Nv)).tocsr()
        Fg = np.zeros(self.Nv)
        np.add.at(Fg, gm.ravel(), F.ravel())
        free = np.nonzero(~self.dir_mask)[0]
        rhs_u = Fg - Ag @ self.uD
        rhs_p = -(Bg @ self.uD)
        # mean of pressure: int m_a over each element
        wp = np.zeros(self.Np)
        xK, hK = m.elem_centroid, m.elem_diam
        lam, wq = tet_rule(2 * self.k)
        from .vem import element_quadrature
        P, W = element_quadrature(m, np.arange(m.nK), 2 * self.k)
        Mq = eval3((P - xK[:, None]) / hK[:, None, None], self.k - 1)
        wp = np.einsum("eq,eqa->ea", W, Mq).ravel()
        if self.pressure_kernel:
            Kf = sp.bmat([[Ag[free][:, free], Bg[:, free].T, None],
                          [Bg[:, free], None, sp.csr_matrix(wp[:, None])],
                          [None, sp.csr_matrix(wp[None, :]), None]]).tocsc()
            rhs = np.concatenate([rhs_u[free], rhs_p, [0.0]])
        else:
            Kf = sp.bmat([[Ag[free][:, free], Bg[:, free].T],
                          [Bg[:, free], sp.csr_matrix((self.Np, self.Np))]]).tocsc()
            rhs = np.concatenate([rhs_u[free], rhs_p])
        x = spsolve(Kf, rhs)
        u = self.uD.copy()
        u[free] = x[: len(free)]
        p = x[len(free): len(free) + self.Np]
        return u, p


def with_viscosity(pb, nuK):
    """The problem `pb` (built with nu = 1 and the default load) with the
    element viscosities nuK: the velocity blocks of the element matrices and
    the load (f is proportional to nu_K) scale by nu_K, the divergence rows do
    not, and the Dirichlet lifting is recomputed.  Shares the mesh, the
    numbering and the unit element matrices with `pb`."""
    import copy
    assert np.all(pb.nu == 1.0), "the base problem must have nu = 1"
    q = copy.copy(pb)
    nuK = np.asarray(nuK, float)
    n = pb.nloc - 1
    Ke = pb.Ke.copy()
    Ke[:, :n, :n] *= nuK[:, None, None]
    Fe = pb.Fe.copy()
    Fe[:, :n] *= nuK[:, None]
    q.Ke, q.Fe, q.nu = Ke, Fe, nuK
    ud_e = pb.uD_red[pb.rmap] * pb.red_dir[pb.rmap]
    q.ge = Fe - np.einsum("eij,ej->ei", Ke, ud_e)
    return q
