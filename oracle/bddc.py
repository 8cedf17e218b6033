"""FP64 reference BDDC for the interface saddle-point problem (Sec. 4).

Test infrastructure only (the CPU oracle): the tests, the smoke check and
the CPU-baseline leg of the benchmark use it; the library never does.

Input: the plain-data workload (per-subdomain reduced local saddle matrices
in CSR, DoF kinds, global interface ids, element volumes of the pressure
DoFs, local right-hand sides; per-entity constraint functionals).

Steps, in the paper's order:

* interior/interface split and Q = Q_I + Q_0 (eq. discVQ): element-constant
  pressures of subdomain i are split into the volume-weighted mean-zero part
  Q_I and the constant p0_i.  Here Q_I is imposed with a Lagrange multiplier
  on the weighted mean, which spans the same space as any explicit basis;
* Dirichlet problems (eq. uipi) and the local Stokes Schur complement
  S_Gamma^(i) (eq. firstSchur), formed densely from sparse-LU solves;
  condensed right-hand side g (eq. globInt);
* the global interface operator S_hat = sum R^T [[S, B0^T],[B0, 0]] R
  (eqs. globInt, ScapGdef);
* change of basis making each primal functional an explicit DoF (Sec. 4.3):
  per entity an orthonormal [Q_Pi Q_Delta] from the SVD of its constraint
  rows, dependent rows dropped (Sec. 5.1);
* scaling: deluxe D_E^(m) = (sum_l Sbar_E^(l))^-1 Sbar_E^(m) on the dual
  coordinates of each entity (Sec. 6), or counting 1/card (eq. pseudoinv);
* M^-1 = Rt_D^T St^-1 Rt_D (eq. BDDCprec), split into local constrained
  Neumann solves and a coarse saddle problem in the primal variables and
  p0; with no-slip boundaries the coarse problem inherits the constant-p0
  kernel and is bordered with the constraint sum |Omega_i| p0_i = 0.

Neumann sides (Sec. 7; wl["pressure_kernel"] false).  The split Q_I + Q_0
rests on a subdomain's constant pressure testing only the fluxes of its
interface DoFs, which holds when the rest of its boundary is no-slip (the
fluxes of its other DoFs cancel between its elements).  A subdomain with a
side on a Neumann face of the domain has open boundary DoFs whose flux the
constant pressure also tests, so there p0 belongs to the subdomain's own
Dirichlet problem: it keeps all its element pressures local and adds no p0
to the interface problem (wl["has_p0"][i] = 0).  The coarse problem then
has no constant-pressure kernel and no border row.  This reading is the
oracle's own; the paper does not spell the split out for Neumann sides.
"""
import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla
from scipy.sparse.linalg import splu

KIND_INTERIOR, KIND_INTERFACE, KIND_PRESSURE = 0, 1, 2


class _DenseLU:
    """Dense LU (LAPACK, partial pivoting) with the splu solve interface."""

    def __init__(self, K):
        self.f = sla.lu_factor(K.toarray())

    def solve(self, b):
        return sla.lu_solve(self.f, b)


class LocalSchur:
    """Static condensation of one subdomain (eqs. uipi, firstSchur).

    condense=False keeps only the factorisation of the Dirichlet problem
    (enough for recover), without forming S_Gamma^(i) and g.
    dense=True factors the Dirichlet matrix with a dense LU instead of the
    sparse one: a second FP64 evaluation of the same formulas, which
    measures how far rounding alone moves the results on ill-conditioned
    problems.
    """

    def __init__(self, sd, condense=True, dense=False, has_p0=True):
        n = len(sd["kind"])
        self.has_p0 = bool(has_p0)
        K = sp.csr_matrix((sd["data"], sd["indices"], sd["indptr"]), shape=(n, n))
        kind = sd["kind"]
        self.iv = np.nonzero(kind == KIND_INTERIOR)[0]
        self.ig = np.nonzero(kind == KIND_INTERFACE)[0]
        self.ip = np.nonzero(kind == KIND_PRESSURE)[0]
        self.gid = sd["gid"][self.ig]
        w = sd["pweight"][self.ip]
        self.w = w
        nv, npr = len(self.iv), len(self.ip)
        A_II = K[self.iv][:, self.iv]
        Bp_I = K[self.ip][:, self.iv]
        A_IG = K[self.iv][:, self.ig]
        Bp_G = K[self.ip][:, self.ig]
        self.A_GG = K[self.ig][:, self.ig].toarray()
        if self.has_p0:
            # K_II' = [[A, Bp^T, 0], [Bp, 0, w], [0, w^T, 0]]: pressures in Q_I
            Kii = sp.bmat([[A_II, Bp_I.T, None],
                           [Bp_I, None, sp.csr_matrix(w[:, None])],
                           [None, sp.csr_matrix(w[None, :]), None]]).tocsc()
            C = sp.vstack([A_IG, Bp_G, sp.csr_matrix((1, len(self.ig)))]).toarray()
        else:
            # all element pressures stay local: K_II = [[A, Bp^T], [Bp, 0]]
            Kii = sp.bmat([[A_II, Bp_I.T], [Bp_I, None]]).tocsc()
            C = sp.vstack([A_IG, Bp_G]).toarray()
        self.lu = _DenseLU(Kii) if dense else splu(Kii)
        self.nv, self.npr = nv, npr
        self.C = C
        rhs = sd["rhs"]
        self.f_I = rhs[self.iv]
        self.f_G = rhs[self.ig]
        self.h_p = rhs[self.ip]
        if condense:
            X = self.lu.solve(C)
            self.S = self.A_GG - C.T @ X
            xb = self.lu.solve(self._rhs_I())
            self.g = self.f_G - C.T @ xb
        # p0 row: B0_Gamma = sum of the element flux rows on the interface
        self.B0 = np.asarray(Bp_G.sum(axis=0)).ravel()
        self.g0 = float(self.h_p.sum())
        self.vol = float(w.sum())

    def _rhs_I(self):
        tail = [0.0] if self.has_p0 else []
        return np.concatenate([self.f_I, self.h_p, tail])

    def recover(self, uG, p0=0.0):
        """Interior velocity and element pressures from (u_Gamma, p0); p0 is
        ignored for a subdomain that keeps its pressures local."""
        x = self.lu.solve(self._rhs_I() - self.C @ uG)
        uI = x[: self.nv]
        c = x[self.nv: self.nv + self.npr]
        return uI, (c + p0 if self.has_p0 else c)


class OracleBDDC:
    def __init__(self, wl, scaling="deluxe", adaptive_theta=0.0, svd_tol=1e-10,
                 adaptive_edges=False, dense_local=False):
        self.wl = wl
        self.pressure_kernel = bool(wl.get("pressure_kernel", True))
        nsub = len(wl["subs"])
        has_p0 = np.asarray(wl.get("has_p0", np.ones(nsub)), bool)
        if has_p0.shape != (nsub,) or bool(has_p0.all()) != self.pressure_kernel:
            raise ValueError("has_p0 must flag every subdomain, and leave some subdomain "
                             "without p0 exactly when the problem has Neumann sides")
        self.nG = wl["n_iface"]
        self.loc = [LocalSchur(sd, dense=dense_local, has_p0=h) for sd, h in zip(wl["subs"], has_p0)]
        # p0 unknowns: one per subdomain that keeps its constant pressure
        self.p0_sub = np.nonzero(has_p0)[0]
        self.p0_pos = -np.ones(nsub, np.int64)
        self.p0_pos[self.p0_sub] = np.arange(len(self.p0_sub))
        self.N = len(self.p0_sub)
        self.n = self.nG + self.N  # global interface vector: u_Gamma then p0
        self.svd_tol = svd_tol
        self.scaling = scaling
        self.adaptive_theta = adaptive_theta
        # entities
        self.ents = wl["ents"]
        self.ent_of_gid = np.zeros(self.nG, np.int64)
        for e, E in enumerate(self.ents):
            self.ent_of_gid[E["gids"]] = e
        self.ent_subs = [[] for _ in self.ents]
        for i, L in enumerate(self.loc):
            for e in np.unique(self.ent_of_gid[L.gid]):
                self.ent_subs[e].append(i)
        self.extra_rows = [None] * len(self.ents)
        self._setup_basis()
        if adaptive_theta > 0:
            from .adaptive import adaptive_rows
            self.eig_info = adaptive_rows(self, adaptive_theta, edges=adaptive_edges)
            self._setup_basis()
        self._setup_scaling()
        self._setup_coarse()

    # ------------------------------------------------------------------ basis
    def _setup_basis(self):
        """Per entity: orthonormal [Q_Pi | Q_Delta] from the SVD of the
        constraint rows (dependent rows dropped, Sec. 5.1)."""
        self.Q = []
        self.npi = []
        for e, E in enumerate(self.ents):
            C = E["con"]
            if self.extra_rows[e] is not None:
                C = np.vstack([C, self.extra_rows[e]]) if C.size else self.extra_rows[e]
            nE = len(E["gids"])
            if C.shape[0] == 0:
                self.Q.append(np.eye(nE))
                self.npi.append(0)
                continue
            U, s, Vt = np.linalg.svd(C, full_matrices=True)
            r = int(np.sum(s > self.svd_tol * s[0]))
            self.Q.append(Vt.T.copy())  # first r columns span the constraints
            self.npi.append(r)
        # global transformed coordinates: per entity [primal | dual]
        self.T = np.zeros((self.nG, self.nG))
        self.pi_idx, self.de_idx = [], []
        for e, E in enumerate(self.ents):
            g = E["gids"]
            self.T[np.ix_(g, g)] = self.Q[e]
            self.pi_idx.append(g[: self.npi[e]])
            self.de_idx.append(g[self.npi[e]:])
        # (transformed coordinate j of entity e is stored at position gids[j])
        self.is_primal = np.zeros(self.nG, bool)
        for e in range(len(self.ents)):
            self.is_primal[self.pi_idx[e]] = True
        for L in self.loc:
            Tl = self.T[np.ix_(L.gid, L.gid)]
            L.St = Tl.T @ L.S @ Tl
            L.B0t = L.B0 @ Tl
            L.prim = self.is_primal[L.gid]
            L.gt = Tl.T @ L.g

    # ---------------------------------------------------------------- scaling
    def _setup_scaling(self):
        """D_E^(m) per entity and subdomain on the dual coordinates."""
        self.D = {}
        for e, E in enumerate(self.ents):
            dual = self.de_idx[e]
            if len(dual) == 0:
                continue
            subs = self.ent_subs[e]
            blocks = {}
            for i in subs:
                L = self.loc[i]
                pos = np.searchsorted(L.gid, dual) if np.all(np.diff(L.gid) > 0) else \
                    np.array([np.nonzero(L.gid == d)[0][0] for d in dual])
                blocks[i] = (pos, L.St[np.ix_(pos, pos)])
            if self.scaling == "deluxe":
                Ssum = sum(b[1] for b in blocks.values())
                for i in subs:
                    self.D[(e, i)] = (blocks[i][0], np.linalg.solve(Ssum, blocks[i][1]))
            else:
                for i in subs:
                    self.D[(e, i)] = (blocks[i][0], np.eye(len(dual)) / len(subs))

    # ----------------------------------------------------------------- coarse
    def _setup_coarse(self):
        """Local constrained Neumann factors and the bordered coarse matrix."""
        gprim = np.nonzero(self.is_primal)[0]
        self.nc = len(gprim)
        cidx = -np.ones(self.nG, np.int64)
        cidx[gprim] = np.arange(self.nc)
        self.cidx = cidx
        self.ncb = self.nc + self.N + (1 if self.pressure_kernel else 0)
        Kc = np.zeros((self.ncb, self.ncb))
        for i, L in enumerate(self.loc):
            P = np.nonzero(L.prim)[0]
            Dl = np.nonzero(~L.prim)[0]
            L.P, L.Dl = P, Dl
            S_DD = L.St[np.ix_(Dl, Dl)]
            S_DP = L.St[np.ix_(Dl, P)]
            L.cho = sla.cho_factor(S_DD) if len(Dl) else None
            L.Phi = -sla.cho_solve(L.cho, S_DP) if len(Dl) else np.zeros((0, len(P)))
            SPi = L.St[np.ix_(P, P)] + S_DP.T @ L.Phi
            c = cidx[L.gid[P]]
            Kc[np.ix_(c, c)] += SPi
            if not L.has_p0:
                continue
            # B0 in primal coordinates (the dual part vanishes: Assumption 1)
            q = self.nc + self.p0_pos[i]
            Kc[q, c] += L.B0t[P]
            Kc[c, q] += L.B0t[P]
            L.B0_dual_norm = np.abs(L.B0t[Dl]).max() if len(Dl) else 0.0
        if self.pressure_kernel:
            vol = np.array([self.loc[i].vol for i in self.p0_sub])
            Kc[-1, self.nc: self.nc + self.N] = vol
            Kc[self.nc: self.nc + self.N, -1] = vol
        self.Kc = Kc
        self.Kc_lu = sla.lu_factor(Kc)

    # ------------------------------------------------------------- operators
    def rhs(self):
        """g_hat (eq. globInt) in original coordinates."""
        g = np.zeros(self.n)
        for i, L in enumerate(self.loc):
            np.add.at(g, L.gid, L.g)
            if L.has_p0:
                g[self.nG + self.p0_pos[i]] = L.g0
        return g

    def apply_S(self, x):
        """S_hat x in original coordinates."""
        y = np.zeros(self.n)
        for i, L in enumerate(self.loc):
            xl = x[L.gid]
            if not L.has_p0:
                np.add.at(y, L.gid, L.S @ xl)
                continue
            q = self.nG + self.p0_pos[i]
            np.add.at(y, L.gid, L.S @ xl + L.B0 * x[q])
            y[q] = L.B0 @ xl
        return y

    def apply_M(self, r):
        """z = M^-1 r (eq. BDDCprec) in original coordinates."""
        rt = np.concatenate([self.T.T @ r[: self.nG], r[self.nG:]])
        # restriction: primal and p0 pass through, duals scaled
        rc = np.zeros(self.ncb)
        gpr = np.nonzero(self.is_primal)[0]
        rc[self.cidx[gpr]] = rt[gpr]
        rc[self.nc: self.nc + self.N] = rt[self.nG:]
        gD = []
        for i, L in enumerate(self.loc):
            g = np.zeros(len(L.Dl))
            gD.append(g)
        for (e, i), (pos, D) in self.D.items():
            L = self.loc[i]
            dual = self.de_idx[e]
            # local dual position of pos within L.Dl
            loc_in_D = np.searchsorted(L.Dl, pos)
            gD[i][loc_in_D] += D.T @ rt[dual]
        for i, L in enumerate(self.loc):
            if len(L.Dl):
                c = self.cidx[L.gid[L.P]]
                np.add.at(rc, c, L.Phi.T @ gD[i])
        uc = sla.lu_solve(self.Kc_lu, rc)
        zt = np.zeros(self.n)
        zt[gpr] = uc[self.cidx[gpr]]
        zt[self.nG:] = uc[self.nc: self.nc + self.N]
        wD = []
        for i, L in enumerate(self.loc):
            if len(L.Dl):
                c = self.cidx[L.gid[L.P]]
                w = sla.cho_solve(L.cho, gD[i]) + L.Phi @ uc[c]
            else:
                w = np.zeros(0)
            wD.append(w)
        for (e, i), (pos, D) in self.D.items():
            L = self.loc[i]
            dual = self.de_idx[e]
            loc_in_D = np.searchsorted(L.Dl, pos)
            zt[dual] += D @ wD[i][loc_in_D]
        return np.concatenate([self.T @ zt[: self.nG], zt[self.nG:]])

    def recover(self, x):
        """Per-subdomain (u_I, element pressures) from the interface solution."""
        out = []
        for i, L in enumerate(self.loc):
            p0 = x[self.nG + self.p0_pos[i]] if L.has_p0 else 0.0
            out.append(L.recover(x[L.gid], p0))
        return out

    def dense_S(self):
        """Dense S_hat (tiny problems only)."""
        S = np.zeros((self.n, self.n))
        for i, L in enumerate(self.loc):
            g = L.gid
            S[np.ix_(g, g)] += L.S
            if L.has_p0:
                q = self.nG + self.p0_pos[i]
                S[q, g] += L.B0
                S[g, q] += L.B0
        return S
