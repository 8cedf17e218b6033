"""Pins of the CPU oracle (BDDC + PCG, Sec. 4-5) against what the paper and
the mathematics fix: brute-force dense Schur complements and direct solves
on tiny meshes, the kernel of S_hat, Assumption 1, the all-primal special
case, the minimum eigenvalue 1 of Theorem teoEst, symmetry of M^-1 and the
(1 + log(H/h))^2 trend."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from inputs.mesh import CubeMesh
from inputs.assemble import Problem
from inputs.decompose import Decomposition, regular_cuts, random_cuts
from oracle.bddc import OracleBDDC
from oracle.pcg import pcg, lanczos_extremes

MIN = ("vertex", "edge", "flux")
FULL = ("vertex", "edge", "face", "flux")


def _setup(n, parts, cons, jitter=0.0, seed=0, scaling="deluxe", k=2):
    pb = Problem(CubeMesh(n, jitter=jitter, seed=seed), k, 1.0, workers=1)
    dec = Decomposition(pb, regular_cuts(n, parts), cons)
    return pb, dec, OracleBDDC(dec.workload(), scaling=scaling)


@pytest.fixture(scope="module")
def tiny():
    return _setup(4, (2, 2, 2), MIN)


@pytest.fixture(scope="module")
def tiny_jit():
    return _setup(4, (2, 2, 2), FULL, jitter=0.15, seed=7)


def _dense_interface_schur(pb, dec):
    """Brute force: eliminate all interior velocities and the Q_I pressures
    of the assembled global reduced system; the remaining unknowns are
    (u_Gamma, p0).  Q_I basis per subdomain from an explicit null space."""
    K, g, free = pb.reduced_system()
    K = K.toarray()
    Nvr = pb.Nvr
    pos = {r: i for i, r in enumerate(free)}
    n_free = len(free)
    iface = [pos[r] for r in dec.iface_red]
    vel_int = [i for i, r in enumerate(free) if r < Nvr and dec.gid_of_red[r] < 0]
    # pressure change of basis c = sum_i (QI_i q_i + 1 p0_i)
    cols_q, cols_p0 = [], []
    for i, sd in enumerate(dec.subs):
        el = sd.elems
        w = pb.mesh.elem_vol[el]
        QI = sla.null_space(w[None, :])
        for j in range(QI.shape[1]):
            v = np.zeros(n_free)
            v[[pos[Nvr + e] for e in el]] = QI[:, j]
            cols_q.append(v)
        v = np.zeros(n_free)
        v[[pos[Nvr + e] for e in el]] = 1.0
        cols_p0.append(v)
    E = np.zeros((n_free, 0))
    basis = []
    for i in vel_int:
        v = np.zeros(n_free)
        v[i] = 1.0
        basis.append(v)
    nI = len(basis) + len(cols_q)
    basis += cols_q
    for i in iface:
        v = np.zeros(n_free)
        v[i] = 1.0
        basis.append(v)
    basis += cols_p0
    T = np.array(basis).T
    Kt = T.T @ K @ T
    gt = T.T @ g
    A, B, C, D = Kt[:nI, :nI], Kt[:nI, nI:], Kt[nI:, :nI], Kt[nI:, nI:]
    S = D - C @ np.linalg.solve(A, B)
    gs = gt[nI:] - C @ np.linalg.solve(A, gt[:nI])
    return S, gs


def test_schur_and_rhs_match_brute_force(tiny_jit):
    pb, dec, o = tiny_jit
    S, gs = _dense_interface_schur(pb, dec)
    Sd = o.dense_S()
    assert np.abs(Sd - S).max() < 1e-11 * np.abs(S).max()
    assert np.abs(o.rhs() - gs).max() < 1e-11 * np.abs(gs).max()


def test_kernel_of_S_hat_is_constant_p0(tiny):
    pb, dec, o = tiny
    S = o.dense_S()
    ev, V = np.linalg.eigh(S)
    small = np.abs(ev) < 1e-10 * np.abs(ev).max()
    assert small.sum() == 1
    v = V[:, np.argmin(np.abs(ev))]
    assert np.abs(v[: o.nG]).max() < 1e-8
    assert np.allclose(np.abs(v[o.nG:]), np.abs(v[o.nG:]).mean(), rtol=1e-8)


def test_floating_subdomain_schur_has_rigid_kernel():
    pb, dec, o = _setup(6, (3, 3, 3), MIN)
    mid = 13  # the subdomain not touching the boundary
    S = o.loc[mid].S
    assert np.abs(S - S.T).max() < 1e-12 * np.abs(S).max()
    ev = np.linalg.eigvalsh(S)
    assert np.all(np.abs(ev[:6]) < 1e-10 * ev[-1]) and ev[6] > 1e-6 * ev[-1]
    ev0 = np.linalg.eigvalsh(o.loc[0].S)  # touches the Dirichlet boundary: SPD
    assert ev0[0] > 1e-8 * ev0[-1]


def test_assumption1_flux_vanishes_on_dual(tiny_jit):
    pb, dec, o = tiny_jit
    for L in o.loc:
        assert L.B0_dual_norm < 1e-13 * np.abs(L.B0).max()


def test_deluxe_partition_of_unity(tiny_jit):
    pb, dec, o = tiny_jit
    for e in range(len(o.ents)):
        mats = [D for (ee, i), (pos, D) in o.D.items() if ee == e]
        if mats:
            assert np.abs(sum(mats) - np.eye(mats[0].shape[0])).max() < 1e-12


def _deluxe_energy_checks(o, rng):
    """For every entity shared by several subdomains: w_q random local values
    on its dual coordinates, v = sum_q D_q w_q (the extension), and
    E(x) = sum_q (w_q - x)^T Sbar_q (w_q - x).  Returns the largest
    |E(v+d) - E(v-d)| / (E(v+d) + E(v-d)) and whether E(v +- d) > E(v)
    held for every trial."""
    worst, above = 0.0, True
    for e in range(len(o.ents)):
        items = [(i, pos, D) for (ee, i), (pos, D) in o.D.items() if ee == e]
        if len(items) < 2:
            continue
        Sb = [o.loc[i].St[np.ix_(pos, pos)] for i, pos, _ in items]
        w = [rng.standard_normal(D.shape[0]) for _, _, D in items]
        v = sum(D @ wq for (_, _, D), wq in zip(items, w))

        def E(x):
            return sum((wq - x) @ S @ (wq - x) for wq, S in zip(w, Sb))

        for _ in range(3):
            d = rng.standard_normal(len(v)) * np.linalg.norm(v) / np.sqrt(len(v))
            ep, em, e0 = E(v + d), E(v - d), E(v)
            worst = max(worst, abs(ep - em) / (ep + em))
            above = above and ep > e0 and em > e0
    return worst, above


def test_deluxe_average_minimises_the_weighted_energy(tiny_jit):
    """Deluxe averaging (Sec. 6): the extension sum_q D_q w_q of local values
    on an entity's dual coordinates minimises sum_q ||w_q - v||^2 in the
    Sbar_q norms (Sbar_q: subdomain q's block of the transformed S_Gamma on
    those coordinates).  A quadratic takes equal values at v* + d and v* - d
    exactly at its minimiser, so the test perturbs symmetrically.  Unlike
    sum_q D_q = I, this fails for transposed blocks D_q^T or a product taken
    in the wrong order."""
    pb, dec, o = tiny_jit
    worst, above = _deluxe_energy_checks(o, np.random.default_rng(3))
    assert worst < 1e-10 and above


def test_preconditioner_symmetric(tiny_jit):
    pb, dec, o = tiny_jit
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(o.n), rng.standard_normal(o.n)
    a[o.nG:] -= a[o.nG:].mean()
    b[o.nG:] -= b[o.nG:].mean()
    lhs, rhs = a @ o.apply_M(b), b @ o.apply_M(a)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + abs(rhs))


def test_pcg_matches_direct_solve(tiny_jit):
    pb, dec, o = tiny_jit
    g = o.rhs()
    x, info = pcg(o.apply_S, o.apply_M, g, tol=1e-12)
    uG, p0 = dec.interface_solution(pb.solve_reduced_direct())
    ref = np.concatenate([uG, p0])
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)


def test_pcg_matches_direct_solve_degree_4():
    """The whole oracle pipeline at k = 4 (decomposition, condensation,
    BDDC, PCG) against the direct solve of the assembled global system."""
    pb, dec, o = _setup(4, (2, 2, 2), FULL, jitter=0.15, seed=4, k=4)
    x, info = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-12)
    u = pb.solve_reduced_direct()
    uG, p0 = dec.interface_solution(u)
    ref = np.concatenate([uG, p0])
    assert np.linalg.norm(x - ref) < 1e-9 * np.linalg.norm(ref)


def test_all_primal_converges_in_one_iteration():
    pb = Problem(CubeMesh(4), 2, 1.0, workers=1)
    dec = Decomposition(pb, regular_cuts(4, (2, 2, 2)), MIN)
    wl = dec.workload()
    for E in wl["ents"]:
        E["con"] = np.eye(len(E["gids"]))
    o = OracleBDDC(wl)
    x, info = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-10)
    assert info["iters"] == 1


def _benign_spectrum(o):
    """Nonzero eigenvalues of M^-1 S_hat on the benign space (dense, tiny
    problems).  With r's p0 part zero, M^-1 r has zero net flux out of every
    subdomain (the coarse problem imposes it), so CG stays in
    V_B = {(u, p0): B0^(i) u = 0 for all i}; M^-1 S_hat maps V_B into itself
    and is self-adjoint in the S_hat form there.  The eigenvalues come from
    the restriction V^T M^-1 S_hat V, V an orthonormal basis of V_B, with the
    constant-p0 kernel (eigenvalue 0) dropped."""
    n = o.n
    M = np.array([o.apply_M(e) for e in np.eye(n)]).T
    S = o.dense_S()
    V = sla.null_space(S[o.nG:, :])
    ev = sla.eigvals(V.T @ M @ S @ V)
    assert np.abs(ev.imag).max() < 1e-9 * np.abs(ev).max()
    ev = np.sort(ev.real)
    return ev[np.abs(ev) > 1e-8]


def test_min_eigenvalue_is_one_dense(tiny):
    """Theorem teoEst: on the benign space lambda_min(M^-1 S_hat) = 1."""
    o = tiny[2]
    nz = _benign_spectrum(o)
    assert nz.min() > 1 - 1e-10
    assert np.sum(np.abs(nz - 1) < 1e-8) >= o.nc  # eigenvalue-1 cluster of at least the coarse size


def test_min_eigenvalue_bound_degree_4():
    """Theorem teoEst at VEM degree 4 (jittered mesh, 2^3 elements per
    subdomain, vertex + edge + face constraints): every nonzero eigenvalue
    of M^-1 S_hat on the benign space is >= 1, and the smallest is 1 (the
    rounding of the dense restriction is about 1e-13)."""
    nz = _benign_spectrum(_setup(4, (2, 2, 2), FULL, jitter=0.15, seed=4, k=4)[2])
    assert 1 - 1e-10 < nz.min() < 1 + 1e-6


def test_ritz_lambda_min_and_log_trend():
    """Ritz values of the CG-Lanczos matrix stay >= 1 and, for the minimal
    coarse space, k_2 / (1 + log(H/h))^2 does not grow along H/h = 2, 4, 5
    (k_2 itself grows from 2.3 to 9.1)."""
    ratios = []
    for n in (4, 8, 10):
        pb, dec, o = _setup(n, (2, 2, 2), MIN)
        x, info = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-10)
        lmin, lmax = lanczos_extremes(info["alphas"], info["betas"])
        assert lmin > 1 - 1e-8
        ratios.append((lmax / lmin) / (1 + np.log(n / 2)) ** 2)
    assert ratios[-1] < 1.5 * max(ratios[:-1])


def test_counting_scaling_converges_to_same_solution():
    pb, dec, od = _setup(8, (2, 2, 2), FULL, jitter=0.15, seed=1)
    oc = OracleBDDC(dec.workload(), scaling="counting")
    g = od.rhs()
    xd, idl = pcg(od.apply_S, od.apply_M, g, tol=1e-8)
    xc, ic = pcg(oc.apply_S, oc.apply_M, g, tol=1e-8)
    assert ic["iters"] < 200
    assert np.linalg.norm(xd - xc) < 1e-6 * np.linalg.norm(xd)


@pytest.mark.parametrize("k", [2, 4])
def test_recover_matches_direct_solve(k):
    """Interior recovery (eq. uipi, Sec. 4.2): given the interface velocity
    and p0 of the direct solve of the assembled reduced system, every
    subdomain's recovered interior velocity and element pressures equal the
    direct solve's.  A wrong sign on the C u_Gamma term or a dropped p0
    fails it."""
    pb, dec, o = _setup(4, (2, 2, 2), FULL, jitter=0.15, seed=5, k=k)
    u = pb.solve_reduced_direct()
    uG, p0 = dec.interface_solution(u)
    rec = o.recover(np.concatenate([uG, p0]))
    for sd, (uI, c) in zip(dec.subs, rec):
        ref_u = u[sd.dofs[sd.kind == 0]]
        ref_p = u[sd.dofs[sd.kind == 2]]
        assert np.linalg.norm(uI - ref_u) <= 1e-10 * np.linalg.norm(ref_u)
        # the pressures are O(h^k) here (the manufactured p is 0), so they are
        # compared on the scale of the local solution
        assert np.linalg.norm(c - ref_p) <= 1e-9 * np.linalg.norm(ref_u)


def test_lanczos_extremes_closed_form():
    """Lanczos from the CG coefficients (Sec. 5, the estimate behind Theorem
    teoEst's condition numbers): for A = diag(d) and M^-1 = diag(m) with
    distinct products d*m and a right-hand side that excites every
    eigenvector, CG terminates after n steps and the tridiagonal matrix
    built from its alphas and betas is similar to M^-1 A, so its extreme
    eigenvalues are min(d*m) and max(d*m).  A wrong diagonal or off-diagonal
    entry of T moves them."""
    rng = np.random.default_rng(2)
    for n in (2, 3, 6, 9):
        d = rng.uniform(0.5, 20.0, n)
        m = rng.uniform(0.2, 3.0, n)
        b = rng.uniform(0.5, 1.5, n)
        x, info = pcg(lambda v: d * v, lambda v: m * v, b, fixed_iters=n)
        lmin, lmax = lanczos_extremes(info["alphas"], info["betas"])
        dm = d * m
        assert abs(lmin - dm.min()) < 1e-10 * dm.max()
        assert abs(lmax - dm.max()) < 1e-10 * dm.max()


def test_lanczos_extremes_match_dense_spectrum(tiny_jit):
    """On the BDDC-preconditioned interface operator: CG from a random
    right-hand side with zero p0 part (so it stays in the benign space) to a
    1e-12 residual.  The largest eigenvalue of its Lanczos matrix equals the
    largest of the dense benign spectrum to 1e-8 (an isolated extreme
    eigenvalue converges first), and the smallest lies in that spectrum's
    range: above lambda_min = 1 (Theorem teoEst) and within 1% of it (the
    eigenvalue-1 cluster of the coarse space is not resolved one by one
    before the residual converges)."""
    o = tiny_jit[2]
    nz = _benign_spectrum(o)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(o.n)
    b[o.nG:] = 0.0
    x, info = pcg(o.apply_S, o.apply_M, b, tol=1e-12, maxit=400)
    lmin, lmax = lanczos_extremes(info["alphas"], info["betas"])
    assert abs(lmax - nz.max()) < 1e-8 * nz.max()
    assert nz.min() - 1e-10 <= lmin <= 1.01 * nz.min()
    assert abs(nz.min() - 1.0) < 1e-10


def test_dense_local_factors_agree_with_sparse(tiny_jit):
    """The oracle's second evaluation (dense LU of the local Dirichlet
    matrices instead of sparse LU) computes the same S_Gamma, g and M^-1 on
    a well-conditioned problem: agreement to rounding."""
    pb, dec, o = tiny_jit
    od = OracleBDDC(dec.workload(), dense_local=True)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(o.n)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(od.rhs(), o.rhs()) < 1e-12
    assert rel(od.apply_S(x), o.apply_S(x)) < 1e-12
    r = o.apply_S(x)
    assert rel(od.apply_M(r)[: o.nG], o.apply_M(r)[: o.nG]) < 1e-11


NEUMANN_CASES = [  # (mesh size, Neumann sides, cuts)
    (4, (0, 1), lambda: regular_cuts(4, (3, 2, 2))),  # 4 of 12 subdomains keep p0
    (4, (0, 1), lambda: regular_cuts(4, (2, 2, 1))),  # none does
    (4, (2, 5), lambda: regular_cuts(4, (2, 3, 2))),
    (5, (4,), lambda: random_cuts(5, 1, 3, 2, 1)),    # uneven cuts
]


@pytest.mark.parametrize("case", range(len(NEUMANN_CASES)))
def test_neumann_sides_match_direct_solve(case):
    """Neumann sides (Sec. 7): subdomains with a side on them eliminate all
    their element pressures locally and keep no p0, the others keep theirs,
    and the coarse problem has no border.  The flag agrees with the box
    position and with the flux structure it stands for (the summed pressure
    rows of a subdomain vanish on its interior velocities exactly when it
    keeps p0); PCG on the interface problem reaches the direct solve of the
    assembled system, and recovery gives every subdomain's interior
    velocity and pressures."""
    n, sides, make_cuts = NEUMANN_CASES[case]
    cuts = make_cuts()
    pb = Problem(CubeMesh(n, jitter=0.15, seed=3), 2, 1.0, workers=1, neumann_sides=sides)
    dec = Decomposition(pb, cuts, FULL)
    wl = dec.workload()
    parts = [len(c) - 1 for c in cuts]
    for s, h in enumerate(wl["has_p0"]):
        seg = (s % parts[0], (s // parts[0]) % parts[1], s // (parts[0] * parts[1]))
        touched = {2 * a for a in range(3) if seg[a] == 0} | \
                  {2 * a + 1 for a in range(3) if seg[a] == parts[a] - 1}
        assert bool(h) == (not touched & set(sides))
    for sd, h in zip(wl["subs"], wl["has_p0"]):
        m = len(sd["kind"])
        K = sp.csr_matrix((sd["data"], sd["indices"], sd["indptr"]), shape=(m, m))
        flux = np.asarray(K[sd["kind"] == 2].sum(axis=0)).ravel()
        inner = np.abs(flux[sd["kind"] == 0]).max()
        assert (inner < 1e-12 * np.abs(flux).max()) == bool(h)
    o = OracleBDDC(wl)
    assert o.N == int(wl["has_p0"].sum()) and o.Kc.shape[0] == o.nc + o.N
    x, info = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-12)
    u = pb.solve_reduced_direct()
    uG, p0 = dec.interface_solution(u)
    ref = np.concatenate([uG, p0])
    assert np.linalg.norm(x - ref) < 1e-9 * np.linalg.norm(ref)
    for sd, (uI, c) in zip(dec.subs, o.recover(x)):
        ref_u = u[sd.dofs[sd.kind == 0]]
        ref_p = u[sd.dofs[sd.kind == 2]]
        assert np.linalg.norm(uI - ref_u) <= 1e-9 * np.linalg.norm(ref_u)
        assert np.linalg.norm(c - ref_p) <= 1e-8 * max(np.linalg.norm(ref_u), np.linalg.norm(ref_p))
    with pytest.raises(ValueError):
        OracleBDDC(dict(wl, has_p0=np.ones(len(wl["subs"]), np.int32)))


@pytest.mark.parametrize("parts", [(3, 2, 2), (2, 2, 1)])
def test_neumann_sides_spectrum(parts):
    """With Neumann sides the interface problem loses the constant-p0
    kernel: on the benign space (zero net flux out of every subdomain that
    keeps p0; the whole space when none does, where S_hat is SPD) M^-1 S_hat
    has no zero eigenvalue, and Theorem teoEst's bound lambda_min = 1 holds
    as in the no-slip case.  The preconditioner stays symmetric."""
    n = 4
    pb = Problem(CubeMesh(n, jitter=0.15, seed=3), 2, 1.0, workers=1, neumann_sides=(0, 1))
    o = OracleBDDC(Decomposition(pb, regular_cuts(n, parts), FULL).workload())
    M = np.array([o.apply_M(e) for e in np.eye(o.n)]).T
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    S = o.dense_S()
    if o.N == 0:
        assert np.linalg.eigvalsh(S).min() > 0
        V = np.eye(o.n)
    else:
        V = sla.null_space(S[o.nG:, :])
    ev = sla.eigvals(V.T @ M @ S @ V)
    assert np.abs(ev.imag).max() < 1e-9 * np.abs(ev).max()
    assert ev.real.min() > 1 - 1e-10


def _preconditioner_by_definition(o, r):
    """M^-1 r of eq. BDDCprec written out densely: R~_D^T S~^-1 R~_D, with S~
    the partially assembled bordered operator on (global primal coordinates,
    each subdomain's own dual coordinates, each subdomain's p0), the
    constant-p0 kernel fixed by the volume border (no-slip boundaries; with
    Neumann sides only the subdomains away from them have p0 and there is
    no border), and R~_D passing primal
    and p0 entries through and scaling the duals by D^T (all in the
    transformed coordinates)."""
    off, pos_of = [], []
    m = o.nc
    for L in o.loc:
        off.append(m)
        m += len(L.Dl)
    q0 = m
    m += o.N
    idx = []
    for i, L in enumerate(o.loc):
        ix = np.empty(len(L.gid), np.int64)
        ix[L.prim] = o.cidx[L.gid[L.prim]]
        ix[~L.prim] = off[i] + np.arange(len(L.Dl))
        idx.append(ix)
    nb = m + (1 if o.pressure_kernel else 0)
    St = np.zeros((nb, nb))
    for i, L in enumerate(o.loc):
        St[np.ix_(idx[i], idx[i])] += L.St
        if L.has_p0:
            St[q0 + o.p0_pos[i], idx[i]] += L.B0t
            St[idx[i], q0 + o.p0_pos[i]] += L.B0t
    if o.pressure_kernel:
        vol = np.array([o.loc[i].vol for i in o.p0_sub])
        St[m, q0:m] = vol
        St[q0:m, m] = vol
    rt = np.concatenate([o.T.T @ r[:o.nG], r[o.nG:]])
    Rd = np.zeros((nb, o.n))  # R~_D in the transformed coordinates
    gpr = np.nonzero(o.is_primal)[0]
    Rd[o.cidx[gpr], gpr] = 1.0
    Rd[q0 + np.arange(o.N), o.nG + np.arange(o.N)] = 1.0
    for (e, i), (pos, D) in o.D.items():
        L = o.loc[i]
        rows = off[i] + np.searchsorted(L.Dl, pos)
        Rd[np.ix_(rows, o.de_idx[e])] += D.T
    zt = Rd.T @ np.linalg.solve(St, Rd @ rt)
    return np.concatenate([o.T @ zt[:o.nG], zt[o.nG:]])


@pytest.mark.parametrize("scaling,sides", [("deluxe", ()), ("counting", ()), ("deluxe", (0, 1))])
def test_preconditioner_equals_its_definition(scaling, sides):
    """The oracle applies M^-1 as local constrained Neumann solves plus the
    coarse problem in the primal variables and p0; that split must equal
    eq. BDDCprec with S~^-1 taken whole (a dense solve of the partially
    assembled operator).  A dropped Phi term, a coarse matrix without the
    Schur complement part, or a wrong scaling side fails it."""
    if sides:
        pb = Problem(CubeMesh(4, jitter=0.15, seed=3), 2, 1.0, workers=1, neumann_sides=sides)
        o = OracleBDDC(Decomposition(pb, regular_cuts(4, (3, 2, 2)), FULL).workload(),
                       scaling=scaling)
        assert 0 < o.N < len(o.loc)
    else:
        pb, dec, o = _setup(4, (2, 2, 2), FULL, jitter=0.15, seed=7, scaling=scaling)
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.standard_normal(o.n)
        got = o.apply_M(r)
        ref = _preconditioner_by_definition(o, r)
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_change_of_basis_makes_constraints_explicit(tiny_jit):
    """Sec. 4.3 and 5.1: per entity the basis [Q_Pi | Q_Delta] is orthogonal,
    has as many primal columns as the constraint rows have rank (dependent
    rows dropped; the rank counted here by Gram-Schmidt), every constraint
    vanishes on the dual columns, and the constraint values of any vector
    depend only on its primal coordinates.  The global T is orthogonal and
    maps each entity's DoFs to themselves."""
    pb, dec, o = tiny_jit
    rng = np.random.default_rng(11)
    for e, E in enumerate(o.ents):
        C = np.asarray(E["con"])
        Q = o.Q[e]
        nE = len(E["gids"])
        assert np.abs(Q.T @ Q - np.eye(nE)).max() < 1e-13
        basis = []
        for row in C:
            v = row.copy()
            for b in basis:
                v -= (b @ v) * b
            if np.linalg.norm(v) > 1e-9 * np.linalg.norm(row):
                basis.append(v / np.linalg.norm(v))
        assert o.npi[e] == len(basis)
        if len(C):
            scale = np.abs(C).max()
            if o.npi[e] < nE:
                assert np.abs(C @ Q[:, o.npi[e]:]).max() < 1e-12 * scale
            u = rng.standard_normal(nE)
            up = Q[:, :o.npi[e]] @ (Q[:, :o.npi[e]].T @ u)
            assert np.abs(C @ u - C @ up).max() < 1e-12 * scale * np.abs(u).sum()
    assert np.abs(o.T.T @ o.T - np.eye(o.nG)).max() < 1e-13
    for e, E in enumerate(o.ents):
        others = np.setdiff1d(np.arange(o.nG), E["gids"])
        assert not np.any(o.T[np.ix_(others, E["gids"])])


def test_pcg_iterates_minimise_energy_over_krylov_space():
    """What defines the k-th PCG iterate (the GPU parity tests compare
    against it): from x0 = 0 it minimises the A-norm of the error over the
    Krylov space K_k(M^-1 A, M^-1 b).  Here it is computed independently by
    a Galerkin solve on an orthonormal basis of that space, for a random SPD
    A and SPD M^-1; the recorded residual is the true one.  A wrong alpha or
    beta, or a preconditioner applied on the wrong side, fails it."""
    rng = np.random.default_rng(8)
    n = 40
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    H = rng.standard_normal((n, n))
    Minv = H @ H.T + 0.5 * n * np.eye(n)
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    for k in range(1, 8):
        x, info = pcg(lambda v: A @ v, lambda v: Minv @ v, b, fixed_iters=k)
        K = [Minv @ b]
        for _ in range(k - 1):
            K.append(Minv @ (A @ K[-1]))
        V, _ = np.linalg.qr(np.array(K).T)
        ref = V @ np.linalg.solve(V.T @ A @ V, V.T @ b)
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(xs)
        assert info["iters"] == k
        assert abs(info["resid"][-1] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) <= 1e-10
