"""Pins of the workload generator (virtual element discretisation, Sec. 3)
against what the paper and the mathematics fix."""
import os
from math import factorial

import numpy as np
import pytest

from inputs.mesh import CubeMesh
from inputs.quadrature import tet_rule, triangle_rule
from inputs.vem import element_matrices, interpolate, element_quadrature
from inputs.poly import mono3, eval3, dim3
from inputs.assemble import Problem, u_curl, grad_u_curl
from inputs.decompose import Decomposition, regular_cuts, random_cuts

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def closed_form_dofs(n, k):
    """3(N_V + (k-1)N_E + dim P_{k-2}(f) N_F) + (D4 + D5 + dim P_{k-1}) N_K."""
    d3 = lambda m: 0 if m < 0 else (m + 1) * (m + 2) * (m + 3) // 6
    nV, nE, nF, nK = (n + 1) ** 3, 3 * n * (n + 1) ** 2, 3 * n * n * (n + 1), n ** 3
    d4 = 3 * d3(k - 3) - d3(k - 4)
    d5 = d3(k - 1) - 1
    return 3 * (nV + (k - 1) * nE + (k * (k - 1) // 2) * nF) + (d4 + d5 + d3(k - 1)) * nK


def _rows():
    out = []
    for line in open(os.path.join(GOLDEN, "paper_cube_dofs.txt")):
        if line.startswith("#") or not line.strip():
            continue
        p = line.split()
        out.append((int(p[0]), int(p[1]), int(p[2])))
    return out


def test_quadrature_exact_on_monomials():
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    lam, w = tet_rule(7)
    X = lam @ P
    for a, b, c in [(3, 2, 2), (0, 0, 7), (1, 4, 2)]:
        ex = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        assert abs((w / 6 * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c).sum() - ex) < 1e-15
    lam, w = triangle_rule(6)
    X = lam @ P[:3, :2]
    for a, b in [(3, 3), (6, 0)]:
        ex = factorial(a) * factorial(b) / factorial(a + b + 2)
        assert abs((w / 2 * X[:, 0] ** a * X[:, 1] ** b).sum() - ex) < 1e-15


def test_dof_counts_match_paper_tables():
    for n, k, printed in _rows():
        cf = closed_form_dofs(n, k)
        if (n, k) == (20, 2):
            assert printed - cf == 1000  # the one row read as a typo
        else:
            assert cf == printed, (n, k)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_generator_counts_equal_closed_form(k):
    pb = Problem(CubeMesh(8), k)
    assert pb.Nv + pb.Np == closed_form_dofs(8, k)


def test_jittered_mesh_planar_faces_and_bound():
    m = CubeMesh(6, jitter=0.15, seed=4)
    X = m.verts[m.face_verts]
    plan = np.abs(np.einsum("fqi,fi->fq", X - X[:, :1], m.face_normal)).max()
    assert plan < 1e-14
    assert np.abs(m.verts - m.vidx * m.h).max() <= 0.15 * m.h + 1e-15
    assert abs(m.elem_vol.sum() - 1.0) < 1e-13


def _poly_field(k, seed):
    rng = np.random.default_rng(seed)
    ex = np.array(mono3(k))
    C = rng.standard_normal((3, len(ex)))

    def u(X):
        return np.stack([X[..., 0] ** a * X[..., 1] ** b * X[..., 2] ** c for a, b, c in ex], -1) @ C.T

    def grad(X):
        G = np.zeros(X.shape[:-1] + (3, 3))
        for d in range(3):
            e = ex.copy()
            f = e[:, d].copy()
            e[:, d] = np.maximum(e[:, d] - 1, 0)
            P = np.stack([X[..., 0] ** a * X[..., 1] ** b * X[..., 2] ** c for a, b, c in e], -1) * f
            G[..., :, d] = P @ C.T
        return G

    def div(X):
        return np.einsum("...cc->...", grad(X))

    return u, grad, div


@pytest.mark.parametrize("k", [2, 3, 4])
def test_projections_reproduce_polynomials(k):
    m = CubeMesh(3, jitter=0.15, seed=1)
    el = np.arange(m.nK)
    out = element_matrices(m, k, el, 1.0, keep=True)
    u, grad, div = _poly_field(k, 0)
    d = interpolate(m, k, el, u, div)
    rng = np.random.default_rng(5)
    X = m.elem_xbar[:, None, :] + 0.02 * rng.standard_normal((m.nK, 4, 3))
    Mx = eval3((X - m.elem_centroid[:, None]) / m.elem_diam[:, None, None], k)
    for key in ("PiN", "P0"):
        c = np.einsum("ecbn,en->ecb", out[key], d)
        assert np.abs(np.einsum("eqb,ecb->eqc", Mx, c) - u(X)).max() < 1e-12
    # Pi^0_{k-1} grad v = grad v
    Mg = eval3((X - m.elem_centroid[:, None]) / m.elem_diam[:, None, None], k - 1)
    G = np.einsum("ecdan,en->ecda", out["Gc"], d)
    assert np.abs(np.einsum("eqa,ecda->eqcd", Mg, G) - grad(X)).max() < 1e-11
    # divergence reconstruction
    dv = np.einsum("ean,en->ea", out["div"], d)
    assert np.abs(np.einsum("eqa,ea->eq", Mg, dv) - div(X)).max() < 1e-11


@pytest.mark.parametrize("k", [2, 3, 4])
def test_element_stiffness_rigid_kernel_and_consistency(k):
    m = CubeMesh(3, jitter=0.15, seed=2)
    el = np.arange(m.nK)
    out = element_matrices(m, k, el, 1.0, keep=True)
    A = out["A"]
    assert np.abs(A - A.transpose(0, 2, 1)).max() < 1e-12 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    scale = ev[:, -1:]
    assert np.all(np.abs(ev[:, :6]) < 1e-12 * scale)  # exactly the 6 rigid modes
    assert np.all(ev[:, 6] > 1e-8 * scale[:, 0])
    u1, g1, d1 = _poly_field(k, 1)
    u2, g2, d2 = _poly_field(k, 2)
    a1 = interpolate(m, k, el, u1, d1)
    a2 = interpolate(m, k, el, u2, d2)
    P, W = element_quadrature(m, el, 2 * k + 2)
    e1 = g1(P)
    e2 = g2(P)
    e1 = 0.5 * (e1 + np.swapaxes(e1, -1, -2))
    e2 = 0.5 * (e2 + np.swapaxes(e2, -1, -2))
    exact = np.einsum("eq,eqcd,eqcd->e", W, e1, e2)
    ah = np.einsum("en,enm,em->e", a1, A, a2)
    assert np.abs(ah - exact).max() < 1e-11
    # divergence rows are exact: b(v, m_a) = int div v m_a
    Mq = eval3((P - m.elem_centroid[:, None]) / m.elem_diam[:, None, None], k - 1)
    exB = np.einsum("eq,eq,eqa->ea", W, d1(P), Mq)
    assert np.abs(np.einsum("ean,en->ea", out["B"], a1) - exB).max() < 1e-13


@pytest.mark.parametrize("k", [2, 3, 4])
def test_patch_test_reduced_and_full(k):
    """u=(y^2,z^2,x^2), p=x+y+z-3/2 (div u = 0) solve -div(nu eps(u)) - grad p = f
    with f = -(nu+1)(1,1,1); the discrete solution is the interpolant."""
    m = CubeMesh(3, jitter=0.15, seed=3)
    u = lambda X: np.stack([X[..., 1] ** 2, X[..., 2] ** 2, X[..., 0] ** 2], -1)
    zero = lambda X: 0 * X[..., 0]
    f = lambda P, el: -2.0 * np.ones(P.shape)
    pb = Problem(m, k, 1.0, force=f, uD=u, divD=zero, keep_full=True, workers=1)
    x = pb.solve_reduced_direct()
    el = np.arange(m.nK)
    d = interpolate(m, k, el, u, zero)
    ui = np.zeros(pb.Nv)
    ui[pb.gmap.ravel()] = d.ravel()
    assert np.abs(x[: pb.Nvr] - ui[pb.full_of_red]).max() < 1e-10
    assert np.abs(x[pb.Nvr:] - (m.elem_centroid.sum(1) - 1.5)).max() < 1e-9
    uf, pf = pb.full_system_direct()
    assert np.abs(uf[pb.full_of_red] - x[: pb.Nvr]).max() < 1e-10


def test_discrete_velocity_divergence_free():
    """div V_h in Q_h: D5(u_h) = 0 and every element flux vanishes."""
    m = CubeMesh(4, jitter=0.15, seed=0)
    pb = Problem(m, 2, 1.0, keep_full=True, workers=1)
    uf, pf = pb.full_system_direct()
    scale = np.abs(uf).max()
    isD5 = np.ones(pb.Nv, bool)
    isD5[pb.full_of_red] = False
    assert np.abs(uf[isD5]).max() < 1e-10 * scale  # round-off of the direct solve
    fl = np.einsum("en,en->e", pb.full["B"][:, 0, :], uf[pb.gmap])
    assert np.abs(fl).max() < 1e-10 * scale


def test_h_convergence_rate():
    """eq. teoConv: |u - Pi u_h|_{1,h} and ||p - p_h||_0 decay like h^k (k=2)."""
    from oracle.postprocess import errors
    eu, ep = [], []
    for n in (2, 4, 8):
        pb = Problem(CubeMesh(n), 2, 1.0, keep_full=True, workers=1)
        uf, pf = pb.full_system_direct()
        a, b = errors(pb, uf, pf, grad_u_curl, lambda X: 0 * X[..., 0])
        eu.append(a)
        ep.append(b)
    ru = np.log2(eu[1] / eu[2])
    rp = np.log2(ep[1] / ep[2])
    assert 1.8 < ru < 2.6, eu
    assert rp > 1.7, ep


def test_h_convergence_rate_degree_4():
    """eq. teoConv at k = 4 (the degree that uses the reduced D4 set): both
    errors decay like h^4 from n = 2 to n = 4 (measured 4.2 and 4.0)."""
    from oracle.postprocess import errors
    eu, ep = [], []
    for n in (2, 4):
        pb = Problem(CubeMesh(n), 4, 1.0, keep_full=True, workers=1)
        uf, pf = pb.full_system_direct()
        a, b = errors(pb, uf, pf, grad_u_curl, lambda X: 0 * X[..., 0])
        eu.append(a)
        ep.append(b)
    assert np.log2(eu[0] / eu[1]) > 3.6, eu
    assert np.log2(ep[0] / ep[1]) > 3.6, ep


def test_decomposition_sizes_c1():
    pb = Problem(CubeMesh(8), 2)
    dec = Decomposition(pb, regular_cuts(8, (2, 2, 2)), ("vertex", "edge", "flux"))
    assert dec.n_iface == 1893
    kinds = np.array(dec.ent_kind)
    assert (kinds == 0).sum() == 1 and (kinds == 1).sum() == 6 and (kinds == 2).sum() == 12
    for sd in dec.subs:
        assert ((sd.kind == 0).sum(), (sd.kind == 1).sum(), (sd.kind == 2).sum()) == (837, 507, 64)


def test_random_cuts_seed0():
    c = random_cuts(48, 4, 12, 6, 0)
    assert [list(x) for x in c] == [[0, 7, 15, 24, 31, 36, 48], [0, 10, 21, 25, 34, 42, 48],
                                    [0, 10, 18, 24, 28, 36, 48]]


def test_family_member_equals_direct_generation():
    """A problem of a viscosity family (unit element matrices scaled per
    element) equals the problem generated directly with that viscosity."""
    from inputs.workloads import make_family, make_workload
    wl, _ = make_workload("c5", seed=1, workers=1, n=4, k=2)
    fam = make_family("c5s", [1], workers=1, mesh_seed=1, n=4, k=2)[0]
    assert len(wl["subs"]) == len(fam["subs"]) and wl["n_iface"] == fam["n_iface"]
    for a, b in zip(wl["subs"], fam["subs"]):
        assert np.array_equal(a["indices"], b["indices"])
        assert np.abs(a["data"] - b["data"]).max() <= 1e-13 * np.abs(a["data"]).max()
        assert np.abs(a["rhs"] - b["rhs"]).max() <= 1e-12 * max(np.abs(a["rhs"]).max(), 1e-300)


def test_paper_table_recipes():
    """The deg* and mesh* recipes are the paper's optimality-test rows (the
    (n, k) of each appears in the printed tables) with 32 subdomains."""
    from inputs.workloads import RECIPES, make_workload
    printed = {(n, k) for n, k, _ in _rows()}
    names = ["deg2", "deg3", "deg4"] + ["mesh%d" % n for n in (16, 20, 24, 28, 32)]
    for name in names:
        r = RECIPES[name]
        assert (r["n"], r["k"]) in printed, name
        assert np.prod(r["parts"]) == 32
    wl, meta = make_workload("deg2", workers=1)
    assert len(wl["subs"]) == 32
    assert meta["problem"].Nv + meta["problem"].Np == 16787


@pytest.mark.parametrize("name", ["c1", "t8j", "deg4"])
def test_workloads_meet_the_assemble_contract(name):
    """What vb_assemble requires of its input (row pointers rising from 0 to
    nnz, column indices in range, known DoF kinds, interface ids covered by
    exactly one entity and held whole by each subdomain, at least two
    pressures, positive element volumes), checked on the generator's output,
    k = 4 included."""
    from inputs.workloads import make_workload
    wl, _ = make_workload(name, workers=1)
    n_iface = wl["n_iface"]
    owner = -np.ones(n_iface, np.int64)
    for e, E in enumerate(wl["ents"]):
        g = np.asarray(E["gids"])
        assert len(g) > 0 and np.all(owner[g] < 0)
        owner[g] = e
        con = np.asarray(E["con"])  # n_con x n rows over the entity's DoFs
        assert con.size == 0 or con.shape[-1] == len(g)
    assert np.all(owner >= 0)
    for sd in wl["subs"]:
        n = len(sd["kind"])
        ip = np.asarray(sd["indptr"])
        assert ip[0] == 0 and ip[-1] == len(sd["indices"]) and np.all(np.diff(ip) >= 0)
        ix = np.asarray(sd["indices"])
        assert ix.min() >= 0 and ix.max() < n
        kind = np.asarray(sd["kind"])
        assert set(np.unique(kind)) <= {0, 1, 2} and np.sum(kind == 2) >= 2
        pw = np.asarray(sd["pweight"])[kind == 2]
        assert np.all(np.isfinite(pw)) and np.all(pw > 0)
        gid = np.asarray(sd["gid"])[kind == 1]
        assert gid.min() >= 0 and gid.max() < n_iface
        for e in np.unique(owner[gid]):  # every entity it touches, whole
            assert np.sum(owner[gid] == e) == len(wl["ents"][e]["gids"])


@pytest.mark.parametrize("name", ["c1", "t12u"])
def test_sub_box_labels_split_each_subdomain(name):
    """The sub-box labels of every subdomain: a geometric halving of its box
    of elements; the eliminated DoFs of two sub-boxes never share a matrix
    entry, every pressure lies in a sub-box, interface DoFs carry -1, and
    the separator (interior velocities labelled -1) is exactly the set of
    interior velocities coupled to two or more sub-boxes."""
    import scipy.sparse as sp
    from inputs.workloads import make_workload
    wl, _ = make_workload(name, workers=2)
    for sd in wl["subs"]:
        kind, part = sd["kind"], sd["part"]
        n = len(kind)
        K = sp.csr_matrix((sd["data"], sd["indices"], sd["indptr"]), shape=(n, n)).tocoo()
        a, b = part[K.row], part[K.col]
        assert not np.any((a >= 0) & (b >= 0) & (a != b))
        assert np.all(part[kind == 2] >= 0) and np.all(part[kind == 1] == -1)
        nb = part.max() + 1
        assert 1 <= nb <= 8 and set(np.unique(part[part >= 0])) == set(range(nb))
        # interior velocity DoFs reached from several sub-boxes' eliminated DoFs
        elim = part >= 0
        touch = sp.csr_matrix((np.ones(K.nnz)[elim[K.col]], (K.row[elim[K.col]], part[K.col][elim[K.col]])),
                              shape=(n, nb))
        multi = np.asarray((touch > 0).sum(axis=1)).ravel() >= 2
        sep = (kind == 0) & (part < 0)
        assert np.all(sep <= multi | (np.asarray((touch > 0).sum(axis=1)).ravel() == 0))
        assert not np.any(multi & (kind == 0) & (part >= 0))


def test_scaled_family_equals_per_problem_decomposition():
    """One decomposition scaled by each problem's subdomain viscosity gives
    the per-problem decomposition's workloads (make_family) to rounding:
    velocity-velocity entries and velocity right-hand sides scale with the
    subdomain's nu, divergence rows and pressure right-hand sides do not."""
    from inputs.workloads import make_family, scaled_family
    seeds = [3, 4]
    ref = make_family("c5s", seeds, workers=1, n=6, parts=(2, 2, 2))
    got = list(scaled_family("c5s", seeds, workers=1, n=6, parts=(2, 2, 2)))
    for a, b in zip(got, ref):
        assert a["n_iface"] == b["n_iface"]
        for sa, sb in zip(a["subs"], b["subs"]):
            for key in ("indptr", "indices", "kind", "gid"):
                assert np.array_equal(sa[key], sb[key]), key
            scale = np.abs(sb["data"]).max()
            assert np.abs(sa["data"] - sb["data"]).max() <= 1e-13 * scale
            assert np.abs(sa["rhs"] - sb["rhs"]).max() <= 1e-13 * np.abs(sb["rhs"]).max()


def test_neumann_sides_free_their_open_interior():
    """The paper's boundary conditions (Sec. 7: Neumann on two faces of the
    cube, no-slip on the others): with the sides x = 0 and x = 1 natural, a
    vertex is Dirichlet exactly when one of its other coordinates is on the
    boundary; the default (no Neumann side) is the whole boundary."""
    m = CubeMesh(4, jitter=0.0)
    n = m.n
    from inputs.assemble import dirichlet_entities
    vb0, eb0, fb0 = dirichlet_entities(m)
    assert np.array_equal(vb0, m.vert_bnd) and np.array_equal(eb0, m.edge_bnd)
    assert np.array_equal(fb0, m.face_bnd)
    vb, eb, fb = dirichlet_entities(m, (0, 1))
    yz = m.vidx[:, 1:]
    assert np.array_equal(vb, np.any((yz == 0) | (yz == n), axis=1))
    # faces: the boundary faces with a y or z normal only
    assert np.array_equal(fb, m.face_bnd & (m.face_axis != 0))
    # edges: both endpoints on one no-slip side
    ev = m.edge_verts
    both = np.zeros(m.nE, bool)
    for a in (1, 2):
        for v in (0, n):
            both |= (m.vidx[ev[:, 0], a] == v) & (m.vidx[ev[:, 1], a] == v)
    assert np.array_equal(eb, both)


def test_neumann_problem_has_no_pressure_kernel():
    """With two Neumann sides the reduced system is nonsingular without the
    mean-pressure constraint (the constant pressure is not in its kernel,
    unlike the no-slip problem), and the direct solve satisfies it; the
    workload carries the flags through decomposition and storage, and the
    library binding refuses it (its condensation assumes the no-slip
    structure)."""
    m = CubeMesh(4, jitter=0.15, seed=2)
    pb = Problem(m, 2, neumann_sides=(0, 1))
    assert not pb.pressure_kernel
    K, g, free = pb.reduced_system()
    ones_p = (free >= pb.Nvr).astype(float)
    assert np.linalg.norm(K @ ones_p) > 1e-3 * np.sqrt(ones_p.sum())
    pb0 = Problem(m, 2)
    K0, g0, free0 = pb0.reduced_system()
    ones0 = (free0 >= pb0.Nvr).astype(float)
    assert np.linalg.norm(K0 @ ones0) < 1e-10 * np.sqrt(ones0.sum())
    x = pb.solve_reduced_direct()
    assert np.linalg.norm(K @ x[free] - g) <= 1e-10 * np.linalg.norm(g)
    dec = Decomposition(pb, regular_cuts(4, (2, 2, 1)))
    wl = dec.workload()
    assert wl["pressure_kernel"] is False
    # interface DoFs on the Neumann side belong to the open faces and edges of
    # the cut planes (x = 0 is not a cut)
    assert all(key[1][0] not in (("cut", 0), ("cut", 2)) for key in dec.ent_key)
    import tempfile
    from inputs.workloads import save_workload, load_workload
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "wl.npz")
        save_workload(path, wl)
        back = load_workload(path)
        assert back["pressure_kernel"] is False
        assert np.array_equal(back["has_p0"], wl["has_p0"])
    # every subdomain of a 2 x 2 x 1 split has a side on x = 0 or x = 1
    assert not wl["has_p0"].any()
    from paper_2304_09770_amd import binding
    with pytest.raises(NotImplementedError):
        binding.vb_assemble(None, wl)


@pytest.mark.parametrize("n,cuts,sides", [
    (8, lambda: regular_cuts(8, (2, 2, 2)), ()),
    (6, lambda: random_cuts(6, 1, 3, 3, 2), ()),
    (6, lambda: regular_cuts(6, (3, 2, 2)), (0, 1)),
    (5, lambda: random_cuts(5, 1, 3, 2, 1), (4,)),
])
def test_entities_are_the_classes_of_shared_dofs(n, cuts, sides):
    """Interface entities (Sec. 5.1) are the classes of interface DoFs
    shared by the same set of subdomains: the decomposition's geometric
    classification (cut planes, their lines and points; Neumann sides
    uncut) must give exactly that partition, and every entity's subdomain
    list must be the set its DoFs are shared by."""
    pb = Problem(CubeMesh(n, jitter=0.1, seed=1), 2, workers=1, neumann_sides=sides)
    dec = Decomposition(pb, cuts(), ("vertex", "edge", "face", "flux"))
    mask = {}
    for s, sd in enumerate(dec.subs):
        for d in sd.dofs[sd.kind == 1]:
            mask[int(d)] = mask.get(int(d), 0) | (1 << s)
    assert sorted(mask) == sorted(int(r) for r in dec.iface_red)
    assert all(bin(m).count("1") >= 2 for m in mask.values())
    classes = {}
    for r, m in mask.items():
        classes.setdefault(m, set()).add(r)
    ents = [set(int(r) for r in dec.iface_red[g]) for g in dec.ent_dofs]
    assert sorted(map(sorted, ents)) == sorted(map(sorted, classes.values()))
    for e, g in enumerate(dec.ent_dofs):
        m = mask[int(dec.iface_red[g[0]])]
        assert set(dec.ent_subs[e].tolist()) == {s for s in range(len(dec.subs)) if m >> s & 1}
