"""Pins of the oracle's adaptive face eigenproblems (Sec. 6) against what the
mathematics fixes: the closed form of the parallel sum, the Schur complement
as the inverse of a block of the inverse, the Loewner bound lambda in [0, 1],
the rigid-mode cluster of faces next to a floating subdomain
(ker X:Y = ker X + ker Y), Sylvester's inertia for the selected count, the
all-selected limit, and the effect on the condition number; for the
optional edge eigenproblems (parallel sums over all subdomains sharing an
edge) the closed form of a several-term parallel sum, lambda in [0, 1], the
all-selected limit and a lower kappa_2 than faces alone."""
import numpy as np
import pytest
import scipy.linalg as sla

from inputs.mesh import CubeMesh
from inputs.assemble import Problem
from inputs.decompose import Decomposition, regular_cuts
from oracle.adaptive import parallel_sum, schur_onto, face_pencil
from oracle.bddc import OracleBDDC
from oracle.pcg import pcg, lanczos_extremes

FULL = ("vertex", "edge", "face", "flux")
CENTER = 13  # subdomain (1,1,1) of a 3x3x3 decomposition: no boundary face


def _spd(rng, n, rank=None):
    G = rng.standard_normal((n, rank or n))
    return G @ G.T + (1e-1 * np.eye(n) if rank is None else 0.0)


def test_parallel_sum_closed_form():
    rng = np.random.default_rng(0)
    X, Y = _spd(rng, 9), _spd(rng, 9)
    ref = np.linalg.inv(np.linalg.inv(X) + np.linalg.inv(Y))
    assert np.abs(parallel_sum(X, Y) - ref).max() < 1e-12 * np.abs(ref).max()
    # diagonal PSD: x y / (x + y), zero where either vanishes
    x, y = np.array([1.0, 2.0, 0.0, 3.0]), np.array([0.0, 2.0, 5.0, 1.0])
    assert np.allclose(parallel_sum(np.diag(x), np.diag(y)),
                       np.diag([0.0, 1.0, 0.0, 0.75]), atol=1e-14)


def test_schur_onto_is_inverse_of_block_of_inverse_and_keeps_kernel():
    rng = np.random.default_rng(1)
    S = _spd(rng, 12)
    keep = [2, 5, 7, 11]
    ref = np.linalg.inv(np.linalg.inv(S)[np.ix_(keep, keep)])
    assert np.abs(schur_onto(S, keep) - ref).max() < 1e-11 * np.abs(ref).max()
    # singular S (rank 9): a kernel vector restricted to `keep` is in the kernel
    Ss = _spd(rng, 12, rank=9)
    z = sla.null_space(Ss)[:, 0]
    R = schur_onto(Ss, keep)
    assert np.linalg.norm(R @ z[keep]) < 1e-9 * np.linalg.norm(R) * np.linalg.norm(z[keep])


@pytest.fixture(scope="module")
def floating():
    pb = Problem(CubeMesh(6, jitter=0.15, seed=3), 2, 1.0, workers=1)
    dec = Decomposition(pb, regular_cuts(6, (3, 3, 3)), FULL)
    return pb, dec, OracleBDDC(dec.workload())


def _faces(o):
    return [e for e, E in enumerate(o.ents) if E["kind"] == 2 and len(o.de_idx[e])]


def test_face_eigenvalues_in_unit_interval_and_rigid_cluster(floating):
    pb, dec, o = floating
    nfloat = 0
    for e in _faces(o):
        Atp, Ap, subs = face_pencil(o, e)
        lam = sla.eigh(Atp, Ap, eigvals_only=True)
        assert lam.min() > -1e-9 and lam.max() < 1 + 1e-9
        small = int(np.sum(lam < 1e-8))
        if CENTER in subs:
            nfloat += 1
            assert small == 6, (e, subs, lam[:8])
        else:
            assert small == 0, (e, subs, lam[:3])
    assert nfloat == 6


def test_selected_count_matches_inertia(floating):
    pb, dec, o = floating
    for e in _faces(o)[:8]:
        Atp, Ap, _ = face_pencil(o, e)
        lam = sla.eigh(Atp, Ap, eigvals_only=True)
        for sigma in (0.1, 0.5):
            _, D, _ = sla.ldl(Atp - sigma * Ap)
            neg = int(np.sum(np.linalg.eigvalsh(D) < 0))   # D: 1x1/2x2 blocks
            assert neg == int(np.sum(lam < sigma))


def test_all_selected_makes_faces_primal(floating):
    pb, dec, o = floating
    oa = OracleBDDC(dec.workload(), adaptive_theta=0.5)   # 1/theta = 2 > every lambda
    for e in _faces(o):
        assert oa.npi[e] == len(o.ents[e]["gids"])


def test_adaptive_bounds_condition_and_keeps_solution():
    """kappa_2 decreases with theta; at theta = 10 it is within the sanity
    band 2 theta (the constant of the bound is not given by the paper, and
    only faces are enriched, so edges cap what small theta can reach); PCG
    reaches the same solution (the direct solve)."""
    from inputs.workloads import sinker_viscosity
    mesh = CubeMesh(6, jitter=0.0, seed=0)
    nu = sinker_viscosity(mesh, n_sinkers=4, radius=0.25, nu_in=1e4, seed=1)
    pb = Problem(mesh, 2, nu, workers=1)
    dec = Decomposition(pb, regular_cuts(6, (3, 3, 3)), FULL)
    wl = dec.workload()
    ref = np.concatenate(dec.interface_solution(pb.solve_reduced_direct()))
    k2 = {}
    for theta in (0.0, 10.0, 2.0):
        o = OracleBDDC(wl, adaptive_theta=theta)
        x, info = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-10)
        lmin, lmax = lanczos_extremes(info["alphas"], info["betas"])
        assert lmin > 1 - 1e-8
        k2[theta] = lmax / lmin
        assert np.linalg.norm(x - ref) <= 1e-6 * np.linalg.norm(ref)
    assert k2[10.0] <= 20.0, k2
    assert k2[0.0] > 10 * k2[10.0], k2
    assert k2[2.0] <= k2[10.0] * 1.001, k2


# ------------------------------------------------- edges (beyond the paper's text)
def _edges(o):
    return [e for e, E in enumerate(o.ents)
            if E["kind"] == 1 and len(o.ent_subs[e]) >= 2 and len(o.de_idx[e])]


def test_parallel_sum_of_several_is_the_inverse_of_summed_inverses():
    rng = np.random.default_rng(2)
    X, Y, Z, W = (_spd(rng, 7) for _ in range(4))
    ref = np.linalg.inv(sum(np.linalg.inv(M) for M in (X, Y, Z, W)))
    fold = parallel_sum(parallel_sum(parallel_sum(X, Y), Z), W)
    assert np.abs(fold - ref).max() < 1e-12 * np.abs(ref).max()


def test_edge_eigenvalues_in_unit_interval(floating):
    """At^(k) <= A^(k) in the Loewner order for every sharing subdomain, and
    the parallel sum is monotone, so the edge pencil's eigenvalues lie in
    [0, 1] like the faces'."""
    pb, dec, o = floating
    edges = _edges(o)
    assert any(len(o.ent_subs[e]) == 4 for e in edges)
    for e in edges:
        Atp, Ap, subs = face_pencil(o, e)
        lam = sla.eigh(Atp, Ap, eigvals_only=True)
        assert lam.min() > -1e-9 and lam.max() < 1 + 1e-9, (e, subs)


def test_all_selected_makes_edges_primal(floating):
    pb, dec, o = floating
    oa = OracleBDDC(dec.workload(), adaptive_theta=0.5, adaptive_edges=True)
    for e in _edges(o):
        assert oa.npi[e] == len(o.ents[e]["gids"])


def test_edge_enrichment_lowers_the_condition_number(floating):
    """At theta = 2 the edges' eigenproblems take kappa_2 below the
    faces-only value; lambda_min stays 1 and PCG reaches the direct solve."""
    pb, dec, o = floating
    wl = dec.workload()
    ref = np.concatenate(dec.interface_solution(pb.solve_reduced_direct()))
    k2 = {}
    for edges in (False, True):
        oe = OracleBDDC(wl, adaptive_theta=2.0, adaptive_edges=edges)
        x, info = pcg(oe.apply_S, oe.apply_M, oe.rhs(), tol=1e-10)
        lmin, lmax = lanczos_extremes(info["alphas"], info["betas"])
        assert lmin > 1 - 1e-8
        assert np.linalg.norm(x - ref) <= 1e-6 * np.linalg.norm(ref)
        k2[edges] = lmax / lmin
    assert k2[True] < k2[False], k2


def test_adaptive_space_with_neumann_sides():
    """Sec. 6 on the paper's boundary conditions (Neumann sides x = 0 and
    x = 1, where subdomains touching them keep no p0): the enriched space
    keeps the direct solve's solution and lowers the condition number of
    the minimal space, with lambda_min still at least 1."""
    pb = Problem(CubeMesh(4, jitter=0.15, seed=3), 2, 1.0, workers=1, neumann_sides=(0, 1))
    dec = Decomposition(pb, regular_cuts(4, (3, 2, 2)), ("vertex", "edge", "flux"))
    wl = dec.workload()
    ref = np.concatenate(dec.interface_solution(pb.solve_reduced_direct()))
    kappa = []
    for theta in (0.0, 0.5):
        o = OracleBDDC(wl, adaptive_theta=theta)
        x, info = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-12)
        assert np.linalg.norm(x - ref) < 1e-9 * np.linalg.norm(ref)
        lmin, lmax = lanczos_extremes(info["alphas"], info["betas"])
        assert lmin > 1 - 1e-8
        kappa.append(lmax / lmin)
    assert kappa[1] < 0.75 * kappa[0]
