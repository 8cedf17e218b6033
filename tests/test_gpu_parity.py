"""Parity of the HIP library against the CPU oracle (FP64 path).

Tolerance: the paper's method in FP64 is required to match the oracle's
solution to 1e-10 relative; operator applications (S_hat x, M^-1 r, g_hat)
are compared to 1e-11 relative (dense FP64 with different factorisations:
the differences are rounding of well-conditioned local solves).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs.workloads import make_workload
from oracle.bddc import OracleBDDC
from oracle.pcg import pcg

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def vb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09770_amd import binding
    binding.load()
    return binding


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("aligned", [False, True])
def test_batched_ldl_schur_matches_definition(vb, aligned):
    """Partial signed LDL^T: trailing block = A22 - A21 A11^-1 A21^T, with
    A11 a saddle matrix [[SPD, B^T], [B, 0]] (velocity pivots +, pressure -).
    aligned: leading dimensions rounded up to 32 (16-byte aligned columns,
    as the library lays out its own matrices), so the trailing updates load
    their panel strips straight into LDS; otherwise n + 3 (the staged
    kernels)."""
    rng = np.random.default_rng(0)
    # small cases, and cases whose elimination crosses the boundaries of the
    # inner (256) and outer (1024) super-panels of the blocked factorisation
    cases = [(200, 150, 120), (97, 70, 64), (130, 129, 100), (64, 64, 64),
             (1300, 1024, 900), (1500, 1100, 1000), (2600, 2300, 2000)]
    mats, ptrs, ns, lds, es, ps, refs = [], [], [], [], [], [], []
    for n, e, p in cases:
        Q = rng.standard_normal((n, n))
        A = Q @ Q.T / n + np.eye(n)
        A[p:e, p:e] = 0.0  # saddle: zero pressure block, B rows full rank
        ld = (n + 31) // 32 * 32 if aligned else n + 3
        M = np.zeros((ld, n))
        M[:n, :n] = A
        t = _dev(M.T.copy())  # column-major storage: row-major transpose
        mats.append(t)
        ptrs.append(t.data_ptr())
        ns.append(n)
        lds.append(ld)
        es.append(e)
        ps.append(p)
        S = A[e:, e:] - A[e:, :e] @ np.linalg.solve(A[:e, :e], A[:e, e:])
        refs.append((A, S))
    dptr = torch.tensor(ptrs, dtype=torch.int64, device=DEV)
    i32 = lambda v: torch.tensor(v, dtype=torch.int32, device=DEV)
    info = i32([0] * len(cases))
    ctx = vb.vb_create()
    try:
        vb.vb_batched_ldl(ctx, dptr, i32(ns), i32(lds), i32(es), i32(ps), info, max(ns), max(es))
    finally:
        vb.vb_destroy(ctx)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0] * len(cases)
    for t, (A, S), n, ld, e, p in zip(mats, refs, ns, lds, es, ps):
        M = t.cpu().numpy().T[:n, :n]
        if e < n:
            Sg = np.tril(M[e:, e:])
            assert np.abs(Sg - np.tril(S)).max() < 1e-11 * np.abs(S).max()
        L = np.tril(M[:e, :e])
        d = np.where(np.arange(e) < p, 1.0, -1.0)
        assert np.abs(L @ np.diag(d) @ L.T - A[:e, :e]).max() < 1e-11 * np.abs(A).max()


def test_batched_ldl_reports_wrong_signed_pivot(vb):
    n = 80
    A = -np.eye(n)  # negative definite but declared all-positive
    t = _dev(A)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    i32 = lambda v: torch.tensor(v, dtype=torch.int32, device=DEV)
    ctx = vb.vb_create()
    try:
        vb.vb_batched_ldl(ctx, torch.tensor([t.data_ptr()], dtype=torch.int64, device=DEV),
                          i32([n]), i32([n]), i32([40]), i32([40]), info, n, 40)
    finally:
        vb.vb_destroy(ctx)
    assert info.item() == 1  # first column


_PROBLEMS = {}


def _problem(name):
    """Workload and oracle, built once per module for both precisions."""
    if name not in _PROBLEMS:
        wl, meta = make_workload(name, workers=1)
        _PROBLEMS[name] = (wl, meta, OracleBDDC(wl))
    return _PROBLEMS[name]


# c1, t8j, t12: tiles and ragged panels, 2/4/8-way sharing; t12u: uneven
# cuts (2..6 elements per side, the shape of the 216-subdomain workload);
# t12b: 6^3-element subdomains (3,560 eliminated columns each in one dense
# factorisation: several outer super-panels on 16-byte aligned matrices);
# t8k3, t6k4: degrees 3 and 4.  nested: the two-level factorisation (each
# subdomain's sub-boxes first, then its separators), else one dense
# factorisation per subdomain.
FP64_CASES = [("c1", True), ("t8j", True), ("t12", True), ("t12u", True), ("t12b", True),
              ("t8k3", True), ("t6k4", True), ("c1", False), ("t12u", False), ("t12b", False)]
MIXED_CASES = [("c1", True), ("t8j", True), ("t12", True), ("t12u", True), ("t8k3", True),
               ("t6k4", True), ("t8j", False), ("t12u", False)]


def _ids(cases):
    return ["%s-%s" % (n, "nested" if nd else "dense") for n, nd in cases]


@pytest.fixture(scope="module", params=FP64_CASES, ids=_ids(FP64_CASES))
def case(request, vb):
    name, nested = request.param
    print("fp64 case", name, "nested" if nested else "dense", flush=True)
    wl, meta, o = _problem(name)
    ctx = vb.vb_create(tol=1e-8)
    vb.vb_assemble(ctx, wl, nested=nested)
    vb.vb_setup(ctx)
    yield name, wl, meta, o, ctx
    vb.vb_destroy(ctx)


def test_rhs_parity(vb, case):
    name, wl, meta, o, ctx = case
    n = vb.vb_interface_size(ctx)
    g = torch.zeros(n, dtype=torch.float64, device=DEV)
    vb.vb_rhs(ctx, g)
    torch.cuda.synchronize()
    assert _rel(g.cpu().numpy(), o.rhs()) < 1e-11


def test_schur_apply_parity(vb, case):
    name, wl, meta, o, ctx = case
    n = vb.vb_interface_size(ctx)
    rng = np.random.default_rng(1)
    for _ in range(2):
        x = rng.standard_normal(n)
        y = torch.zeros(n, dtype=torch.float64, device=DEV)
        vb.vb_schur_apply(ctx, _dev(x), y)
        torch.cuda.synchronize()
        assert _rel(y.cpu().numpy(), o.apply_S(x)) < 1e-11


def test_preconditioner_parity(vb, case):
    name, wl, meta, o, ctx = case
    n = vb.vb_interface_size(ctx)
    rng = np.random.default_rng(2)
    for _ in range(2):
        r = o.apply_S(rng.standard_normal(n))  # a residual in the range of S_hat
        z = torch.zeros(n, dtype=torch.float64, device=DEV)
        vb.vb_apply(ctx, _dev(r), z)
        torch.cuda.synchronize()
        zo = o.apply_M(r)
        nG = o.nG
        # p0 part defined up to the constant kernel: compare velocity part and p0 differences
        zg = z.cpu().numpy()
        assert _rel(zg[:nG], zo[:nG]) < 1e-10
        dp = (zg[nG:] - zg[nG:].mean()) - (zo[nG:] - zo[nG:].mean())
        assert np.linalg.norm(dp) < 1e-10 * max(np.linalg.norm(zo[nG:]), 1e-300) + 1e-12 * np.linalg.norm(zo)


def test_pcg_same_iterate_and_solution(vb, case):
    name, wl, meta, o, ctx = case
    n = vb.vb_interface_size(ctx)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    info = vb.vb_pcg_solve(ctx, x)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    K = info["iterations"]
    assert info["true_rel_residual"] <= 1e-8 * 1.01
    xo, oi = pcg(o.apply_S, o.apply_M, o.rhs(), fixed_iters=K)
    assert _rel(xg, xo) < 1e-10, (K, _rel(xg, xo))
    assert info["lambda_min"] > 1 - 1e-6
    # against the direct solve of the assembled system
    pb, dec = meta["problem"], meta["decomposition"]
    uG, p0 = dec.interface_solution(pb.solve_reduced_direct())
    ref = np.concatenate([uG, p0])
    assert _rel(xg, ref) < 1e-6


def test_interior_recovery_parity(vb, case):
    name, wl, meta, o, ctx = case
    n = vb.vb_interface_size(ctx)
    xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-12)
    xd = _dev(xo)
    rec = o.recover(xo)
    for s in (0, len(wl["subs"]) - 1):
        sd = wl["subs"][s]
        u = vb.vb_get_local_solution(ctx, xd, s, len(sd["kind"]))
        kind = sd["kind"]
        uI, c = rec[s]
        assert _rel(u[kind == 0], uI) < 1e-10
        # pressures are O(h^2) here (exact pressure 0): compare the local
        # solution vector as a whole, the scale both local solves work in
        both_g = np.concatenate([u[kind == 0], u[kind == 2]])
        both_o = np.concatenate([uI, c])
        assert _rel(both_g, both_o) < 1e-10
        assert _rel(u[kind == 1], xo[sd["gid"][kind == 1]]) < 1e-15


# ------------------------------------------------------------ mixed precision
# FP32 local factors and Schur operators with FP64 refinement.  The refined
# solution is the FP64 one: the outer residual is formed in FP64 from the
# sparse local systems, so the tolerance is the FP64 path's (1e-10 relative
# against the oracle solved to 1e-13), not an FP32 one.

@pytest.fixture(scope="module", params=MIXED_CASES, ids=_ids(MIXED_CASES))
def mixed_case(request, vb):
    name, nested = request.param
    print("mixed case", name, "nested" if nested else "dense", flush=True)
    wl, meta, o = _problem(name)
    ctx = vb.vb_create(precision=vb.VB_PREC_MIXED, tol=1e-12)
    vb.vb_assemble(ctx, wl, nested=nested)
    vb.vb_setup(ctx)
    yield name, wl, meta, o, ctx
    vb.vb_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
def test_two_level_factorisation_equals_single_level(vb, precision):
    """The two-level (sub-boxes, then separators) factorisation is an exact
    reordering of the single-level one: same S_hat, g_hat, solution and
    local solutions to rounding (FP64); in mixed precision both reach the
    FP64 solution."""
    wl, meta, o = _problem("t12u")
    out = []
    for nested in (True, False):
        ctx = vb.vb_create(precision=precision, tol=1e-8 if precision == 0 else 1e-12)
        try:
            vb.vb_assemble(ctx, wl, nested=nested)
            vb.vb_setup(ctx)
            n = vb.vb_interface_size(ctx)
            g = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_rhs(ctx, g)
            xr = torch.tensor(np.random.default_rng(4).standard_normal(n), device=DEV)
            y = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_schur_apply(ctx, xr, y)
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            info = vb.vb_pcg_solve(ctx, x)
            u = torch.zeros(vb.vb_local_size(ctx), dtype=torch.float64, device=DEV)
            vb.vb_recover_all(ctx, x, u)
            torch.cuda.synchronize()
            out.append((g.cpu().numpy(), y.cpu().numpy(), x.cpu().numpy(), u.cpu().numpy(), info))
        finally:
            vb.vb_destroy(ctx)
    (g1, y1, x1, u1, i1), (g0, y0, x0, u0, i0) = out
    if precision == 0:
        assert _rel(g1, g0) < 1e-12 and _rel(y1, y0) < 1e-12
        assert i1["iterations"] == i0["iterations"]
        assert _rel(x1, x0) < 1e-11 and _rel(u1, u0) < 1e-10
    else:
        assert _rel(x1, x0) < 1e-10 and _rel(u1, u0) < 1e-9


def test_mixed_solution_parity(vb, mixed_case):
    name, wl, meta, o, ctx = mixed_case
    n = vb.vb_interface_size(ctx)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    info = vb.vb_pcg_solve(ctx, x)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    assert 1 <= info["refinement_steps"] <= 12, info
    assert info["true_rel_residual"] <= 1e-12
    # FP64 interface residual of the refined solution, on the oracle's operator
    g = o.rhs()
    assert np.linalg.norm(g - o.apply_S(xg)) <= 1e-10 * np.linalg.norm(g)
    xo, _ = pcg(o.apply_S, o.apply_M, g, tol=1e-13)
    assert _rel(xg, xo) < 1e-10, _rel(xg, xo)


def test_mixed_interior_recovery_parity(vb, mixed_case):
    name, wl, meta, o, ctx = mixed_case
    xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-12)
    xd = _dev(xo)
    rec = o.recover(xo)
    for s in (0, len(wl["subs"]) - 1):
        sd = wl["subs"][s]
        u = vb.vb_get_local_solution(ctx, xd, s, len(sd["kind"]))
        kind = sd["kind"]
        uI, c = rec[s]
        both_g = np.concatenate([u[kind == 0], u[kind == 2]])
        both_o = np.concatenate([uI, c])
        assert _rel(both_g, both_o) < 1e-10
        assert _rel(u[kind == 1], xo[sd["gid"][kind == 1]]) < 1e-15


def test_mixed_recovery_from_the_solve_state(vb, mixed_case):
    """Recovery at the interface solution of the last mixed solve starts from
    the interior state refined with it, on the condensed residual of the
    solve's final check (one pass); a second recovery at the same x starts
    from the state the first one left.  Both must give the oracle's recovery
    from that same interface solution."""
    name, wl, meta, o, ctx = mixed_case
    n = vb.vb_interface_size(ctx)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    vb.vb_pcg_solve(ctx, x)
    nloc = sum(len(sd["kind"]) for sd in wl["subs"])
    u = torch.zeros(nloc, dtype=torch.float64, device=DEV)
    u2 = torch.zeros(nloc, dtype=torch.float64, device=DEV)
    vb.vb_recover_all(ctx, x, u)
    vb.vb_recover_all(ctx, x, u2)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    rec = o.recover(xg)
    for ug in (u.cpu().numpy(), u2.cpu().numpy()):
        off = 0
        for s, sd in enumerate(wl["subs"]):
            kind = sd["kind"]
            us = ug[off: off + len(kind)]
            off += len(kind)
            uI, c = rec[s]
            assert _rel(np.concatenate([us[kind == 0], us[kind == 2]]), np.concatenate([uI, c])) < 1e-10
            assert _rel(us[kind == 1], xg[sd["gid"][kind == 1]]) < 1e-15


@pytest.mark.parametrize("inner_tol", [0.0, 1e-2])
def test_mixed_refinement_history_and_inner_tolerance(vb, inner_tol):
    """vb_refinement_history reports the condensed residual before every
    refinement step (1 first) and after the last (at or below the
    tolerance), decreasing, and the inner iterations, which add up to the
    solve's; a looser inner tolerance (vb_options.inner_tol) reaches the
    oracle's solution all the same."""
    wl, meta, o = _problem("t12u")
    ctx = vb.vb_create(precision=vb.VB_PREC_MIXED, tol=1e-12, inner_tol=inner_tol)
    try:
        vb.vb_assemble(ctx, wl, nested=True)
        vb.vb_setup(ctx)
        assert vb.vb_refinement_history(ctx) == ([], [])
        n = vb.vb_interface_size(ctx)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = vb.vb_pcg_solve(ctx, x)
        rel, inner = vb.vb_refinement_history(ctx)
        torch.cuda.synchronize()
    finally:
        vb.vb_destroy(ctx)
    print("inner_tol", inner_tol, "history", rel, inner, flush=True)
    assert len(inner) == info["refinement_steps"] and len(rel) == len(inner) + 1
    assert rel[0] == 1.0 and rel[-1] <= 1e-12 and all(b < a for a, b in zip(rel, rel[1:]))
    assert sum(inner) == info["iterations"] and min(inner) >= 1
    xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-13)
    assert _rel(x.cpu().numpy(), xo) < 1e-10


def test_mixed_operators_are_fp32_roundings(vb, mixed_case):
    """S_hat and M^-1 from the FP32 factorisations differ from the FP64 ones
    by FP32 rounding amplified by the local conditioning, and are not
    identical."""
    name, wl, meta, o, ctx = mixed_case
    n = vb.vb_interface_size(ctx)
    x = np.random.default_rng(3).standard_normal(n)
    y = torch.zeros(n, dtype=torch.float64, device=DEV)
    vb.vb_schur_apply(ctx, _dev(x), y)
    torch.cuda.synchronize()
    d = _rel(y.cpu().numpy(), o.apply_S(x))
    assert 1e-12 < d < 1e-3, d
    # M^-1 is built from that S_hat (its local Neumann factors are FP32 too;
    # coarse factorisation and deluxe scaling FP64): its relative change is
    # the change of S_hat, or FP32 rounding, amplified by the conditioning of
    # the local Neumann blocks S_DD that it inverts
    # (compared like the FP64 preconditioner: on a residual in the range of
    # S_hat, the p0 part up to the constant kernel)
    r = o.apply_S(x)
    z = torch.zeros(n, dtype=torch.float64, device=DEV)
    vb.vb_apply(ctx, _dev(r), z)
    torch.cuda.synchronize()
    zg, zo, nG = z.cpu().numpy(), o.apply_M(r), o.nG
    zg[nG:] -= zg[nG:].mean()
    zo[nG:] -= zo[nG:].mean()
    dm = _rel(zg, zo)
    kappa = max(np.linalg.cond(L.St[np.ix_(L.Dl, L.Dl)]) for L in o.loc if len(L.Dl))
    assert 1e-12 < dm < 10.0 * kappa * max(d, 2.0 ** -24), (dm, d, kappa)
