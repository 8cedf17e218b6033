"""Several independent problems in one context (one launch per step covers
every subdomain of every problem; PCG keeps scalars and convergence per
problem) and the HIP-graph replay of the PCG iteration.

Each problem of a batched context must reproduce its own single-problem
solve: same iteration count (the recurrences are the same, only the
grouping of the reductions' partial sums can differ) and the same solution
to 1e-10 relative; the operators of the batched context are block diagonal.
The graph-replayed iteration must give the eager iteration's result (same
kernels and arguments), on every one of several solves in a row.  Forming
the local Neumann matrices in waves of subdomains (a setup memory limit)
runs the same per-subdomain arithmetic, so it must not change the result;
neither must forming, factoring and condensing the dense local Dirichlet
matrices in waves (compact condensed blocks, factors recomputed for the
interior recovery)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs.workloads import make_workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CASES = [("c1", 0), ("t8j", 0), ("t6f", 0)]


@pytest.fixture(scope="module")
def vb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09770_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def wls():
    return [make_workload(name, seed=seed, workers=1)[0] for name, seed in CASES]


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _single(vb, wl, **kw):
    ctx = vb.vb_create(**kw)
    vb.vb_assemble(ctx, wl)
    vb.vb_setup(ctx)
    n = vb.vb_interface_size(ctx)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    info = vb.vb_pcg_solve(ctx, x)
    out = {"x": x.cpu().numpy(), "info": info, "n_iface": int(wl["n_iface"]),
           "n_sub": len(wl["subs"])}
    g = torch.zeros(n, dtype=torch.float64, device=DEV)
    vb.vb_rhs(ctx, g)
    out["g"] = g.cpu().numpy()
    vb.vb_destroy(ctx)
    return out


def _split(vb, ctx, v, k):
    L = vb.vb_problem_layout(ctx, k)
    a = v[L["iface_offset"]: L["iface_offset"] + L["n_iface"]]
    b = v[L["p0_offset"]: L["p0_offset"] + L["n_sub"]]
    return np.concatenate([a, b])


def test_batched_problems_match_single_solves(vb, wls):
    ref = [_single(vb, wl) for wl in wls]
    ctx = vb.vb_create()
    try:
        for wl in wls:
            vb.vb_assemble(ctx, wl)
        assert vb.vb_num_problems(ctx) == len(wls)
        vb.vb_setup(ctx)
        n = vb.vb_interface_size(ctx)
        assert n == sum(len(r["x"]) for r in ref)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = vb.vb_pcg_solve(ctx, x)
        g = torch.zeros(n, dtype=torch.float64, device=DEV)
        vb.vb_rhs(ctx, g)
        xg, gg = x.cpu().numpy(), g.cpu().numpy()
        its = []
        for k, r in enumerate(ref):
            pi = vb.vb_problem_solve_info(ctx, k)
            its.append(pi["iterations"])
            assert pi["iterations"] == r["info"]["iterations"], (k, pi["iterations"], r["info"]["iterations"])
            assert pi["true_rel_residual"] <= 1e-8 * 1.01
            assert pi["latency_ms"] > 0.0
            assert _rel(_split(vb, ctx, gg, k), r["g"]) < 1e-13
            assert _rel(_split(vb, ctx, xg, k), r["x"]) < 1e-10
        assert info["iterations"] == max(its)
        # block-diagonal operators: S_hat and M^-1 of the batch act per problem
        rng = np.random.default_rng(0)
        v = rng.standard_normal(n)
        y = torch.zeros(n, dtype=torch.float64, device=DEV)
        vb.vb_schur_apply(ctx, torch.tensor(v, device=DEV), y)
        yb = y.cpu().numpy()
        zb = torch.zeros(n, dtype=torch.float64, device=DEV)
        vb.vb_apply(ctx, torch.tensor(yb, device=DEV), zb)
        zb = zb.cpu().numpy()
    finally:
        vb.vb_destroy(ctx)
    for k, wl in enumerate(wls):
        c1 = vb.vb_create()
        vb.vb_assemble(c1, wl)
        vb.vb_setup(c1)
        nk = vb.vb_interface_size(c1)
        vk = torch.tensor(_split_layout(v, ref, k), device=DEV)
        yk = torch.zeros(nk, dtype=torch.float64, device=DEV)
        vb.vb_schur_apply(c1, vk, yk)
        zk = torch.zeros(nk, dtype=torch.float64, device=DEV)
        vb.vb_apply(c1, yk, zk)
        yk, zk = yk.cpu().numpy(), zk.cpu().numpy()
        vb.vb_destroy(c1)
        assert _rel(_split_layout(yb, ref, k), yk) < 1e-13
        assert _rel(_split_layout(zb, ref, k), zk) < 1e-11


def _split_layout(v, ref, k):
    """Problem k's part of a batched vector, from the single-problem sizes
    (interface sizes and subdomain counts in problem order)."""
    ni = [r["n_iface"] for r in ref]
    ns = [r["n_sub"] for r in ref]
    g0 = sum(ni[:k])
    p0 = sum(ni) + sum(ns[:k])
    return np.concatenate([v[g0: g0 + ni[k]], v[p0: p0 + ns[k]]])


def test_graph_replay_matches_eager(vb, wls):
    wl = wls[1]
    eager = _single(vb, wl)
    stream = torch.cuda.Stream(device=DEV)
    ctx = vb.vb_create(stream=stream.cuda_stream)
    try:
        vb.vb_assemble(ctx, wl)
        with torch.cuda.stream(stream):
            vb.vb_setup(ctx)
            n = vb.vb_interface_size(ctx)
            for rep in range(3):
                x = torch.zeros(n, dtype=torch.float64, device=DEV)
                torch.cuda.synchronize()
                info = vb.vb_pcg_solve(ctx, x)
                stream.synchronize()
                assert info["iterations"] == eager["info"]["iterations"]
                assert _rel(x.cpu().numpy(), eager["x"]) < 1e-13, rep
    finally:
        vb.vb_destroy(ctx)


def test_mixed_batched_reaches_fp64(vb, wls):
    ref = [_single(vb, wl, tol=1e-12) for wl in wls]
    ctx = vb.vb_create(precision=vb.VB_PREC_MIXED, tol=1e-12)
    try:
        for wl in wls:
            vb.vb_assemble(ctx, wl)
        vb.vb_setup(ctx)
        n = vb.vb_interface_size(ctx)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = vb.vb_pcg_solve(ctx, x)
        xg = x.cpu().numpy()
        for k, r in enumerate(ref):
            pi = vb.vb_problem_solve_info(ctx, k)
            assert pi["refinement_steps"] >= 1
            assert _rel(_split(vb, ctx, xg, k), r["x"]) < 1e-9
    finally:
        vb.vb_destroy(ctx)


@pytest.fixture(scope="module")
def oracles(wls):
    from oracle.bddc import OracleBDDC
    return [OracleBDDC(wl) for wl in wls]


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_graph_path_matches_oracle(vb, wls, oracles, precision):
    """Every problem of a batched context, solved on a stream of its own
    (the PCG iteration replayed as a HIP graph), against the oracle:
    FP64: the iterate after the problem's own iteration count equals the
    oracle's iterate after as many iterations (1e-10); mixed: the refined
    solution equals the oracle's solution to 1e-13 (1e-10)."""
    from oracle.pcg import pcg
    stream = torch.cuda.Stream(device=DEV)
    tol = 1e-8 if precision == 0 else 1e-12
    ctx = vb.vb_create(precision=precision, tol=tol, stream=stream.cuda_stream)
    try:
        for wl in wls:
            vb.vb_assemble(ctx, wl)
        with torch.cuda.stream(stream):
            vb.vb_setup(ctx)
            n = vb.vb_interface_size(ctx)
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_pcg_solve(ctx, x)
            stream.synchronize()
        xg = x.cpu().numpy()
        for k, o in enumerate(oracles):
            pi = vb.vb_problem_solve_info(ctx, k)
            xk = _split(vb, ctx, xg, k)
            if precision == 0:
                xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), fixed_iters=pi["iterations"])
            else:
                xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-13)
            assert _rel(xk, xo) < 1e-10, (k, precision, _rel(xk, xo))
    finally:
        vb.vb_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
def test_neumann_waves_match_one_wave(vb, wls, precision):
    wl = wls[2]
    one = _single(vb, wl, precision=precision)
    # a limit below any subdomain's augmented matrix: one subdomain per wave
    waves = _single(vb, wl, precision=precision, setup_mem_limit=1.0)
    assert waves["info"]["iterations"] == one["info"]["iterations"]
    assert _rel(waves["x"], one["x"]) < 1e-14


def test_dirichlet_waves_match_resident(vb, wls):
    # waves of dense local matrices: the single-level factorisation (the
    # two-level one keeps its smaller matrices resident)
    wl = wls[2]
    nloc = sum(len(sd["kind"]) for sd in wl["subs"])
    out = []
    for lim in (0.0, 1.0):  # resident; one subdomain per wave
        ctx = vb.vb_create(local_mem_limit=lim)
        try:
            vb.vb_assemble(ctx, wl, nested=False)
            vb.vb_setup(ctx)
            n = vb.vb_interface_size(ctx)
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            info = vb.vb_pcg_solve(ctx, x)
            u = torch.zeros(nloc, dtype=torch.float64, device=DEV)
            vb.vb_recover_all(ctx, x, u)
            torch.cuda.synchronize()
            out.append((info, x.cpu().numpy(), u.cpu().numpy()))
        finally:
            vb.vb_destroy(ctx)
    (i0, x0, u0), (i1, x1, u1) = out
    assert i1["iterations"] == i0["iterations"]
    assert _rel(x1, x0) < 1e-14
    assert _rel(u1, u0) < 1e-14


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_launch_matches_graph_and_oracle(vb, wls, oracles, precision):
    """The PCG iterations as one persistent cooperative launch (phases
    separated by grid barriers, convergence decided on the device) against
    the graph-replayed iteration: the same arithmetic in the same order, so
    the same iteration counts and solutions to rounding, for every problem of
    a batched context; and against the oracle (FP64: the iterate after the
    problem's own iteration count; mixed: the oracle's solution to 1e-13)."""
    from oracle.pcg import pcg
    tol = 1e-8 if precision == 0 else 1e-12
    out = {}
    for launch in (vb.VB_PCG_GRAPH, vb.VB_PCG_PERSISTENT):
        stream = torch.cuda.Stream(device=DEV)
        ctx = vb.vb_create(precision=precision, tol=tol, stream=stream.cuda_stream,
                           pcg_launch=launch)
        try:
            for wl in wls:
                vb.vb_assemble(ctx, wl)
            with torch.cuda.stream(stream):
                vb.vb_setup(ctx)
                n = vb.vb_interface_size(ctx)
                res = []
                for rep in range(2):  # a second solve reuses the launch plan
                    x = torch.zeros(n, dtype=torch.float64, device=DEV)
                    vb.vb_pcg_solve(ctx, x)
                    stream.synchronize()
                    res.append(x.cpu().numpy())
            assert vb.vb_pcg_launch_used(ctx) == launch
            its = [vb.vb_problem_solve_info(ctx, k)["iterations"] for k in range(len(wls))]
            out[launch] = (res, its, [_split(vb, ctx, res[0], k) for k in range(len(wls))])
        finally:
            vb.vb_destroy(ctx)
    (rg, ig, xg), (rp, ip, xp) = out[vb.VB_PCG_GRAPH], out[vb.VB_PCG_PERSISTENT]
    assert ip == ig
    assert _rel(rp[0], rg[0]) < 1e-14 and _rel(rp[1], rp[0]) < 1e-14
    for k, o in enumerate(oracles):
        if precision == 0:
            xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), fixed_iters=ip[k])
        else:
            xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-13)
        assert _rel(xp[k], xo) < 1e-10, (k, _rel(xp[k], xo))


@pytest.mark.parametrize("precision", [0, 1])
def test_symmetric_schur_kernel_matches_full_and_oracle(vb, wls, oracles, precision):
    """S_hat p and the local Neumann solves' S_DeltaDelta^-1 through the lower
    triangle of each symmetric local operator (tiled symmetric kernel)
    against the full-matrix GEMVs: the operators are symmetric to rounding,
    so S_hat x agrees to 1e-13, M^-1 r to 1e-12 and the solutions to the PCG
    tolerance; against the oracle as every other path."""
    from oracle.pcg import pcg
    tol = 1e-8 if precision == 0 else 1e-12
    out = {}
    for kern in (1, 2):
        ctx = vb.vb_create(precision=precision, tol=tol, schur_kernel=kern)
        try:
            for wl in wls:
                vb.vb_assemble(ctx, wl)
            vb.vb_setup(ctx)
            assert vb.vb_tuned_tile(ctx, 4) == (1 if kern == 2 else 0)
            assert vb.vb_tuned_tile(ctx, 5) == (1 if kern == 2 else 0)
            n = vb.vb_interface_size(ctx)
            v = torch.tensor(np.random.default_rng(9).standard_normal(n), device=DEV)
            y = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_schur_apply(ctx, v, y)
            z = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_apply(ctx, y, z)
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_pcg_solve(ctx, x)
            its = [vb.vb_problem_solve_info(ctx, k)["iterations"] for k in range(len(wls))]
            xs = [_split(vb, ctx, x.cpu().numpy(), k) for k in range(len(wls))]
            out[kern] = (y.cpu().numpy(), z.cpu().numpy(), xs, its)
        finally:
            vb.vb_destroy(ctx)
    (y1, z1, x1, i1), (y2, z2, x2, i2) = out[1], out[2]
    assert _rel(y2, y1) < 1e-13 if precision == 0 else _rel(y2, y1) < 1e-6
    # M^-1 r on the interface entries (the p0 entries are fixed up to constants)
    nG = len(y1) - sum(len(w["subs"]) for w in wls)
    assert _rel(z2[:nG], z1[:nG]) < (1e-12 if precision == 0 else 1e-5), _rel(z2[:nG], z1[:nG])
    for k, o in enumerate(oracles):
        if precision == 0:
            xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), fixed_iters=i2[k])
        else:
            xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-13)
        assert _rel(x2[k], xo) < 1e-10, (k, _rel(x2[k], xo))
