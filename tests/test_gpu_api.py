"""The entry points' contract on the GPU, through the C-ABI.

* call order: vb_setup before vb_assemble, and vb_pcg_solve / vb_apply
  before vb_setup, return VB_ERR_STATE;
* option checks: an unsupported panel width, precision or scaling, a
  negative or NaN memory limit, a NaN tolerance or a negative adaptive
  threshold make vb_create return VB_ERR_ARG;
* the iteration cap: with maxit = 3 vb_pcg_solve returns
  VB_ERR_NOT_CONVERGED and still writes its iterate, which is the third PCG
  iterate of the oracle (same recurrences, Sec. 7);
* repeated setups of one context give the same solution bit for bit (the
  setup reuses its device buffers from one setup to the next, so nothing of
  the previous setup may leak into the next);
* counting scaling (the pseudo-inverse weights of the paper's
  multiplicity-based averaging) against the oracle with the same scaling;
* mixed precision retries a subdomain whose FP32 Dirichlet factorisation
  breaks down in FP64 (a pivot floor set from the host forces the
  breakdown) and still reaches the oracle's solution;
* bad input data map to error codes (every kernel still runs to its end):
  a local velocity block that is not positive definite makes vb_setup return
  VB_ERR_NOT_SPD naming the subdomain (in mixed precision after its FP64
  retry breaks down too), a primal space without the face
  fluxes makes it return VB_ERR_SINGULAR_COARSE, and a NaN in a right-hand
  side makes vb_pcg_solve return VB_ERR_BREAKDOWN; inconsistent CSR row
  pointers or a
  zero element volume make vb_assemble return VB_ERR_ARG and leave the
  context as it was.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs.workloads import make_workload
from oracle.bddc import OracleBDDC
from oracle.pcg import pcg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
VB_ERR_ARG, VB_ERR_STATE, VB_ERR_NOT_SPD, VB_ERR_BREAKDOWN, VB_ERR_NOT_CONVERGED = -1, -2, -5, -7, -8
VB_ERR_SINGULAR_COARSE = -6


@pytest.fixture(scope="module")
def vb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09770_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def c1():
    wl, _ = make_workload("c1", workers=1)
    return wl


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_call_order(vb, c1):
    ctx = vb.vb_create()
    try:
        with pytest.raises(vb.VBError) as e:
            vb.vb_setup(ctx)
        assert e.value.code == VB_ERR_STATE
        vb.vb_assemble(ctx, c1)
        n = vb.vb_interface_size(ctx)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        with pytest.raises(vb.VBError) as e:
            vb.vb_pcg_solve(ctx, x)
        assert e.value.code == VB_ERR_STATE
        with pytest.raises(vb.VBError) as e:
            vb.vb_apply(ctx, x, torch.zeros_like(x))
        assert e.value.code == VB_ERR_STATE
        vb.vb_setup(ctx)  # the right order still works afterwards
        info = vb.vb_pcg_solve(ctx, x)
        assert info["true_rel_residual"] <= 1e-8 * 1.01
    finally:
        vb.vb_destroy(ctx)


@pytest.mark.parametrize("kw", [dict(panel=48), dict(precision=7), dict(scaling=3),
                                dict(setup_mem_limit=-1.0), dict(local_mem_limit=float("nan")),
                                dict(tol=float("nan")), dict(adaptive_theta=-1.0)])
def test_bad_options(vb, kw):
    with pytest.raises(vb.VBError) as e:
        vb.vb_create(**kw)
    assert e.value.code == VB_ERR_ARG


def test_iteration_cap_writes_the_iterate(vb, c1):
    o = OracleBDDC(c1)
    ctx = vb.vb_create(maxit=3)
    try:
        vb.vb_assemble(ctx, c1)
        vb.vb_setup(ctx)
        n = vb.vb_interface_size(ctx)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = vb.vb_pcg_solve(ctx, x, raise_on_error=False)
        torch.cuda.synchronize()
    finally:
        vb.vb_destroy(ctx)
    assert info["status"] == VB_ERR_NOT_CONVERGED
    assert info["iterations"] == 3
    assert 1e-8 < info["true_rel_residual"] < 1.0
    xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), fixed_iters=3)
    assert _rel(x.cpu().numpy(), xo) < 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_repeated_setup_is_reproducible(vb, c1, precision):
    ctx = vb.vb_create(precision=precision)
    try:
        vb.vb_assemble(ctx, c1)
        n = vb.vb_interface_size(ctx)
        out = []
        for _ in range(3):
            vb.vb_setup(ctx)
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            info = vb.vb_pcg_solve(ctx, x)
            torch.cuda.synchronize()
            out.append((info["iterations"], x.cpu().numpy()))
    finally:
        vb.vb_destroy(ctx)
    for it, x in out[1:]:
        assert it == out[0][0]
        assert np.array_equal(x, out[0][1])


def test_counting_scaling_parity(vb, c1):
    o = OracleBDDC(c1, scaling="counting")
    ctx = vb.vb_create(scaling=vb.VB_SCALING_COUNTING, tol=1e-12)
    try:
        vb.vb_assemble(ctx, c1)
        vb.vb_setup(ctx)
        n = vb.vb_interface_size(ctx)
        r = o.apply_S(np.random.default_rng(5).standard_normal(n))
        z = torch.zeros(n, dtype=torch.float64, device=DEV)
        vb.vb_apply(ctx, torch.tensor(r, device=DEV), z)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = vb.vb_pcg_solve(ctx, x)
        torch.cuda.synchronize()
    finally:
        vb.vb_destroy(ctx)
    zg, zo, nG = z.cpu().numpy(), o.apply_M(r), o.nG
    assert _rel(zg[:nG], zo[:nG]) < 1e-10
    dp = (zg[nG:] - zg[nG:].mean()) - (zo[nG:] - zo[nG:].mean())
    assert np.linalg.norm(dp) < 1e-10 * np.linalg.norm(zo)
    xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-13)
    assert _rel(x.cpu().numpy(), xo) < 1e-10
    assert info["lambda_min"] > 1 - 1e-6


def _copy(wl):
    return {"n_iface": wl["n_iface"], "ents": wl["ents"],
            "subs": [{k: np.array(v, copy=True) for k, v in sd.items()} for sd in wl["subs"]]}


@pytest.mark.parametrize("precision", [0, 1])
def test_non_spd_local_block_is_reported(vb, c1, precision):
    """Also in mixed precision, where the block is first retried in FP64."""
    bad = _copy(c1)
    sd = bad["subs"][3]
    vel = sd["kind"] != 2  # velocity DoFs (interior and interface)
    rows = np.repeat(np.arange(len(sd["kind"])), np.diff(sd["indptr"]))
    vv = vel[rows] & vel[sd["indices"]]
    sd["data"][vv] *= -1.0  # the velocity block negative definite
    ctx = vb.vb_create(precision=precision)
    try:
        vb.vb_assemble(ctx, bad)
        with pytest.raises(vb.VBError) as e:
            vb.vb_setup(ctx)
        assert e.value.code == VB_ERR_NOT_SPD
        assert "block 3 " in str(e.value)
        if precision == 1:
            assert "FP64 retry" in str(e.value)
    finally:
        vb.vb_destroy(ctx)


def _scaled(wl, s, c):
    """The workload with subdomain s's local matrix and right-hand side
    multiplied by c: the same saddle structure (a coefficient jump), every
    pivot of its factorisation multiplied by c."""
    w = _copy(wl)
    w["subs"][s]["data"] = w["subs"][s]["data"] * c
    w["subs"][s]["rhs"] = w["subs"][s]["rhs"] * c
    return w


@pytest.mark.parametrize("nested", [False, True])
def test_fp64_retry_of_fp32_breakdown(vb, c1, nested):
    """Mixed precision, VB_ERR_NOT_SPD's retry clause.  On c1 every pivot of
    a local Dirichlet factorisation lies far above 1e-7: velocity pivots are
    at least lambda_min of the interior velocity block (2.3e-2; eliminating
    pressures first only raises them), pressure pivots lie in the spectrum of
    a pressure Schur complement (smallest nonzero eigenvalue 3e-4).  With
    subdomain 3's local system multiplied by 1e-10 its pivots are at most
    1e-10 times the largest diagonal entry (4.3), so a pivot floor of 1e-7
    makes exactly that block break down in FP32.  vb_setup factors it again
    in FP64, reports it, and the refined solution matches the oracle's on the
    scaled workload as every mixed case does.  A floor above every pivot
    retries every subdomain, with the same solution; no floor, none."""
    cases = [(_scaled(c1, 3, 1e-10), 1e-7, [3]), (c1, 1e300, list(range(8))), (c1, 0.0, [])]
    for wl, floor, expect in cases:
        print("fp64 retry case: floor", floor, "nested", nested, flush=True)
        o = OracleBDDC(wl)
        ctx = vb.vb_create(precision=vb.VB_PREC_MIXED, tol=1e-12, fp32_pivot_min=floor)
        try:
            vb.vb_assemble(ctx, wl, nested=nested)
            vb.vb_setup(ctx)
            assert vb.vb_fp64_retries(ctx) == expect
            n = vb.vb_interface_size(ctx)
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            info = vb.vb_pcg_solve(ctx, x)
            torch.cuda.synchronize()
            assert info["true_rel_residual"] <= 1e-12
            xg = x.cpu().numpy()
            g = o.rhs()
            assert np.linalg.norm(g - o.apply_S(xg)) <= 1e-10 * np.linalg.norm(g)
            xo, _ = pcg(o.apply_S, o.apply_M, g, tol=1e-13)
            assert _rel(xg, xo) < 1e-10, _rel(xg, xo)
        finally:
            vb.vb_destroy(ctx)


def test_bad_sub_box_labels_are_rejected(vb, c1):
    """Sub-box labels whose eliminated DoFs couple across sub-boxes, or a
    pressure on the separator, make vb_assemble return VB_ERR_ARG."""
    coupled = _copy(c1)
    sd = coupled["subs"][0]
    inner = np.nonzero(sd["part"] >= 0)[0]
    sd["part"][inner[0]] = (sd["part"][inner[0]] + 1) % (sd["part"].max() + 1)
    sep_p = _copy(c1)
    sd = sep_p["subs"][1]
    sd["part"][np.nonzero(sd["kind"] == 2)[0][0]] = -1
    for bad, what in ((coupled, "coupled"), (sep_p, ">= 0 for pressures")):
        ctx = vb.vb_create()
        try:
            with pytest.raises(vb.VBError) as e:
                vb.vb_assemble(ctx, bad)
            assert e.value.code == VB_ERR_ARG and what in str(e.value), str(e.value)
        finally:
            vb.vb_destroy(ctx)


def test_primal_space_without_fluxes_gives_singular_coarse(vb, c1):
    """Without the face flux constraints (Assumption 1: the flux of every
    face must be a primal functional) the coarse problem has no flux rows,
    the p0 block of the bordered coarse matrix keeps rank one, and its
    factorisation must stop with VB_ERR_SINGULAR_COARSE."""
    bad = _copy(c1)
    ents = []
    for E in bad["ents"]:
        if E["kind"] == 2:  # faces: c1's only face row is the flux
            E = dict(E, con=np.zeros((0, len(E["gids"]))))
        ents.append(E)
    bad["ents"] = ents
    ctx = vb.vb_create()
    try:
        vb.vb_assemble(ctx, bad)
        with pytest.raises(vb.VBError) as e:
            vb.vb_setup(ctx)
        assert e.value.code == VB_ERR_SINGULAR_COARSE, str(e.value)
        assert "coarse factorisation of problem 0" in str(e.value)
    finally:
        vb.vb_destroy(ctx)


def test_nan_rhs_is_reported(vb, c1):
    bad = _copy(c1)
    bad["subs"][0]["rhs"][0] = np.nan
    ctx = vb.vb_create()
    try:
        vb.vb_assemble(ctx, bad)
        vb.vb_setup(ctx)
        n = vb.vb_interface_size(ctx)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = vb.vb_pcg_solve(ctx, x, raise_on_error=False)
    finally:
        vb.vb_destroy(ctx)
    assert info["status"] == VB_ERR_BREAKDOWN


def test_bad_assembly_data_is_rejected_and_rolled_back(vb, c1):
    bad_ptr = _copy(c1)
    ip = bad_ptr["subs"][1]["indptr"]
    ip[5], ip[6] = ip[6], ip[5]  # row pointers no longer rise
    bad_w = _copy(c1)
    sd = bad_w["subs"][2]
    sd["pweight"][np.nonzero(sd["kind"] == 2)[0][0]] = 0.0
    ctx = vb.vb_create()
    try:
        for bad in (bad_ptr, bad_w):
            with pytest.raises(vb.VBError) as e:
                vb.vb_assemble(ctx, bad)
            assert e.value.code == VB_ERR_ARG
        assert vb.vb_num_problems(ctx) == 0
        vb.vb_assemble(ctx, c1)  # the context is still empty and usable
        vb.vb_setup(ctx)
        x = torch.zeros(vb.vb_interface_size(ctx), dtype=torch.float64, device=DEV)
        info = vb.vb_pcg_solve(ctx, x)
        assert info["true_rel_residual"] <= 1e-8 * 1.01
    finally:
        vb.vb_destroy(ctx)
