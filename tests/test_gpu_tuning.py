"""The dense factorisations' panel width and outer super-panel
(vb_options.panel, vb_options.tune_factor) on the GPU, through the C-ABI.

Every panel width and super-panel the autotuner may choose factors the same
matrices up to rounding, and the triangular sweeps of the refinement and
of the interior recovery follow the panel width the factorisation used.  So
a context left at the defaults (64-wide panels, 16-panel super-panels), one
with 32-wide panels, and one whose factorisations are tuned on its own
first setup give the same S_hat x, M^-1 r, solution and local solutions
within rounding, and the solution is the oracle's.  Cases: t12b single
level (3,560 eliminated columns per subdomain: several outer super-panels
for every candidate) and t12u two-level (fronts, second level and Neumann
matrices: all three classes tuned)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs.workloads import make_workload
from oracle.bddc import OracleBDDC
from oracle.pcg import pcg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CANDIDATES = {(64, 1024), (64, 512), (64, 2048), (32, 512)}


@pytest.fixture(scope="module")
def vb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09770_amd import binding
    binding.load()
    return binding


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


_CASES = {}


def _case(name):
    if name not in _CASES:
        wl, _ = make_workload(name, workers=1)
        o = OracleBDDC(wl)
        xo, _ = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-13)
        _CASES[name] = (wl, xo)
    return _CASES[name]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name,nested", [("t12b", False), ("t12u", True)])
def test_panel_width_and_tuned_factorisation(vb, name, nested, precision):
    print("tuning case", name, "nested" if nested else "single level", "precision", precision,
          flush=True)
    wl, xo = _case(name)
    runs = []
    for kw in (dict(tune_factor=2), dict(tune_factor=2, panel=32), dict(tune_factor=1)):
        ctx = vb.vb_create(precision=precision, tol=1e-12, **kw)
        try:
            vb.vb_assemble(ctx, wl, nested=nested)
            vb.vb_setup(ctx)
            nb = [vb.vb_tuned_tile(ctx, w) for w in (6, 7, 8)]
            sb = [vb.vb_tuned_tile(ctx, w) for w in (9, 10, 11)]
            levels = (0, 1, 2) if nested else (0, 2)
            for c in levels:
                if kw["tune_factor"] == 2:
                    p = kw.get("panel", 64)
                    assert (nb[c], sb[c]) == (p, 16 * p), (nb, sb)
                else:
                    assert (nb[c], sb[c]) in CANDIDATES, (nb, sb)
            if not nested:
                assert nb[1] == 0 and sb[1] == 0
            n = vb.vb_interface_size(ctx)
            v = torch.tensor(np.random.default_rng(3).standard_normal(n), device=DEV)
            y = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_schur_apply(ctx, v, y)
            z = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_apply(ctx, y, z)
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            vb.vb_pcg_solve(ctx, x)
            u = torch.zeros(vb.vb_local_size(ctx), dtype=torch.float64, device=DEV)
            vb.vb_recover_all(ctx, x, u)
            torch.cuda.synchronize()
            runs.append((y.cpu().numpy(), z.cpu().numpy(), x.cpu().numpy(), u.cpu().numpy()))
        finally:
            vb.vb_destroy(ctx)
    nG = len(runs[0][0]) - len(wl["subs"])
    y0, z0, x0, u0 = runs[0]
    for y, z, x, u in runs[1:]:
        if precision == 0:
            assert _rel(y, y0) < 1e-12 and _rel(z[:nG], z0[:nG]) < 1e-11
        else:  # FP32 operators: the blockings round differently
            assert _rel(y, y0) < 1e-5 and _rel(z[:nG], z0[:nG]) < 1e-4
        assert _rel(x, x0) < 1e-10 and _rel(u, u0) < 1e-9
    for y, z, x, u in runs:
        assert _rel(x, xo) < 1e-10, _rel(x, xo)
