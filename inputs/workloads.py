"""Seeded synthetic workloads shaped like the paper's CUBE tests (Sec. 7).

Each recipe fixes mesh size n, jitter, degree k, viscosity, subdomain cuts
and the candidate primal functionals; ``make_workload`` returns the plain
data the hot path consumes plus the generator objects (for tests).

  c1  8^3 cube elements, k=2, nu=1, 2x2x2 subdomains, vertex + edge
      averages + face flux
  c2  32^3, plane jitter 0.15h (seed 0), k=2, nu=1, 4x4x4 subdomains,
      vertex + edge + face averages (+ flux, dependent)
  c3  48^3, plane jitter 0.15h (seed 0), k=2, nu=1, 6x6x6 uneven
      subdomains (4..12 elements per side, cuts seed 0)
  c4  32^3 cube elements, k=2, 8 spheres of radius 0.1 with nu=1e4 inside
      (centres uniform, seed 0), 4x4x4 subdomains
  c5  one of 32 problems: 24^3, plane jitter 0.15h, k=3, 3x3x3 subdomains,
      nu constant per subdomain, log-uniform in [1e-3, 1e3] (seed p)
Small parity cases: t8j (8^3 jittered, full constraints), t12 (12^3, 3x3x3),
t12u (12^3, uneven cuts of 2..6 elements), t12b (12^3, 2x2x2: about 3,000
eliminated columns per subdomain), t8k3 (8^3, k=3), t6k4 (6^3, k=4);
adaptive cases: t6f (6^3 jittered, 3x3x3: a floating centre subdomain),
t8f (8^3 jittered, 4x4x4: faces between two floating subdomains),
t12s (12^3, 3x3x3, 4 sinkers of radius 0.25 with nu=1e4).
With the paper's boundary conditions (zero-traction Neumann on the sides
x = 0 and x = 1, no-slip on the other four; no constant-pressure kernel):
t8n (8^3 jittered, 2x2x2), t12n (12^3 jittered, 3x3x3).
The paper's optimality tables (32 subdomains as 4x4x2 boxes, minimal
constraints): deg2, deg3, deg4 (8^3, k = 2, 3, 4: the degree test) and
mesh16, mesh20, mesh24, mesh28, mesh32 (n^3, k = 2: the mesh test).
"""
import numpy as np

from .mesh import CubeMesh
from .assemble import Problem
from .decompose import Decomposition, regular_cuts, random_cuts

MIN = ("vertex", "edge", "flux")
FULL = ("vertex", "edge", "face", "flux")


def sinker_viscosity(mesh, n_sinkers=8, radius=0.1, nu_in=1e4, nu_out=1.0, seed=0):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_sinkers, 3))
    d = np.linalg.norm(mesh.elem_centroid[:, None, :] - centres[None], axis=2)
    return np.where(np.any(d <= radius, axis=1), nu_in, nu_out)


def subdomain_viscosity(mesh, cuts, seed):
    rng = np.random.default_rng(seed)
    parts = [len(c) - 1 for c in cuts]
    nsub = parts[0] * parts[1] * parts[2]
    nu_sub = 10.0 ** rng.uniform(-3.0, 3.0, size=nsub)
    seg = [np.searchsorted(cuts[a], mesh.eidx[:, a], side="right") - 1 for a in range(3)]
    sid = seg[0] + parts[0] * (seg[1] + parts[1] * seg[2])
    return nu_sub[sid]


RECIPES = {
    "c1": dict(n=8, jitter=0.0, k=2, parts=(2, 2, 2), cons=MIN),
    "c2": dict(n=32, jitter=0.15, k=2, parts=(4, 4, 4), cons=FULL),
    "c3": dict(n=48, jitter=0.15, k=2, random_cuts=(4, 12, 6), cons=FULL),
    "c4": dict(n=32, jitter=0.0, k=2, parts=(4, 4, 4), cons=FULL, sinkers=True),
    # C4's sinkers with 12^3-element subdomains: faces of 12 x 12 elements
    # (about 1,500 dual coordinates each), where the dense face eigensolve
    # grows as the cube of the face size
    "c4l": dict(n=36, jitter=0.0, k=2, parts=(3, 3, 3), cons=FULL, sinkers=True),
    "c5": dict(n=24, jitter=0.15, k=3, parts=(3, 3, 3), cons=FULL, nu_per_sub=True),
    "t8j": dict(n=8, jitter=0.15, k=2, parts=(2, 2, 2), cons=FULL),
    "t12": dict(n=12, jitter=0.15, k=2, parts=(3, 3, 3), cons=FULL),
    "t16": dict(n=16, jitter=0.15, k=2, parts=(2, 2, 2), cons=FULL),
    # parity cases for the shapes of the larger configurations: uneven cuts
    # (2..6 elements per side), subdomains of 6^3 elements (about 3,000
    # eliminated columns each: several super-panels of the factorisation),
    # degrees 3 and 4
    "t12u": dict(n=12, jitter=0.15, k=2, random_cuts=(2, 6, 3), cons=FULL),
    "t12b": dict(n=12, jitter=0.15, k=2, parts=(2, 2, 2), cons=FULL),
    "t8k3": dict(n=8, jitter=0.15, k=3, parts=(2, 2, 2), cons=FULL),
    "t6k4": dict(n=6, jitter=0.15, k=4, parts=(2, 2, 2), cons=FULL),
    "t6f": dict(n=6, jitter=0.15, k=2, parts=(3, 3, 3), cons=FULL),
    "t8f": dict(n=8, jitter=0.15, k=2, parts=(4, 4, 4), cons=FULL),
    "t12s": dict(n=12, jitter=0.0, k=2, parts=(3, 3, 3), cons=FULL, sinkers=True,
                 sinker_n=4, sinker_r=0.25),
    "t16s": dict(n=16, jitter=0.0, k=2, parts=(4, 4, 4), cons=FULL, sinkers=True),
    # C5's shape at 12^3 per problem (a family on one jittered mesh, nu per problem)
    "c5s": dict(n=12, jitter=0.15, k=3, parts=(3, 3, 3), cons=FULL, nu_per_sub=True),
    "t8n": dict(n=8, jitter=0.15, k=2, parts=(2, 2, 2), cons=FULL, neumann=(0, 1)),
    "t12n": dict(n=12, jitter=0.15, k=2, parts=(3, 3, 3), cons=FULL, neumann=(0, 1)),
}
for _k in (2, 3, 4):
    RECIPES["deg%d" % _k] = dict(n=8, jitter=0.0, k=_k, parts=(4, 4, 2), cons=MIN)
for _n in (16, 20, 24, 28, 32):
    RECIPES["mesh%d" % _n] = dict(n=_n, jitter=0.0, k=2, parts=(4, 4, 2), cons=MIN)


def make_workload(name, seed=0, workers=None, progress=None, **over):
    """progress: optional callable taking a status string (long generations)."""
    r = dict(RECIPES[name])
    r.update(over)
    mesh = CubeMesh(r["n"], jitter=r["jitter"], seed=seed)
    if "random_cuts" in r:
        lo, hi, parts = r["random_cuts"]
        cuts = random_cuts(r["n"], lo, hi, parts, seed)
    else:
        cuts = regular_cuts(r["n"], r["parts"])
    nu = 1.0
    if r.get("sinkers"):
        nu = sinker_viscosity(mesh, n_sinkers=r.get("sinker_n", 8), radius=r.get("sinker_r", 0.1),
                              seed=seed)
    if r.get("nu_per_sub"):
        nu = subdomain_viscosity(mesh, cuts, seed)
    pb = Problem(mesh, r["k"], nu, workers=workers, progress=progress,
                 neumann_sides=r.get("neumann", ()))
    if progress:
        progress("element matrices done")
    dec = Decomposition(pb, cuts, r["cons"])
    if progress:
        progress("decomposition done")
    wl = dec.workload()
    if progress:
        progress("subdomain matrices done")
    return wl, {"recipe": r, "problem": pb, "decomposition": dec, "name": name}


def make_family(name, seeds, workers=None, mesh_seed=0, **over):
    """Independent problems of recipe `name` sharing one mesh (jitter seed
    `mesh_seed`): the unit-viscosity element matrices are computed once and
    each problem's viscosity (per subdomain, drawn from its own seed) scales
    them.  Returns a list of workloads."""
    from .assemble import with_viscosity
    r = dict(RECIPES[name])
    r.update(over)
    assert r.get("nu_per_sub"), "families vary the per-subdomain viscosity"
    mesh = CubeMesh(r["n"], jitter=r["jitter"], seed=mesh_seed)
    cuts = regular_cuts(r["n"], r["parts"])
    base = Problem(mesh, r["k"], 1.0, workers=workers)
    out = []
    for sd in seeds:
        pb = with_viscosity(base, subdomain_viscosity(mesh, cuts, sd))
        out.append(Decomposition(pb, cuts, r["cons"]).workload())
    return out


def scaled_family(name, seeds, element_data=None, workers=None, mesh_seed=0, base=None, **over):
    """The workloads of make_family(name, seeds) from one decomposition: the
    unit-viscosity problem is decomposed once and each problem's subdomain
    viscosity scales its subdomain's velocity-velocity entries and velocity
    right-hand side (the divergence rows and the pressure right-hand side
    do not depend on nu; the subdomain matrices are sums over the
    subdomain's elements, whose viscosity is the subdomain's).  The same
    workloads as make_family up to rounding.  element_data: optional unit
    element matrices (see Problem).  base: an already decomposed
    (Decomposition, unit workload) pair to reuse.  Yields the workloads one
    by one."""
    r = dict(RECIPES[name])
    r.update(over)
    assert r.get("nu_per_sub"), "families vary the per-subdomain viscosity"
    mesh = CubeMesh(r["n"], jitter=r["jitter"], seed=mesh_seed)
    cuts = regular_cuts(r["n"], r["parts"])
    if base is None:
        pb = Problem(mesh, r["k"], 1.0, workers=workers, element_data=element_data)
        dec = Decomposition(pb, cuts, r["cons"])
        base = (dec, dec.workload())
    dec, wl0 = base
    for sd in seeds:
        nu_el = subdomain_viscosity(mesh, cuts, sd)
        nu_sub = np.zeros(len(wl0["subs"]))
        nu_sub[dec.elem_sub] = nu_el
        subs = []
        for s, sd0 in enumerate(wl0["subs"]):
            kind = np.asarray(sd0["kind"])
            vel = kind != 2
            rows = np.repeat(np.arange(len(kind)), np.diff(sd0["indptr"]))
            vv = vel[rows] & vel[sd0["indices"]]
            data = np.array(sd0["data"], copy=True)
            data[vv] *= nu_sub[s]
            rhs = np.array(sd0["rhs"], copy=True)
            rhs[vel] *= nu_sub[s]
            subs.append(dict(sd0, data=data, rhs=rhs))
        yield {"n_iface": wl0["n_iface"], "subs": subs, "ents": wl0["ents"]}


def save_workload(path, wl):
    """Store a workload as one .npz of plain arrays (no pickles)."""
    arrs = {"n_iface": np.array([wl["n_iface"]]), "nsub": np.array([len(wl["subs"])]),
            "nent": np.array([len(wl["ents"])]),
            "pressure_kernel": np.array([int(wl.get("pressure_kernel", True))])}
    if "has_p0" in wl:
        arrs["has_p0"] = np.asarray(wl["has_p0"], np.int32)
    for i, sd in enumerate(wl["subs"]):
        for k, v in sd.items():
            arrs["s%d_%s" % (i, k)] = v
    for e, E in enumerate(wl["ents"]):
        arrs["e%d_kind" % e] = np.array([E["kind"]])
        arrs["e%d_gids" % e] = E["gids"]
        arrs["e%d_con" % e] = E["con"]
    np.savez(path, **arrs)


def load_workload(path):
    z = np.load(path, allow_pickle=False)
    subs = []
    for i in range(int(z["nsub"][0])):
        subs.append({k: z["s%d_%s" % (i, k)] for k in
                     ("indptr", "indices", "data", "kind", "gid", "pweight", "rhs", "part")
                     if "s%d_%s" % (i, k) in z})
    ents = []
    for e in range(int(z["nent"][0])):
        ents.append({"kind": int(z["e%d_kind" % e][0]), "gids": z["e%d_gids" % e],
                     "con": z["e%d_con" % e]})
    pk = bool(z["pressure_kernel"][0]) if "pressure_kernel" in z else True
    wl = {"n_iface": int(z["n_iface"][0]), "subs": subs, "ents": ents, "pressure_kernel": pk}
    if "has_p0" in z:
        wl["has_p0"] = np.array(z["has_p0"], np.int32)
    return wl


def mlp_init_params(F, H, seed=0):
    """Seeded initial weights of the constraint predictor's network
    (uniform in +-1/sqrt(fan_in), biases zero), float32, in the flat layout
    [W1 (H x F), b1, W2 (H x H), b2, w3 (H), b3]."""
    rng = np.random.default_rng(seed)
    a1, a2 = 1.0 / np.sqrt(F), 1.0 / np.sqrt(H)
    parts = [rng.uniform(-a1, a1, H * F), np.zeros(H), rng.uniform(-a2, a2, H * H), np.zeros(H),
             rng.uniform(-a2, a2, H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)
