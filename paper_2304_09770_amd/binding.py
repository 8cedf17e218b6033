"""ctypes binding of libvembddc (include/vembddc.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Device vectors
are torch CUDA tensors (float64) or raw device addresses; the library does
all the arithmetic.  The binding refuses to run without the built library
(there is no CPU fallback).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvembddc.so")

VB_OK = 0
ERRORS = {-1: "VB_ERR_ARG", -2: "VB_ERR_STATE", -3: "VB_ERR_OOM", -4: "VB_ERR_DEVICE",
          -5: "VB_ERR_NOT_SPD", -6: "VB_ERR_SINGULAR_COARSE", -7: "VB_ERR_BREAKDOWN",
          -8: "VB_ERR_NOT_CONVERGED"}
VB_PREC_FP64, VB_PREC_MIXED = 0, 1
VB_SCALING_DELUXE, VB_SCALING_COUNTING = 0, 1
VB_PCG_AUTO, VB_PCG_GRAPH, VB_PCG_PERSISTENT = 0, 1, 2


class vb_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("scaling", C.c_int), ("tol", C.c_double),
                ("maxit", C.c_int), ("svd_tol", C.c_double), ("panel", C.c_int),
                ("stream", C.c_void_p), ("profile", C.c_int), ("adaptive_theta", C.c_double),
                ("predictor", C.c_void_p),
                ("setup_mem_limit", C.c_double), ("local_mem_limit", C.c_double),
                ("pcg_launch", C.c_int), ("schur_kernel", C.c_int),
                ("fp32_pivot_min", C.c_double), ("tune_factor", C.c_int),
                ("inner_tol", C.c_double)]


class vb_problem(C.Structure):
    _fields_ = [("iface_offset", C.c_int64), ("n_iface", C.c_int64), ("p0_offset", C.c_int64),
                ("sub_offset", C.c_int), ("n_sub", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vb_face_info(C.Structure):
    _fields_ = [("entity", C.c_int), ("sub_i", C.c_int), ("sub_j", C.c_int),
                ("n_dual", C.c_int), ("n_selected", C.c_int), ("predicted", C.c_int),
                ("path", C.c_int), ("passes", C.c_int), ("sum_shift", C.c_double)]


class vb_kernel_stat(C.Structure):
    _fields_ = [("launches", C.c_int), ("total_ms", C.c_double), ("work", C.c_double)]


class vb_subdomain(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("indptr", C.POINTER(C.c_int64)),
                ("indices", C.POINTER(C.c_int64)), ("data", C.POINTER(C.c_double)),
                ("kind", C.POINTER(C.c_int32)), ("gid", C.POINTER(C.c_int64)),
                ("pweight", C.POINTER(C.c_double)), ("rhs", C.POINTER(C.c_double)),
                ("part", C.POINTER(C.c_int32))]


class vb_entity(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("gids", C.POINTER(C.c_int64)),
                ("n_con", C.c_int32), ("con", C.POINTER(C.c_double))]


class vb_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("rel_residual", C.c_double),
                ("true_rel_residual", C.c_double), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("n_coarse", C.c_int), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("status", C.c_int), ("refinement_steps", C.c_int),
                ("latency_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load the built library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libvembddc.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "vb_create": (C.c_int, [C.POINTER(P), C.POINTER(vb_options)]),
        "vb_destroy": (None, [P]),
        "vb_last_error": (C.c_char_p, [P]),
        "vb_assemble": (C.c_int, [P, C.c_int64, C.c_int, C.POINTER(vb_subdomain), C.c_int,
                                  C.POINTER(vb_entity)]),
        "vb_setup": (C.c_int, [P]),
        "vb_interface_size": (C.c_int64, [P]),
        "vb_rhs": (C.c_int, [P, P]),
        "vb_schur_apply": (C.c_int, [P, P, P]),
        "vb_apply": (C.c_int, [P, P, P]),
        "vb_pcg_solve": (C.c_int, [P, P, C.POINTER(vb_solve_info)]),
        "vb_get_local_solution": (C.c_int, [P, P, C.c_int, C.POINTER(C.c_double)]),
        "vb_recover_all": (C.c_int, [P, P, P]),
        "vb_local_size": (C.c_int64, [P, C.c_int]),
        "vb_set_profile": (C.c_int, [P, C.c_int]),
        "vb_pcg_launch_used": (C.c_int, [P]),
        "vb_fp64_retries": (C.c_int, [P, C.c_int, C.POINTER(C.c_int32)]),
        "vb_refinement_history": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(C.c_double),
                                            C.POINTER(C.c_int32)]),
        "vb_vem_element_matrices": (C.c_int, [P, C.c_int, C.c_int64, P, P, C.c_int, P, P, P]),
        "vb_vem_dofs": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "vb_setup_phases": (C.c_int, [P, C.c_int, C.POINTER(C.c_double)]),
        "vb_batched_ldl": (C.c_int, [P, C.c_int, P, P, P, P, P, P, C.c_int, C.c_int]),
        "vb_batched_ldl_noalloc": (C.c_int, [P, C.c_int, P, P, P, P, P, P, C.c_int, C.c_int]),
        "vb_kernel_stats": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(vb_kernel_stat)]),
        "vb_adaptive_info": (C.c_int, [P, C.c_int, C.POINTER(vb_face_info), C.c_int,
                                       C.POINTER(C.c_double)]),
        "vb_num_problems": (C.c_int, [P]),
        "vb_tuned_tile": (C.c_int, [P, C.c_int]),
        "vb_problem_layout": (C.c_int, [P, C.c_int, C.POINTER(vb_problem)]),
        "vb_problem_solve_info": (C.c_int, [P, C.c_int, C.POINTER(vb_solve_info)]),
        "vb_face_samples": (C.c_int64, [P, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
        "vb_mlp_add_data": (C.c_int, [P, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int64]),
        "vb_mlp_create": (C.c_int, [C.POINTER(P), C.POINTER(C.c_float), P]),
        "vb_mlp_destroy": (None, [P]),
        "vb_mlp_last_error": (C.c_char_p, [P]),
        "vb_mlp_add_samples": (C.c_int, [P, P]),
        "vb_mlp_num_samples": (C.c_int64, [P]),
        "vb_mlp_train": (C.c_int, [P, C.c_int, C.c_float, C.POINTER(C.c_double)]),
        "vb_mlp_forward": (C.c_int, [P, P, C.c_int64, P]),
        "vb_mlp_loss_grad": (C.c_int, [P, P, P, C.c_int64, P, C.POINTER(C.c_double)]),
        "vb_mlp_get_params": (C.c_int, [P, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                        C.POINTER(C.c_float)]),
        "vb_mlp_set_params": (C.c_int, [P, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                        C.POINTER(C.c_float)]),
        "vb_mlp_set_warm_start": (C.c_int, [P, C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["vb_create", "vb_destroy", "vb_last_error", "vb_assemble", "vb_setup",
            "vb_interface_size", "vb_rhs", "vb_schur_apply", "vb_apply", "vb_pcg_solve",
            "vb_get_local_solution", "vb_recover_all", "vb_batched_ldl", "vb_kernel_stats",
            "vb_adaptive_info", "vb_face_samples", "vb_mlp_create", "vb_mlp_destroy",
            "vb_mlp_last_error", "vb_mlp_add_samples", "vb_mlp_num_samples", "vb_mlp_train",
            "vb_mlp_forward", "vb_mlp_loss_grad", "vb_mlp_get_params", "vb_mlp_set_params",
            "vb_mlp_set_warm_start", "vb_mlp_add_data", "vb_num_problems", "vb_problem_layout",
            "vb_problem_solve_info", "vb_tuned_tile", "vb_local_size", "vb_set_profile",
            "vb_batched_ldl_noalloc", "vb_pcg_launch_used", "vb_fp64_retries",
            "vb_vem_element_matrices", "vb_vem_dofs", "vb_setup_phases", "vb_refinement_history"]


class VBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


def _ptr(t, dtype=None, n=None):
    """Device address of a torch tensor, or an int taken as a raw device
    address.  A tensor must be on the GPU and contiguous; its element type
    (`dtype`, e.g. "float64") and minimum length `n` are checked when given,
    so that a host tensor, a wrong element type or a short vector is refused
    here instead of reaching the kernels."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not getattr(t, "is_cuda", False):
        raise ValueError("expected a GPU tensor, got %s" % getattr(t, "device", type(t).__name__))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise TypeError("expected a %s tensor, got %s" % (dtype, t.dtype))
    if n is not None and t.numel() < n:
        raise ValueError("expected at least %d elements, got %d" % (n, t.numel()))
    return t.data_ptr()


def _vec(ctx, t):
    """An interface vector of the context: float64, vb_interface_size long."""
    return _ptr(t, "float64", vb_interface_size(ctx))


def _np(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a, a.ctypes.data_as(C.POINTER(np.ctypeslib.as_ctypes_type(dt)))


def _check(ctx, rc):
    if rc != VB_OK:
        raise VBError(rc, load().vb_last_error(ctx).decode())


# ------------------------------------------------------------- C-ABI names
def vb_create(precision=VB_PREC_FP64, scaling=VB_SCALING_DELUXE, tol=1e-8, maxit=1000,
              svd_tol=1e-10, panel=0, stream=None, profile=0, adaptive_theta=0.0,
              predictor=None, setup_mem_limit=0.0, local_mem_limit=0.0, pcg_launch=0,
              schur_kernel=0, fp32_pivot_min=0.0, tune_factor=0, inner_tol=0.0):
    lib = load()
    opt = vb_options(precision, scaling, tol, maxit, svd_tol, panel, stream, profile,
                     adaptive_theta, predictor, setup_mem_limit, local_mem_limit, pcg_launch,
                     schur_kernel, fp32_pivot_min, tune_factor, inner_tol)
    ctx = C.c_void_p()
    rc = lib.vb_create(C.byref(ctx), C.byref(opt))
    if rc != VB_OK:
        raise VBError(rc, "vb_create")
    return ctx


def vb_destroy(ctx):
    load().vb_destroy(ctx)


def vb_assemble(ctx, workload, nested=True):
    """workload: dict(n_iface, subs=[dict(indptr, indices, data, kind, gid,
    pweight, rhs[, part])], ents=[dict(kind, gids, con)]) (numpy arrays).
    nested: pass the sub-box labels `part` when the workload has them (the
    two-level local factorisation); False: one dense factorisation per
    subdomain.  A workload with Neumann sides (pressure_kernel false) is
    refused: the library condenses each subdomain's constant pressure as
    coupled only through its interface fluxes, and borders the coarse
    problem against the constant-pressure kernel of no-slip boundaries."""
    if not workload.get("pressure_kernel", True):
        raise NotImplementedError("vb_assemble: workloads with Neumann sides are not supported")
    keep = []
    subs = (vb_subdomain * len(workload["subs"]))()
    for i, sd in enumerate(workload["subs"]):
        ip, ipp = _np(sd["indptr"], np.int64)
        ix, ixp = _np(sd["indices"], np.int64)
        dv, dvp = _np(sd["data"], np.float64)
        kd, kdp = _np(sd["kind"], np.int32)
        gd, gdp = _np(sd["gid"], np.int64)
        pw, pwp = _np(sd["pweight"], np.float64)
        rh, rhp = _np(sd["rhs"], np.float64)
        keep += [ip, ix, dv, kd, gd, pw, rh]
        ptp = None
        if nested and sd.get("part") is not None:
            pt, ptp = _np(sd["part"], np.int32)
            keep.append(pt)
        subs[i] = vb_subdomain(len(kd), len(ix), ipp, ixp, dvp, kdp, gdp, pwp, rhp, ptp)
    ents = (vb_entity * max(1, len(workload["ents"])))()
    for e, E in enumerate(workload["ents"]):
        g, gp = _np(E["gids"], np.int64)
        con = np.ascontiguousarray(E["con"], dtype=np.float64).reshape(-1, len(g))
        c, cp = _np(con.ravel(), np.float64)
        keep += [g, c]
        ents[e] = vb_entity(int(E["kind"]), len(g), gp, con.shape[0], cp)
    rc = load().vb_assemble(ctx, int(workload["n_iface"]), len(workload["subs"]), subs,
                            len(workload["ents"]), ents)
    _check(ctx, rc)


def vb_setup(ctx):
    _check(ctx, load().vb_setup(ctx))


def vb_interface_size(ctx):
    return int(load().vb_interface_size(ctx))


def vb_rhs(ctx, g):
    _check(ctx, load().vb_rhs(ctx, _vec(ctx, g)))


def vb_schur_apply(ctx, x, y):
    _check(ctx, load().vb_schur_apply(ctx, _vec(ctx, x), _vec(ctx, y)))


def vb_apply(ctx, r, z):
    _check(ctx, load().vb_apply(ctx, _vec(ctx, r), _vec(ctx, z)))


def vb_pcg_solve(ctx, x, raise_on_error=True):
    info = vb_solve_info()
    rc = load().vb_pcg_solve(ctx, _vec(ctx, x), C.byref(info))
    if raise_on_error:
        _check(ctx, rc)
    return info.as_dict()


def vb_local_size(ctx, sub=-1):
    """Local DoFs of subdomain `sub`, or (sub = -1) of all subdomains."""
    n = int(load().vb_local_size(ctx, int(sub)))
    _check(ctx, n if n < 0 else 0)
    return n


def vb_get_local_solution(ctx, x, sub, n=None):
    """Subdomain `sub`'s local DoF vector (host).  The buffer is sized by the
    library (vb_local_size); `n`, if given, must equal that size."""
    m = vb_local_size(ctx, sub)
    if n is not None and int(n) != m:
        raise ValueError("subdomain %d has %d local DoFs, not %d" % (sub, m, n))
    out = np.zeros(m)
    rc = load().vb_get_local_solution(ctx, _vec(ctx, x), int(sub),
                                      out.ctypes.data_as(C.POINTER(C.c_double)))
    _check(ctx, rc)
    return out


def vb_recover_all(ctx, x, out):
    """out: None, or a float64 device tensor of at least vb_local_size(ctx)
    elements."""
    n = vb_local_size(ctx) if out is not None else None
    _check(ctx, load().vb_recover_all(ctx, _vec(ctx, x), _ptr(out, "float64", n)))


def vb_batched_ldl(ctx, ptrs, n, ld, e, p, info, max_n, max_e):
    b = len(n)
    rc = load().vb_batched_ldl(ctx, b, _ptr(ptrs, "int64", b), _ptr(n, "int32", b),
                               _ptr(ld, "int32", b), _ptr(e, "int32", b), _ptr(p, "int32", b),
                               _ptr(info, "int32", b), int(max_n), int(max_e))
    _check(ctx, rc)


def vb_batched_ldl_noalloc(ctx, ptrs, n, ld, e, p, info, max_n, max_e):
    b = len(n)
    rc = load().vb_batched_ldl_noalloc(ctx, b, _ptr(ptrs, "int64", b), _ptr(n, "int32", b),
                                       _ptr(ld, "int32", b), _ptr(e, "int32", b),
                                       _ptr(p, "int32", b), _ptr(info, "int32", b), int(max_n),
                                       int(max_e))
    _check(ctx, rc)


VB_NOALLOC_SCRATCH_BYTES = 32 << 20


def vb_kernel_stats(ctx, which, reset=False):
    st = vb_kernel_stat()
    _check(ctx, load().vb_kernel_stats(ctx, int(which), int(bool(reset)), C.byref(st)))
    return {"launches": st.launches, "total_ms": st.total_ms, "work": st.work}


def vb_pcg_launch_used(ctx):
    return int(load().vb_pcg_launch_used(ctx))


SETUP_PHASES = ("local Dirichlet", "primal constraints", "change of basis", "right-hand side",
                "local Neumann", "coarse", "scaling", "iteration structures", "recovery structures")


def vb_setup_phases(ctx):
    """{phase name: ms} of the last vb_setup."""
    buf = (C.c_double * len(SETUP_PHASES))()
    n = load().vb_setup_phases(ctx, len(SETUP_PHASES), buf)
    if n < 0:
        raise VBError(n, "vb_setup_phases")
    return {SETUP_PHASES[i]: float(buf[i]) for i in range(min(n, len(SETUP_PHASES)))}


def vb_vem_dofs(k):
    n, p = C.c_int(), C.c_int()
    rc = load().vb_vem_dofs(int(k), C.byref(n), C.byref(p))
    if rc != VB_OK:
        raise VBError(rc, "vb_vem_dofs")
    return n.value, p.value


def vb_vem_element_matrices(ctx, k, X8, nu, A, B, F=None):
    """X8: (E, 8, 3) or (E, 24) float64 device tensor; nu: (E,) or None;
    A: (E, N, N), B: (E, nP, N), F: (E, N) or None, float64 device tensors."""
    N, nP = vb_vem_dofs(k)
    E = X8.shape[0]
    if X8.numel() != 24 * E or A.numel() < E * N * N or B.numel() < E * nP * N:
        raise ValueError("vb_vem_element_matrices: array sizes")
    if nu is not None and nu.numel() < E:
        raise ValueError("vb_vem_element_matrices: nu")
    if F is not None and F.numel() < E * N:
        raise ValueError("vb_vem_element_matrices: F")
    _check(ctx, load().vb_vem_element_matrices(
        ctx, int(k), int(E), _ptr(X8, "float64"), _ptr(nu, "float64") if nu is not None else None,
        1 if F is not None else 0, _ptr(A, "float64"), _ptr(B, "float64"),
        _ptr(F, "float64") if F is not None else None))


def vb_fp64_retries(ctx):
    """Subdomains whose Dirichlet factorisation the last vb_setup redid in FP64."""
    lib = load()
    n = lib.vb_fp64_retries(ctx, 0, None)
    if n < 0:
        raise VBError(n, "vb_fp64_retries")
    buf = (C.c_int32 * max(n, 1))()
    n = lib.vb_fp64_retries(ctx, n, buf)
    return [int(buf[i]) for i in range(n)]


def vb_refinement_history(ctx, problem=0):
    """(rel, inner) of the last mixed-precision solve of one problem: the
    relative condensed residual before each refinement step and after the
    last, and the inner PCG iterations of each step."""
    lib = load()
    n = lib.vb_refinement_history(ctx, problem, 0, None, None)
    if n < 0:
        raise VBError(n, "vb_refinement_history")
    if n == 0:
        return [], []
    rel = (C.c_double * (n + 1))()
    inner = (C.c_int32 * max(n, 1))()
    n = lib.vb_refinement_history(ctx, problem, n + 1, rel, inner)
    return [float(rel[i]) for i in range(n + 1)], [int(inner[i]) for i in range(n)]


def vb_set_profile(ctx, on):
    _check(ctx, load().vb_set_profile(ctx, int(bool(on))))


def vb_adaptive_info(ctx):
    """List of per-face dicts (entity, sub_i, sub_j, n_dual, n_selected,
    eigenvalues) of the adaptive coarse space of the last setup."""
    lib = load()
    nf = lib.vb_adaptive_info(ctx, 0, None, 0, None)
    if nf < 0:
        _check(ctx, nf)
    faces = (vb_face_info * max(nf, 1))()
    rc = lib.vb_adaptive_info(ctx, nf, faces, 0, None)
    if rc < 0:
        _check(ctx, rc)
    ne = sum(faces[i].n_selected for i in range(nf) if faces[i].n_selected < faces[i].n_dual)
    eigs = np.zeros(max(ne, 1))
    rc = lib.vb_adaptive_info(ctx, nf, faces, ne, eigs.ctypes.data_as(C.POINTER(C.c_double)))
    if rc < 0:
        _check(ctx, rc)
    out, o = [], 0
    for i in range(nf):
        f = faces[i]
        k = f.n_selected if f.n_selected < f.n_dual else 0
        out.append({"entity": f.entity, "subs": (f.sub_i, f.sub_j), "n_dual": f.n_dual,
                    "n_selected": f.n_selected, "predicted": f.predicted, "path": f.path,
                    "passes": f.passes, "sum_shift": f.sum_shift,
                    "eigenvalues": eigs[o: o + k].copy()})
        o += k
    return out


# ---------------------------------------------------------- learned predictor
VB_MLP_FEATURES, VB_MLP_NPARAMS = 12, 1505


def _mcheck(m, rc):
    if rc < 0:
        raise VBError(rc, load().vb_mlp_last_error(m).decode())


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def vb_face_samples(ctx):
    """(X, y) host arrays of the last adaptive setup's face coordinates
    (labels NaN where the face was not solved by the exact eigensolve)."""
    lib = load()
    n = lib.vb_face_samples(ctx, 0, None, None)
    _check(ctx, n if n < 0 else 0)
    X = np.zeros((n, VB_MLP_FEATURES), np.float32)
    y = np.zeros(n, np.float32)
    rc = lib.vb_face_samples(ctx, n, _fptr(X), _fptr(y))
    _check(ctx, rc if rc < 0 else 0)
    return X, y


def vb_mlp_add_data(m, X, y):
    X = np.ascontiguousarray(X, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    _mcheck(m, load().vb_mlp_add_data(m, _fptr(X), _fptr(y), len(y)))


def vb_mlp_create(init, stream=None):
    init = np.ascontiguousarray(init, dtype=np.float32)
    assert init.size == VB_MLP_NPARAMS
    m = C.c_void_p()
    rc = load().vb_mlp_create(C.byref(m), _fptr(init), stream)
    if rc != VB_OK:
        raise VBError(rc, "vb_mlp_create")
    return m


def vb_mlp_destroy(m):
    load().vb_mlp_destroy(m)


def vb_mlp_add_samples(m, ctx):
    rc = load().vb_mlp_add_samples(m, ctx)
    _mcheck(m, rc)
    return rc


def vb_mlp_num_samples(m):
    return int(load().vb_mlp_num_samples(m))


def vb_mlp_train(m, epochs, lr):
    hist = np.zeros(max(epochs, 1))
    rc = load().vb_mlp_train(m, int(epochs), float(lr), hist.ctypes.data_as(C.POINTER(C.c_double)))
    _mcheck(m, rc)
    return hist[:epochs]


def vb_mlp_forward(m, X, s):
    N = int(X.shape[0])
    _mcheck(m, load().vb_mlp_forward(m, _ptr(X, "float32", N * VB_MLP_FEATURES), N,
                                     _ptr(s, "float32", N)))


def vb_mlp_loss_grad(m, X, y, g):
    loss = C.c_double()
    N = int(X.shape[0])
    _mcheck(m, load().vb_mlp_loss_grad(m, _ptr(X, "float32", N * VB_MLP_FEATURES),
                                       _ptr(y, "float32", N), N,
                                       _ptr(g, "float32", VB_MLP_NPARAMS), C.byref(loss)))
    return loss.value


def vb_mlp_get_params(m):
    p = np.zeros(VB_MLP_NPARAMS, np.float32)
    mu = np.zeros(VB_MLP_FEATURES, np.float32)
    sd = np.zeros(VB_MLP_FEATURES, np.float32)
    _mcheck(m, load().vb_mlp_get_params(m, _fptr(p), _fptr(mu), _fptr(sd)))
    return p, mu, sd


def vb_mlp_set_params(m, p, mu, sd):
    p = np.ascontiguousarray(p, np.float32)
    mu = np.ascontiguousarray(mu, np.float32)
    sd = np.ascontiguousarray(sd, np.float32)
    _mcheck(m, load().vb_mlp_set_params(m, _fptr(p), _fptr(mu), _fptr(sd)))


def vb_mlp_set_warm_start(m, on):
    _mcheck(m, load().vb_mlp_set_warm_start(m, int(bool(on))))


# ------------------------------------------------------------ several problems
def vb_num_problems(ctx):
    return int(load().vb_num_problems(ctx))


def vb_problem_layout(ctx, problem):
    out = vb_problem()
    _check(ctx, load().vb_problem_layout(ctx, int(problem), C.byref(out)))
    return out.as_dict()


def vb_problem_solve_info(ctx, problem):
    out = vb_solve_info()
    _check(ctx, load().vb_problem_solve_info(ctx, int(problem), C.byref(out)))
    return out.as_dict()


def vb_tuned_tile(ctx, which):
    return int(load().vb_tuned_tile(ctx, int(which)))
