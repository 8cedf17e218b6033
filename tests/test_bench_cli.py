"""bench.py on the CPU: more than one GPU is refused with a message (this
build has no multi-GPU path), before any GPU work; the setup flop counts it
reports match brute force and the textbook dense LU count."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_dense_condensation_flops_match_brute_force():
    import numpy as np
    b = _bench()
    subs = []
    for nv, npr, ng in [(7, 3, 5), (20, 4, 0), (1, 2, 9)]:
        subs.append({"kind": np.array([0] * nv + [2] * npr + [1] * ng)})
    want = 0
    for nv, npr, ng in [(7, 3, 5), (20, 4, 0), (1, 2, 9)]:
        e, m = nv + npr - 1, nv + npr - 1 + ng
        for j in range(e):  # rank-1 update of the trailing lower triangle
            want += sum(2 for r in range(j + 1, m) for c in range(j + 1, r + 1))  # multiply-add
            want += m - j - 1  # the column below the pivot scaled by it
    assert b.dense_condensation_flops({"subs": subs}) == float(want)


def test_sparse_lu_flops_of_a_dense_matrix_is_the_textbook_count():
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.linalg import splu
    b = _bench()
    n = 40
    A = np.random.default_rng(0).standard_normal((n, n)) + n * np.eye(n)
    lu = splu(sp.csc_matrix(A), permc_spec="NATURAL")
    want = sum(2 * k * k + k for k in range(n))  # 2n^3/3 + O(n^2)
    assert b.sparse_lu_flops(lu) == float(want)


def test_setup_flops_report_on_a_small_workload():
    from inputs.workloads import make_workload
    from oracle.bddc import LocalSchur
    b = _bench()
    wl, _ = make_workload("c1", workers=1)
    lu = LocalSchur(wl["subs"][0], condense=False).lu
    rep = b.setup_flops(wl, [b.sparse_lu_flops(lu)], 10.0)
    assert 0 < rep["sparse_factor_est"] < rep["dense_single_level"]
    assert rep["dense_tflops_per_setup_s"] == rep["dense_single_level"] / 1e-2 / 1e12
    # the two-level factorisation: fronts of the 2x2x2 sub-boxes, then the
    # separators, fewer operations than one dense factorisation
    assert 0 < rep["nested_executed"] < rep["dense_single_level"]
    assert rep["nested_tflops_per_setup_s"] == rep["nested_executed"] / 1e-2 / 1e12


def test_nested_flops_match_brute_force():
    """One subdomain of 8 DoFs: sub-box 0 = {0, 1 (pressure)}, sub-box 1 =
    {2, 3 (pressure)}, separator {4}, interface {5, 6}; row couplings give
    B_0 = {4, 5}, B_1 = {4, 6}."""
    import numpy as np
    import scipy.sparse as sp
    b = _bench()
    kind = np.array([0, 2, 0, 2, 0, 1, 1, 2])
    part = np.array([0, 0, 1, 1, -1, -1, -1, 0])
    edges = [(0, 1), (0, 4), (1, 5), (2, 3), (2, 4), (3, 6), (0, 7), (4, 5), (5, 6)]
    A = sp.lil_matrix((8, 8))
    for i, j in edges:
        A[i, j] = A[j, i] = 1.0
    for i in range(8):
        A[i, i] = 1.0
    A = A.tocsr()
    wl = {"subs": [{"kind": kind, "part": part, "indptr": A.indptr, "indices": A.indices}]}
    brute = lambda m, e: sum(t * t - 1 for t in range(m - e + 1, m + 1))
    # sub-box 0: rows {0, 1, 7}, e = 2, B = {4, 5}; sub-box 1: rows {2, 3},
    # e = 1, B = {4, 6}; second level: separator {4} + 2 sub-box constants,
    # e = 2, onto 2 interface DoFs
    want = brute(2 + 1 + 2, 2) + brute(1 + 1 + 2, 1) + brute(2 + 2, 2)
    assert b.nested_condensation_flops(wl) == float(want)


def test_cpu_baseline_sample_and_full_oracle_on_c1():
    from inputs.workloads import make_workload
    b = _bench()
    wl, _ = make_workload("c1", workers=1)
    rep = b.cpu_baseline(wl, budget_s=0.0)  # the bound still takes one subdomain
    assert rep["kind"] == "oracle" and rep["value"] > 0 and rep["cores"] >= 1
    assert "1 of 8 subdomains" in rep["sample"]
    full = b.oracle_full_c1()
    assert full["iterations"] > 0 and full["solves_per_s"] > 0
    assert full["setup_s"] > 0 and full["pcg_s"] > 0 and full["recovery_s"] > 0
