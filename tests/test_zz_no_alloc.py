"""vb_batched_ldl_noalloc (working memory in a fixed per-GPU device array)
against vb_batched_ldl (working memory allocated per call), through the
C-ABI: the same kernels on the same inputs, so the factors must agree bit
for bit.  Two calls in a row, the second with a smaller batch and smaller
matrices (the fixed array keeps the first call's contents); a matrix with
inconsistent sizes is left untouched with info = -1; a request beyond the
array's size is refused with VB_ERR_ARG before any kernel runs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
VB_ERR_ARG = -1


@pytest.fixture(scope="module")
def vb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_09770_amd import binding
    binding.load()
    return binding


def _batch(cases, seed, aligned):
    """Saddle matrices [[SPD, B^T], [B, 0]] (column-major device copies)."""
    rng = np.random.default_rng(seed)
    host = []
    for n, e, p in cases:
        Q = rng.standard_normal((n, n))
        A = Q @ Q.T / n + np.eye(n)
        A[p:e, p:e] = 0.0
        ld = (n + 31) // 32 * 32 if aligned else n + 3
        M = np.zeros((n, ld))  # row b of M = column b of the stored matrix
        M[:, :n] = A.T
        host.append((M, n, ld, e, p))
    return host


def _run(vb, fn, host):
    mats = [torch.tensor(M, dtype=torch.float64, device=DEV) for M, *_ in host]
    i32 = lambda v: torch.tensor(v, dtype=torch.int32, device=DEV)
    ptrs = torch.tensor([t.data_ptr() for t in mats], dtype=torch.int64, device=DEV)
    ns, lds, es, ps = ([h[k] for h in host] for k in (1, 2, 3, 4))
    info = i32([7] * len(host))
    ctx = vb.vb_create()
    try:
        fn(ctx, ptrs, i32(ns), i32(lds), i32(es), i32(ps), info, max(ns), max(es))
    finally:
        vb.vb_destroy(ctx)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in mats], info.cpu().numpy()


@pytest.mark.parametrize("aligned", [True, False])
def test_noalloc_matches_allocating_entry_point_twice(vb, aligned):
    first = [(200, 150, 120), (1300, 1100, 1000), (97, 70, 64), (2100, 1800, 1500)]
    second = [(130, 129, 100), (640, 600, 500)]  # smaller batch, smaller matrices
    for k, cases in enumerate((first, second)):
        host = _batch(cases, seed=10 + k, aligned=aligned)
        ref, ref_info = _run(vb, vb.vb_batched_ldl, host)
        got, got_info = _run(vb, vb.vb_batched_ldl_noalloc, host)
        assert ref_info.tolist() == [0] * len(cases)
        assert got_info.tolist() == [0] * len(cases)
        for (M, n, ld, e, p), a, b in zip(host, ref, got):
            # every stored entry, factor and Schur complement (lower
            # triangle) and the untouched rest alike
            assert np.array_equal(a, b), (k, n, e, np.abs(a - b).max())
            L = np.tril(b.T[:e, :e])
            d = np.where(np.arange(e) < p, 1.0, -1.0)
            A = M.T[:n, :n]
            assert np.abs(L @ np.diag(d) @ L.T - A[:e, :e]).max() < 1e-11 * np.abs(A).max()


def test_noalloc_inconsistent_matrix_is_skipped(vb):
    host = _batch([(100, 80, 60), (120, 90, 70)], seed=3, aligned=True)
    M1, n1, ld1, e1, p1 = host[1]
    host[1] = (M1, n1, ld1, n1 + 5, p1)  # e > n
    before = host[1][0].copy()
    got, info = _run(vb, vb.vb_batched_ldl_noalloc, host)
    assert info.tolist() == [0, -1]
    assert np.array_equal(got[1], before)
    ref, ref_info = _run(vb, vb.vb_batched_ldl, host[:1])
    assert np.array_equal(got[0], ref[0])


def test_noalloc_refuses_requests_beyond_its_array(vb):
    # 9 matrices eliminating 8192 columns need 9 * 4 MiB of inverse blocks
    n = 8192
    t = torch.zeros(1, dtype=torch.float64, device=DEV)
    i32 = lambda v: torch.tensor(v, dtype=torch.int32, device=DEV)
    b = 9
    ptrs = torch.tensor([t.data_ptr()] * b, dtype=torch.int64, device=DEV)
    ctx = vb.vb_create()
    try:
        with pytest.raises(vb.VBError) as e:
            vb.vb_batched_ldl_noalloc(ctx, ptrs, i32([n] * b), i32([n] * b), i32([n] * b),
                                      i32([0] * b), i32([0] * b), n, n)
        assert e.value.code == VB_ERR_ARG
        assert "VB_NOALLOC_SCRATCH_BYTES" in str(e.value)
    finally:
        vb.vb_destroy(ctx)
