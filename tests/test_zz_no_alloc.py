"""The entry point that allocates nothing (ccm_matvec_t_noalloc), called
through the C ABI, equals ccm_matvec_t with a caller scratch buffer bit for
bit on two calls in a row, the second on a smaller matrix (the library's
buffer keeps the first call's partial sums and must not leak them)."""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "gpu tests need a GPU"


def _call_noalloc(c, m, x, y):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = c.lib.ccm_matvec_t_noalloc(ctypes.byref(m.desc), ctypes.c_void_p(x.data_ptr()),
                                    c._lib.I32 if x.dtype == torch.int32 else c._lib.I64,
                                    ctypes.c_void_p(y.data_ptr()), s)
    return rc


def _call_with_scratch(c, m, x, y):
    nb = int(c.lib.ccm_matvec_t_scratch_bytes(ctypes.byref(m.desc)))
    scratch = torch.empty(max(nb, 8) // 8, dtype=torch.int64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = c.lib.ccm_matvec_t(ctypes.byref(m.desc), ctypes.c_void_p(x.data_ptr()),
                            c._lib.I32 if x.dtype == torch.int32 else c._lib.I64,
                            ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(scratch.data_ptr()),
                            nb, s)
    torch.cuda.synchronize()
    return rc


@pytest.mark.parametrize("b,signed", [(1, False), (5, True), (12, False), (31, True)])
def test_noalloc_matches_scratch_path_twice(b, signed):
    import paper_1303_0270_amd as c
    rng = np.random.default_rng(100 + b)
    for rows, cols in ((4000, 3000), (700, 130)):  # the second call is smaller
        lo, hi = ((-(1 << (b - 1)), 1 << (b - 1)) if signed else (0, 1 << b))
        A = rng.integers(lo, hi, size=(rows, cols), dtype=np.int64)
        m = c.compress(torch.from_numpy(A).cuda())
        x = torch.from_numpy(rng.integers(-(1 << 15), 1 << 15, size=rows)).to(torch.int32).cuda()
        y_ref = torch.full((cols,), -1, dtype=torch.int64, device="cuda")
        y = torch.full((cols,), -2, dtype=torch.int64, device="cuda")
        assert _call_with_scratch(c, m, x, y_ref) == 0
        assert _call_noalloc(c, m, x, y) == 0
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), (rows, cols)
        # and both equal the oracle
        want = oracle.matvec_t(oracle.compress(A), x.cpu().numpy())
        assert np.array_equal(y.cpu().numpy(), want)


def test_noalloc_rejects_too_many_columns():
    import paper_1303_0270_amd as c
    m = c.compress(torch.zeros((2, 65537), dtype=torch.int64, device="cuda"))
    x = torch.zeros(2, dtype=torch.int32, device="cuda")
    y = torch.zeros(65537, dtype=torch.int64, device="cuda")
    assert _call_noalloc(c, m, x, y) == c._lib.E_NOMEM
