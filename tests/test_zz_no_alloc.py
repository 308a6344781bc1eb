"""jz_knn_noalloc (through the C ABI): the kNN entry point that takes its
scratch from the library's fixed device array instead of allocating. Its
output must equal jz_knn's bit for bit on the same tree, on two calls in a
row (the second on a smaller input, so it reuses the array the first one
left behind), and a call too large for the array is refused with
JZ_E_CAPACITY."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2604_05885_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def jz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_05885_amd import api
    return api


def noalloc_knn(jz, t, k):
    idx = torch.empty((t.n, k), dtype=torch.int32, device="cuda")
    d2 = torch.empty((t.n, k), dtype=torch.float32, device="cuda")
    st = jz.lib.jz_knn_noalloc(t.handle, k, ctypes.c_void_p(idx.data_ptr()),
                               ctypes.c_void_p(d2.data_ptr()),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, idx, d2


def test_noalloc_equals_jz_knn_two_calls(jz):
    cases = [(inputs.clustered(400000, 64, 91), 16), (inputs.clustered(30000, 8, 92), 8)]
    for p, k in cases:
        with jz.jz_build(torch.from_numpy(p).cuda()) as t:
            wi, wd = t.knn(k)
            st, gi, gd = noalloc_knn(jz, t, k)
            assert st == jz.JZ_OK, jz.lib.jz_last_error()
            torch.cuda.synchronize()
            assert torch.equal(gi, wi)
            assert torch.equal(gd.view(torch.int32), wd.view(torch.int32))
    # the smaller case also against the oracle
    p, k = cases[1]
    oi, od = oracle.knn_bf(p, k)
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy().view(np.uint32), od.view(np.uint32))


def test_noalloc_rejects_calls_beyond_its_scratch(jz):
    p = inputs.uniform(1 << 23, 93)
    with jz.jz_build(torch.from_numpy(p).cuda()) as t:
        st, _, _ = noalloc_knn(jz, t, 32)
        assert st == jz.JZ_E_CAPACITY
        assert b"fixed scratch" in jz.lib.jz_last_error()
        # the regular entry point still works on the same tree, and a small
        # call after the refused one succeeds
        i, _ = t.knn(32)
    p = inputs.uniform(5000, 94)
    with jz.jz_build(torch.from_numpy(p).cuda()) as t:
        st, gi, gd = noalloc_knn(jz, t, 4)
        assert st == jz.JZ_OK
        wi, wd = t.knn(4)
        assert torch.equal(gi, wi) and torch.equal(gd, wd)
