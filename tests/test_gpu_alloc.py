"""Device memory from a caller's allocator (jz_allocator, through the C ABI):
torch's caching allocator gives the same results as the library's own pool,
every block is returned, and an allocator that fails at any point of a call
makes that call return JZ_E_OOM without leaking a block."""
import gc

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


def test_torch_allocator_results_and_accounting(jz):
    p = inputs.clustered(30000, 16, 61)
    b = inputs.linking_length(30000, 0.3)
    d = torch.from_numpy(p).cuda()
    torch.cuda.synchronize()
    A = jz.TorchAllocator()
    # tensors of earlier tests freed by the garbage collector meanwhile would
    # lower torch's count: collect first and hold the collector off
    gc.collect()
    gc.disable()
    try:
        before = torch.cuda.memory_allocated()
        t = jz.jz_build(d, allocator=A)
        held = t.size()
        grown = torch.cuda.memory_allocated() - before
    finally:
        gc.enable()
    with t:
        assert held >= 30000 * 16 and A.live > 0
        assert A.live_bytes >= held and grown >= held
        i, d2 = t.knn(16)
        lab = t.fof(b)
        torch.cuda.synchronize()
        live_tree = A.live
    assert A.live == 0 and live_tree > 0
    del i, d2, lab
    wi, wd = oracle.knn_bf(p, 16)
    with jz.jz_build(d, allocator="torch") as t:
        i, d2 = t.knn(16)
        lab = t.fof(b)
        torch.cuda.synchronize()
        assert np.array_equal(i.cpu().numpy(), wi)
        assert np.array_equal(d2.cpu().numpy().view(np.uint32), wd.view(np.uint32))
        assert np.array_equal(lab.cpu().numpy(), oracle.fof_bf(p, b))
    assert jz.torch_allocator().live == 0
    offs = np.array([0, 10000, 10000, 30000])
    with jz.jz_forest_build(d, offs, allocator="torch") as f:
        i, _ = f.knn(8)
        torch.cuda.synchronize()
        assert np.array_equal(i[10000:].cpu().numpy(), oracle.knn_bf(p[10000:], 8)[0])
    assert jz.torch_allocator().live == 0


def test_torch_allocator_from_two_threads(jz):
    """jz_knn_fof takes memory from the calling thread (kNN half) and from a
    second thread of the library's (FoF half, on its own stream) at once:
    the results are the oracle's, and every block is returned."""
    p = inputs.clustered(30000, 16, 63)
    b = inputs.linking_length(30000, 0.2)
    d = torch.from_numpy(p).cuda()
    wi, wd = oracle.knn_bf(p, 12)
    wl = oracle.fof_bf(p, b)
    A = jz.TorchAllocator()
    for _ in range(2):
        with jz.jz_build(d, allocator=A) as t:
            i, d2, lab = t.knn_fof(12, b)
            torch.cuda.synchronize()
            assert np.array_equal(i.cpu().numpy(), wi)
            assert np.array_equal(d2.cpu().numpy().view(np.uint32), wd.view(np.uint32))
            assert np.array_equal(lab.cpu().numpy(), wl)
        assert A.live == 0 and A.live_bytes == 0
    assert A.allocs > 0


class FailingAllocator:
    """torch's caching allocator, except that allocation number ``fail_at``
    (1-based, counted from ``arm()``) returns NULL."""

    def __init__(self, jz):
        self.inner = jz.TorchAllocator()
        self.fail_at = 0
        self.count = 0
        self.failed = False
        A = jz.Allocator
        self._a = A._fields_[1][1](self._alloc)
        self._f = A._fields_[2][1](self._free)
        self.struct = A(None, self._a, self._f)

    def arm(self, fail_at):
        self.fail_at, self.count, self.failed = fail_at, 0, False

    def _alloc(self, ctx, nbytes, stream):
        self.count += 1
        if self.count == self.fail_at:
            self.failed = True
            return None
        return self.inner._alloc(ctx, nbytes, stream)

    def _free(self, ctx, ptr, nbytes, stream):
        self.inner._free(ctx, ptr, nbytes, stream)

    @property
    def live(self):
        return self.inner.live


def test_allocator_failure_is_oom_without_leak(jz):
    p = inputs.clustered(20000, 8, 62)
    b = inputs.linking_length(20000, 0.3)
    d = torch.from_numpy(p).cuda()
    wi, wd = oracle.knn_bf(p, 8)
    wl = oracle.fof_bf(p, b)
    A = FailingAllocator(jz)
    # how many allocations each call makes
    A.arm(0)
    with jz.jz_build(d, allocator=A) as t:
        n_build = A.count
        A.arm(0)
        t.knn(8)
        n_knn = A.count
        A.arm(0)
        t.fof(b)
        n_fof = A.count
    assert A.live == 0 and n_build > 5 and n_knn > 3 and n_fof > 3
    for m in range(1, n_build + 1):
        A.arm(m)
        with pytest.raises(jz.JzError) as e:
            jz.jz_build(d, allocator=A)
        assert e.value.status == jz.JZ_E_OOM and A.failed, m
        assert A.live == 0, ("build", m, A.live)
    A.arm(0)
    with jz.jz_build(d, allocator=A) as t:
        held = A.live
        for what, call, n_calls in (("knn", lambda: t.knn(8), n_knn),
                                    ("fof", lambda: t.fof(b), n_fof)):
            # a call may make fewer allocations than its first run (list
            # capacities learned by then): stop at the first run that succeeds
            for m in range(1, n_calls + 1):
                A.arm(m)
                try:
                    call()
                except jz.JzError as e:
                    assert A.failed and e.status == jz.JZ_E_OOM, (what, m, e)
                else:
                    assert not A.failed, (what, m)
                    break
                assert A.live == held, (what, m, A.live, held)
        # the tree is intact after failed calls
        A.arm(0)
        i, d2 = t.knn(8)
        lab = t.fof(b)
        torch.cuda.synchronize()
        assert np.array_equal(i.cpu().numpy(), wi)
        assert np.array_equal(d2.cpu().numpy().view(np.uint32), wd.view(np.uint32))
        assert np.array_equal(lab.cpu().numpy(), wl)
    assert A.live == 0
