"""GPU tests of the continuous-batching server (through the C ABI): every
request's result equals its standalone result and the oracle, whatever batch
it ran in."""
import json

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


def make_requests(seed=3):
    rng = np.random.default_rng(seed)
    sizes = [0, 1, 7, 300, 5000, 20000, 48, 1000, 3000, 65, 12000, 2, 700]
    reqs = []
    for i, n in enumerate(sizes):
        p = inputs.clustered(n, max(1, n // 800), seed=1000 + i) if n else np.zeros((0, 3), np.float32)
        if i % 3 == 2:
            reqs.append(("fof", p, float(inputs.linking_length(max(n, 1), rng.uniform(0.1, 0.6)))))
        else:
            reqs.append(("knn", p, int(rng.choice([8, 16]))))
    return reqs


def standalone(jz, op, p, arg):
    with jz.jz_build(torch.from_numpy(p).cuda()) as t:
        if op == "knn":
            i, d = t.knn(arg)
            torch.cuda.synchronize()
            return i.cpu().numpy(), d.cpu().numpy()
        lab = t.fof(arg)
        torch.cuda.synchronize()
        return (lab.cpu().numpy(),)


@pytest.mark.parametrize("streams,max_sets", [(3, 4), (1, 4096), (4, 1)])
def test_server_results_equal_standalone(jz, streams, max_sets):
    reqs = make_requests()
    dev = [torch.from_numpy(p).cuda() for _, p, _ in reqs]
    torch.cuda.synchronize()
    with jz.Server(streams=streams, max_batch_sets=max_sets) as S:
        tickets = []
        for (op, p, arg), d in zip(reqs, dev):
            tickets.append(S.submit_knn(d, arg) if op == "knn" else S.submit_fof(d, arg))
        outs = []
        for t in tickets:
            o, _ = S.wait(t)
            outs.append(tuple(x.cpu().numpy() for x in o))
            S.release(t)
        st = S.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    if max_sets > 1 and streams == 1:
        assert st["batches"] < len(reqs)  # requests were batched
    for (op, p, arg), got in zip(reqs, outs):
        want = standalone(jz, op, p, arg)
        for g, w in zip(got, want):
            assert np.array_equal(g.view(np.uint32) if g.dtype == np.float32 else g,
                                  w.view(np.uint32) if w.dtype == np.float32 else w)
        if op == "knn":
            oi, od = oracle.knn_bf(p, arg) if p.shape[0] else (np.zeros((0, arg), np.int32),) * 2
            assert np.array_equal(got[0], oi)
        else:
            assert np.array_equal(got[0], oracle.fof_bf(p, arg))


def test_server_budget(jz):
    p = torch.from_numpy(inputs.uniform(4000, 8)).cuda()
    torch.cuda.synchronize()
    # a budget that admits one request at a time still completes everything
    with jz.Server(hbm_budget=8_000_000, streams=2) as S:
        ts = [S.submit_knn(p, 8) for _ in range(5)]
        res = [S.wait(t)[0] for t in ts]
        for r in res[1:]:
            assert torch.equal(r[0], res[0][0]) and torch.equal(r[1], res[0][1])
    # a request larger than the whole budget is rejected at submit
    with jz.Server(hbm_budget=1_000_000) as S:
        with pytest.raises(jz.JzError) as e:
            S.submit_knn(p, 8)
        assert e.value.status == jz.JZ_E_OOM
        with pytest.raises(jz.JzError) as e:
            S.submit_knn(p, 300)
        assert e.value.status == jz.JZ_E_UNSUPPORTED


def test_autotune_cache_file(jz, tmp_path, monkeypatch):
    """Winners are appended to the JZ_TUNE_CACHE file, and a signature not yet
    tuned in this process is taken from the file without timing."""
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("JZ_TUNE_CACHE", str(path))
    p = inputs.clustered(5000, 8, 78)
    d = torch.from_numpy(p).cuda()
    opts, ms = jz.jz_autotune(d, k=5)
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    e = json.loads(lines[0])
    assert (e["k"], e["fof"], e["sets"], e["log2n"]) == (5, 0, 1, 12)
    assert (e["leaf_max"], e["coarsen"], e["n_target"], e["ngr"]) == (
        opts.leaf_max, opts.coarsen, opts.n_target, opts.ngr)
    # a hand-written entry for another signature is used as it stands
    e2 = dict(e, k=6, leaf_max=48, coarsen=16, n_target=500, ngr=16, ms=12.5)
    with open(path, "a") as f:
        f.write(json.dumps(e2, separators=(",", ":")) + "\n")
    got, ms2 = jz.jz_autotune(d, k=6)
    assert (got.leaf_max, got.coarsen, got.n_target, got.ngr, ms2) == (48, 16, 500, 16, 12.5)


def test_server_admits_a_later_request_that_fits(jz):
    """With a budget the oldest request cannot get while another batch holds
    part of it, a later small request starts ahead of it; every result is
    still the standalone one."""
    big = torch.from_numpy(inputs.uniform(60000, 31)).cuda()
    small = torch.from_numpy(inputs.uniform(2000, 32)).cuda()
    torch.cuda.synchronize()
    with jz.jz_build(big) as t:
        wi, wd = t.knn(8)
    with jz.jz_build(small) as t:
        si, sd = t.knn(8)
    torch.cuda.synchronize()
    # budget: one big request (about 214 B per point plus 1 MiB) plus a few
    # small ones, but not two big ones
    budget = int(60000 * 300 + (1 << 21) * 3)
    with jz.Server(hbm_budget=budget, streams=2) as S:
        ts = [S.submit_knn(big, 8), S.submit_knn(big, 8)] + [S.submit_knn(small, 8) for _ in range(6)]
        res = [S.wait(x)[0] for x in ts]
    for r in res[:2]:
        assert torch.equal(r[0], wi) and torch.equal(r[1], wd)
    for r in res[2:]:
        assert torch.equal(r[0], si) and torch.equal(r[1], sd)


def test_autotune_picks_valid_options(jz):
    p = inputs.clustered(30000, 16, 77)
    d = torch.from_numpy(p).cuda()
    b = inputs.linking_length(30000)
    opts, ms = jz.jz_autotune(d, k=8, b=b)
    assert opts.leaf_max in (32, 48, 64) and opts.coarsen in (4, 8, 16) and ms > 0
    assert opts.n_target in (500, 1000, 2000) and opts.ngr in (16, 32, 64)
    again, ms2 = jz.jz_autotune(d, k=8, b=b)  # remembered
    assert (again.leaf_max, again.coarsen, ms2) == (opts.leaf_max, opts.coarsen, ms)
    with jz.jz_build(d, opts) as t:
        i, dd = t.knn(8)
        lab = t.fof(b)
        torch.cuda.synchronize()
        wi, wd = oracle.knn_bf(p, 8)
        assert np.array_equal(i.cpu().numpy(), wi) and np.array_equal(dd.cpu().numpy(), wd)
        assert np.array_equal(lab.cpu().numpy(), oracle.fof_bf(p, b))


def test_servers_in_sequence_reuse_cached_memory(jz):
    """Servers created and destroyed one after another: each leaves device
    blocks in the library's cache that its worker streams used last; the next
    server's streams, and a plain call on the default stream, take them over
    after the streams they were used on are gone. Every request must
    succeed and give the same result."""
    p = torch.from_numpy(inputs.clustered(200000, 64, 31)).cuda()
    b = float(inputs.linking_length(200000, 0.2))
    torch.cuda.synchronize()
    first = None
    for rep in range(4):
        with jz.Server(streams=2, max_batch_sets=2) as S:
            ts = [S.submit_knn(p, 16), S.submit_fof(p, b), S.submit_knn(p, 16)]
            outs = [S.wait(t)[0] for t in ts]
            st = S.stats()
            assert st["failed"] == 0, (rep, st)
            got = (outs[0][0].cpu(), outs[1][0].cpu(), outs[2][0].cpu())
            for t in ts:
                S.release(t)
        assert torch.equal(got[0], got[2])
        if first is None:
            first = got
        else:
            assert all(torch.equal(a, c) for a, c in zip(first, got)), rep
    with jz.jz_build(p) as t:
        i, _ = t.knn(16)
        assert torch.equal(i.cpu(), first[0])


def test_server_orders_requests_after_the_callers_stream(jz):
    """Points written on the caller's stream and submitted at once, without a
    synchronization: a side stream is kept busy, then generates the points
    and makes a non-contiguous view of them contiguous. Each request must
    read the finished points (the server waits for the event recorded on the
    caller's stream at submission)."""
    n = 20000
    g = torch.Generator(device="cuda")
    with jz.Server(streams=2) as S:
        for rep in range(3):
            g.manual_seed(100 + rep)
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                a = torch.rand((2048, 2048), device="cuda", generator=g)
                for _ in range(8):  # keep the stream busy before the points exist
                    a = a @ a
                    a = a / a.abs().max()
                base = torch.rand((n, 4), device="cuda", generator=g)
                pts = base[:, 1:]  # non-contiguous: submit makes a contiguous copy on s
                t1 = S.submit_knn(pts, 8)
                t2 = S.submit_fof(pts, float(inputs.linking_length(n, 0.3)))
            (i, d2), _ = S.wait(t1)
            (lab,), _ = S.wait(t2)
            torch.cuda.synchronize()
            p = pts.contiguous().cpu().numpy()
            wi, wd = oracle.knn_bf(p, 8)
            assert np.array_equal(i.cpu().numpy(), wi), rep
            assert np.array_equal(d2.cpu().numpy().view(np.uint32), wd.view(np.uint32)), rep
            assert np.array_equal(lab.cpu().numpy(),
                                  oracle.fof_bf(p, float(inputs.linking_length(n, 0.3)))), rep
            S.release(t1)
            S.release(t2)
