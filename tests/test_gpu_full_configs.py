"""GPU parity at the full sizes of the benchmark configurations (through the
C ABI), in the launch configuration the benchmark uses:

* N = 2^27 clustered (2^16 clumps), kNN k = 32 and FoF at alpha = 0.2:
  every kNN row against the exact kd-tree oracle, sampled rows against brute
  force, whole-output invariants on the GPU, and every FoF label against the
  kd-tree oracle;
* 4096 ragged clustered sets (N log-uniform in [2^10, 2^18]) solved as one
  forest: every set equal to its standalone solve, sampled sets against the
  oracle;
* a Poisson request stream (N log-uniform in [2^12, 2^22], mixed kNN / FoF)
  through the continuous-batching server: every result equal to its
  standalone solve, sampled requests against the oracle.
"""
import time

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


def say(*a):
    print(*a, flush=True)


def knn_rows_equal(gi, gd, rows, p, k, what):
    wi, wd = oracle.knn_bf(p, k, rows=rows)
    bad = np.nonzero(np.any(gi != wi, axis=1) |
                     np.any(gd.view(np.uint32) != wd.view(np.uint32), axis=1))[0]
    assert bad.size == 0, "%s: %d sampled rows differ (first row %d)" % (what, bad.size,
                                                                        rows[bad[0]])


def knn_invariants(pts, idx, d2):
    """Properties every exact self-query result has, checked on the GPU:
    entries in range and distinct per row, rows ascending by (dist2, index),
    the first entry at distance 0, and every dist2 equal to the fixed
    expression evaluated for the reported pair."""
    n, k = idx.shape
    assert int(idx.min()) >= 0 and int(idx.max()) < n
    assert bool((d2[:, 0] == 0).all())
    if k > 1:
        dd, ii = d2[:, 1:], idx[:, 1:]
        dp, ip = d2[:, :-1], idx[:, :-1]
        assert bool(((dd > dp) | ((dd == dp) & (ii > ip))).all())
    for c in range(0, n, 1 << 22):
        e = min(n, c + (1 << 22))
        q = pts[c:e].unsqueeze(1)
        s = pts[idx[c:e].long()]
        dx = q[..., 0] - s[..., 0]
        dy = q[..., 1] - s[..., 1]
        dz = q[..., 2] - s[..., 2]
        xx = dx * dx
        yy = dy * dy
        zz = dz * dz
        ref = (xx + yy) + zz
        assert torch.equal(ref.view(torch.int32), d2[c:e].view(torch.int32))


@pytest.mark.timeout(1200)
def test_config_2p27_k32(jz):
    """Every one of the 2^27 x 32 kNN entries against the exact kd-tree oracle
    (compared in row chunks: the result is 32 GiB), 2^11 random rows against
    brute force (each row is 2^27 evaluations), whole-output invariants on
    the GPU, and every FoF label against the kd-tree oracle."""
    n = 2 ** 27
    t0 = time.time()
    p = inputs.clustered(n, 2 ** 16, 3)
    b = inputs.linking_length(n, 0.2)
    say("inputs %.1fs" % (time.time() - t0))
    d = torch.from_numpy(p).cuda()
    with jz.jz_build(d) as t:
        idx, d2 = t.knn(32)
        lab = t.fof(b)
        torch.cuda.synchronize()
        say("gpu done %.1fs" % (time.time() - t0))
        knn_invariants(d, idx, d2)
        gl = lab.cpu().numpy()
        del lab
    del d
    rows = np.random.default_rng(27).choice(n, 2 ** 11, replace=False)
    for r0 in range(0, rows.size, 256):
        rs = rows[r0:r0 + 256]
        ridx = torch.from_numpy(rs).cuda()
        knn_rows_equal(idx[ridx].cpu().numpy(), d2[ridx].cpu().numpy(), rs, p, 32, "2^27 k=32")
        say("brute-force rows %d %.1fs" % (r0 + rs.size, time.time() - t0))
    chunk = 1 << 22
    with oracle.KdTree(p) as kd:
        say("kd-tree %.1fs" % (time.time() - t0))
        for c in range(0, n, chunk):
            wi, wd = kd.rows(c, chunk, 32)
            gi = idx[c:c + chunk].cpu().numpy()
            gd = d2[c:c + chunk].cpu().numpy()
            bad = np.nonzero(np.any(gi != wi, axis=1) |
                             np.any(gd.view(np.uint32) != wd.view(np.uint32), axis=1))[0]
            assert bad.size == 0, "2^27 k=32: %d rows differ in rows [%d, %d), first %d" % (
                bad.size, c, c + chunk, c + bad[0])
            if (c // chunk) % 8 == 7:
                say("kd rows up to %d %.1fs" % (c + chunk, time.time() - t0))
    del idx, d2
    torch.cuda.empty_cache()
    assert np.array_equal(gl, oracle.fof_kd(p, b))
    say("fof %.1fs" % (time.time() - t0))


def test_config_batched_4096(jz):
    t0 = time.time()
    p, off, b = inputs.batched_sets(4096, 4)
    say("inputs %.1fs, %d points" % (time.time() - t0, off[-1]))
    d = torch.from_numpy(p).cuda()
    with jz.jz_forest_build(d, off) as f:
        idx, d2 = f.knn(16)
        lab = f.fof(b)
        torch.cuda.synchronize()
    say("forest %.1fs" % (time.time() - t0))
    for s in range(4096):
        a, e = int(off[s]), int(off[s + 1])
        with jz.jz_build(d[a:e]) as t:
            si, sd = t.knn(16)
            sl = t.fof(b[s])
            assert torch.equal(si, idx[a:e]), s
            assert torch.equal(sd.view(torch.int32), d2[a:e].view(torch.int32)), s
            assert torch.equal(sl, lab[a:e]), s
    say("standalone %.1fs" % (time.time() - t0))
    sizes = np.diff(off)
    rng = np.random.default_rng(44)
    picks = list(rng.choice(4096, 6, replace=False)) + [int(np.argmax(sizes)),
                                                       int(np.argmin(sizes))]
    for s in picks:
        a, e = int(off[s]), int(off[s + 1])
        ps = p[a:e]
        ki, kd = oracle.knn_kd(ps, 16)
        assert np.array_equal(idx[a:e].cpu().numpy(), ki), s
        assert np.array_equal(d2[a:e].cpu().numpy().view(np.uint32), kd.view(np.uint32)), s
        assert np.array_equal(lab[a:e].cpu().numpy(), oracle.fof_kd(ps, b[s])), s
    say("oracle %.1fs" % (time.time() - t0))


def test_config_served_stream(jz):
    t0 = time.time()
    sched = inputs.served_requests(48, 5)
    pts = [torch.from_numpy(inputs.clustered(r["n"], r["clumps"], r["seed"])).cuda()
           for r in sched]
    torch.cuda.synchronize()
    say("inputs %.1fs, %d points" % (time.time() - t0, sum(r["n"] for r in sched)))
    tickets = []
    with jz.Server() as S:
        start = time.perf_counter()
        for r, d in zip(sched, pts):
            while time.perf_counter() - start < r["t"]:
                time.sleep(2e-5)
            if r["op"] == "knn":
                tickets.append(S.submit_knn(d, r["k"]))
            else:
                tickets.append(S.submit_fof(d, inputs.linking_length(r["n"], r["alpha"])))
        outs = []
        for tk in tickets:
            o, _ = S.wait(tk)
            outs.append(o)
        st = S.stats()
        assert st["completed"] == len(sched) and st["failed"] == 0
        say("served %.1fs, %d batches" % (time.time() - t0, st["batches"]))
        for i, (r, d, o) in enumerate(zip(sched, pts, outs)):
            with jz.jz_build(d) as t:
                if r["op"] == "knn":
                    si, sd = t.knn(r["k"])
                    assert torch.equal(si, o[0]), i
                    assert torch.equal(sd.view(torch.int32), o[1].view(torch.int32)), i
                else:
                    sl = t.fof(inputs.linking_length(r["n"], r["alpha"]))
                    assert torch.equal(sl, o[0]), i
        say("standalone %.1fs" % (time.time() - t0))
        order = np.argsort([r["n"] for r in sched])
        for i in list(order[:3]) + [int(order[len(order) // 2])]:
            r = sched[i]
            ps = pts[i].cpu().numpy()
            if r["op"] == "knn":
                ki, kd = oracle.knn_kd(ps, r["k"])
                assert np.array_equal(outs[i][0].cpu().numpy(), ki), i
                assert np.array_equal(outs[i][1].cpu().numpy().view(np.uint32),
                                      kd.view(np.uint32)), i
            else:
                assert np.array_equal(outs[i][0].cpu().numpy(),
                                      oracle.fof_kd(ps, inputs.linking_length(r["n"],
                                                                              r["alpha"]))), i
        for tk in tickets:
            S.release(tk)
    say("oracle %.1fs" % (time.time() - t0))
