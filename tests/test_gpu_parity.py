"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

kNN indices and squared distances, and FoF labels, must match bit for bit
(integer results: exact; the float32 distances come from the same fixed
expression on both sides, so they are compared bitwise too).
"""
import numpy as np
import pytest

import oracle
from oracle import planes
from paper_2604_05885_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def jz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_05885_amd import api
    return api


def to_dev(p):
    return torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()


def gpu_knn(jz, p, k, **opts):
    with jz.jz_build(to_dev(p), jz.default_opts(**opts) if opts else None) as t:
        idx, d2 = t.knn(k)
        torch.cuda.synchronize()
        return idx.cpu().numpy(), d2.cpu().numpy(), t.stats()


def gpu_fof(jz, p, b, **opts):
    with jz.jz_build(to_dev(p), jz.default_opts(**opts) if opts else None) as t:
        lab = t.fof(b)
        torch.cuda.synchronize()
        return lab.cpu().numpy(), t.stats()


def assert_knn_equal(got_i, got_d, want_i, want_d, what=""):
    bad = np.nonzero(np.any(got_i != want_i, axis=1) | np.any(
        got_d.view(np.uint32) != want_d.view(np.uint32), axis=1))[0]
    assert bad.size == 0, "%s: %d rows differ, first %s: got %s %s want %s %s" % (
        what, bad.size, bad[:1], got_i[bad[:1]], got_d[bad[:1]], want_i[bad[:1]], want_d[bad[:1]])


def small_sets():
    rng = np.random.default_rng(7)
    yield "uniform-16384", inputs.uniform(16384, 1)
    yield "uniform-1000", inputs.uniform(1000, 11)
    yield "clustered-20000", inputs.clustered(20000, 16, 12)
    yield "grid-dups-3000", (rng.integers(0, 6, size=(3000, 3)) * 0.125).astype(np.float32)
    yield "lattice-8", inputs.lattice(8)
    yield "tiny-1", inputs.uniform(1, 2)
    yield "tiny-47", inputs.uniform(47, 3)
    yield "tiny-49", inputs.uniform(49, 4)
    yield "line", np.stack([np.arange(5000) * np.float32(1e-3), np.zeros(5000), np.zeros(5000)],
                           axis=1).astype(np.float32)
    yield "all-identical-300", np.full((300, 3), 0.25, dtype=np.float32)
    yield "negative-wide", (inputs.uniform(4000, 5) * 2e3 - 1e3).astype(np.float32)


@pytest.mark.parametrize("k", [1, 8, 16, 32])
def test_knn_small_sets(jz, k):
    for name, p in small_sets():
        gi, gd, _ = gpu_knn(jz, p, k)
        wi, wd = oracle.knn_bf(p, k)
        assert_knn_equal(gi, gd, wi, wd, "%s k=%d" % (name, k))


@pytest.mark.parametrize("k", [33, 64, 100])
def test_knn_more_than_32(jz, k):
    """k > 32: leaf passes of 32 neighbours, each after the last (dist2,
    index) key of the pass before, against brute force."""
    for name, p in [("uniform-6000", inputs.uniform(6000, 31)),
                    ("clustered-8000", inputs.clustered(8000, 8, 32)),
                    ("grid-dups-2000", (np.random.default_rng(33).integers(0, 5, size=(2000, 3))
                                        * 0.125).astype(np.float32)),
                    ("tiny-70", inputs.uniform(70, 34))]:
        gi, gd, _ = gpu_knn(jz, p, k)
        wi, wd = oracle.knn_bf(p, k)
        assert_knn_equal(gi, gd, wi, wd, "%s k=%d" % (name, k))


def test_knn_more_than_32_lattice_shells(jz):
    """A cubic lattice: interior points have distance shells of 1, 6, 12, 8,
    6, 24, 24, 12, 30 points (r^2/a^2 = 0, 1, 2, 3, 4, 5, 6, 8, 9), so the
    pass boundaries at 32 and 64 neighbours fall inside shells of equal
    distances (cumulative 1, 7, 19, 27, 33, 57, 81): the ties across a pass
    boundary continue by index. Checked against brute force and against the
    closed-form shell sizes."""
    p = inputs.lattice(12)
    a2 = np.float32(2.0 ** -8)
    for k in (40, 70, 96):
        gi, gd, _ = gpu_knn(jz, p, k)
        wi, wd = oracle.knn_bf(p, k)
        assert_knn_equal(gi, gd, wi, wd, "lattice k=%d" % k)
        # the centre point's row: shell radii in order
        c = int(np.argmin(((p - p.mean(axis=0)) ** 2).sum(axis=1)))
        shells = np.repeat([0, 1, 2, 3, 4, 5, 6, 8, 9], [1, 6, 12, 8, 6, 24, 24, 12, 30])[:k]
        assert np.array_equal(gd[c], shells.astype(np.float32) * a2), k


def test_knn_config_small_uniform_k8(jz, fp64_log):
    """N = 16384 uniform, k = 8: the whole result against brute force, and the
    binary64 cross-check of every row (reported, not asserted)."""
    p = inputs.uniform(16384, 1)
    gi, gd, st = gpu_knn(jz, p, 8)
    wi, wd = oracle.knn_bf(p, 8)
    assert_knn_equal(gi, gd, wi, wd)
    flips = oracle.knn_f64_report(p, gi)
    fp64_log.append("uniform N=16384 k=8: %d of 16384 kNN rows differ in binary64 (rows %s)"
                    % (flips.size, flips[:8].tolist()))
    b = inputs.linking_length(16384, 0.2)
    lab, _ = gpu_fof(jz, p, b)
    rep = oracle.fof_f64_report(p, b, labels=lab)
    fp64_log.append("uniform N=16384 FoF alpha=0.2: pairs linked only in float32 %d, only in "
                    "binary64 %d, partition differs: %s" % (
                        rep["pairs_f32_only"], rep["pairs_f64_only"], rep["partition_differs"]))


@pytest.mark.parametrize("leaf_max,k", [(1, 4), (7, 5), (64, 32), (32, 12)])
def test_knn_tree_shapes(jz, leaf_max, k):
    p = inputs.clustered(6000, 8, 21)
    gi, gd, _ = gpu_knn(jz, p, k, leaf_max=leaf_max, ngr=3, n_target=10)
    wi, wd = oracle.knn_bf(p, k)
    assert_knn_equal(gi, gd, wi, wd, "leaf_max=%d" % leaf_max)


def test_knn_long_lists(jz):
    """Leaves of at most 8 points in dense clumps with k = 32: many leaf lists
    are longer than the 256 entries staged in LDS, some longer than the 1024
    a wave sorts in its LDS scratch. With the default sort_max every list is
    put in order (in LDS, or in HBM before its level); with sort_max = 512
    the longer ones are read unordered. Both must equal the exact kd-tree
    oracle."""
    p = inputs.clustered(60000, 16, 21)
    wi, wd = oracle.knn_kd(p, 32)
    gi, gd, st = gpu_knn(jz, p, 32, leaf_max=8)
    assert st["lists_sorted_long"] > 0 and st["lists_unordered"] == 0, st
    # leaf lists longer than 1024 entries went through the multi-wave HBM
    # sorter, and walk lists longer than 256 through the one-wave one
    assert st["lists_presorted_leaf"][1] > 0, st
    assert sum(c[0] for c in st["lists_presorted_walk"]) > 0, st
    assert_knn_equal(gi, gd, wi, wd, "long lists")
    gi, gd, st = gpu_knn(jz, p, 32, leaf_max=8, sort_max=512)
    assert st["lists_sorted_long"] > 0 and st["lists_unordered"] > 0, st
    assert_knn_equal(gi, gd, wi, wd, "long lists, sort_max=512")
    # the same with list capacities far too small: levels are run again and
    # read lists that their first attempt already sorted in place (k = 31,
    # used by no other test, so no learned capacity applies; its exact
    # result is the first 31 columns of the k = 32 one)
    gi, gd, st = gpu_knn(jz, p, 31, leaf_max=8, list_per_node=1.0)
    assert st["reruns"] >= 1 and st["lists_sorted_long"] > 0, st
    assert_knn_equal(gi, gd, wi[:, :31], wd[:, :31], "long lists, rerun")


def test_knn_capacity_regrow_same_result(jz):
    # k = 13 is used by no other test, so no learned capacity applies yet
    p = inputs.clustered(8000, 8, 22)
    gi, gd, st = gpu_knn(jz, p, 13, list_per_node=1.0)
    wi, wd = oracle.knn_bf(p, 13)
    assert_knn_equal(gi, gd, wi, wd)
    assert st["reruns"] >= 1


def test_knn_capacity_error_without_regrow(jz):
    p = inputs.uniform(8000, 23)
    with pytest.raises(jz.JzError) as e:
        gpu_knn(jz, p, 16, list_per_node=1.0, auto_regrow=0)
    assert e.value.status == jz.JZ_E_CAPACITY


@pytest.mark.parametrize("alpha", [0.0, 0.1, 0.2, 0.5, 1.5])
def test_fof_small_sets(jz, alpha):
    for name, p in small_sets():
        b = inputs.linking_length(p.shape[0], alpha) if alpha > 0 else 0.0
        got, _ = gpu_fof(jz, p, b)
        want = oracle.fof_bf(p, b)
        assert np.array_equal(got, want), (name, alpha, np.nonzero(got != want)[0][:5])


def test_fof_lattice_inclusive(jz):
    p = inputs.lattice(10)
    a = 2.0 ** -4
    got, _ = gpu_fof(jz, p, a)
    assert np.all(got == 0)
    got, _ = gpu_fof(jz, p, np.nextafter(np.float32(a), np.float32(0)))
    assert np.array_equal(got, np.arange(p.shape[0]))


def test_fof_dense_clumps(jz):
    p = inputs.clustered(200000, 6, 31, sigma_range=(0.001, 0.003))
    b = inputs.linking_length(200000, 0.2)
    got, st = gpu_fof(jz, p, b)
    want = oracle.fof_kd(p, b)
    assert np.array_equal(got, want)


def subnormal_set():
    """Uniform points plus a cluster at the origin on the grid m * 2^-70
    (m in [0, 8)^3, with repeats): their dist2 are subnormal float32 values
    (down to 2^-140) or exactly 0."""
    rng = np.random.default_rng(71)
    tiny = (rng.integers(0, 8, size=(600, 3)) * 2.0 ** -70).astype(np.float32)
    p = np.concatenate([inputs.uniform(3000, 72), tiny])
    return p[rng.permutation(p.shape[0])]


def test_knn_fof_subnormal_distances(jz):
    p = subnormal_set()
    d = oracle.dist2_f32(p[:, None, :][:50], p[None, :, :])
    assert np.any((d > 0) & (d < np.finfo(np.float32).tiny))  # subnormals occur
    for k in (8, 32):
        gi, gd, _ = gpu_knn(jz, p, k)
        wi, wd = oracle.knn_bf(p, k)
        assert_knn_equal(gi, gd, wi, wd, "subnormal k=%d" % k)
    for b in (0.0, 2.0 ** -70, 1.5 * 2.0 ** -69, inputs.linking_length(p.shape[0], 0.2)):
        got, _ = gpu_fof(jz, p, b)
        assert np.array_equal(got, oracle.fof_bf(p, b)), b


def infinite_set():
    """Uniform points plus two small groups near x = +3e38 and x = -3e38: a
    coordinate difference between groups overflows, so those pairs have
    dist2 = +inf, and the rows of the far groups end in +inf entries
    ordered by index."""
    rng = np.random.default_rng(81)
    far = np.zeros((12, 3), dtype=np.float32)
    far[:6, 0] = np.float32(3e38) - rng.integers(0, 4, 6).astype(np.float32) * np.float32(2e31)
    far[6:, 0] = np.float32(-3e38) + rng.integers(0, 4, 6).astype(np.float32) * np.float32(2e31)
    far[:, 1:] = rng.random((12, 2)).astype(np.float32)
    p = np.concatenate([inputs.uniform(2000, 82), far])
    return p[rng.permutation(p.shape[0])]


def test_knn_fof_infinite_distances(jz):
    p = infinite_set()
    for k in (8, 16, 32):
        gi, gd, _ = gpu_knn(jz, p, k)
        wi, wd = oracle.knn_bf(p, k)
        assert np.isinf(wd).any(), k
        assert_knn_equal(gi, gd, wi, wd, "infinite dist2 k=%d" % k)
    # b = 3e19: fl(b*b) = +inf, so every pair links, also those at +inf
    for b in (0.05, 1e30, 3e19):
        got, _ = gpu_fof(jz, p, b)
        assert np.array_equal(got, oracle.fof_bf(p, b)), b
    assert np.all(gpu_fof(jz, p, 3e19)[0] == 0)


def test_empty_input(jz):
    p = np.zeros((0, 3), dtype=np.float32)
    with jz.jz_build(torch.zeros((0, 3), dtype=torch.float32, device="cuda")) as t:
        idx, d2 = t.knn(4)
        lab = t.fof(0.1)
        assert idx.shape == (0, 4) and lab.shape == (0,)
    del p


def test_errors(jz):
    p = inputs.uniform(100, 1)
    p[17, 1] = np.nan
    with pytest.raises(jz.JzError) as e:
        jz.jz_build(to_dev(p))
    assert e.value.status == jz.JZ_E_NONFINITE
    q = inputs.uniform(100, 1)
    q[3, 0] = np.inf
    with pytest.raises(jz.JzError) as e:
        jz.jz_build(to_dev(q))
    assert e.value.status == jz.JZ_E_NONFINITE
    with jz.jz_build(to_dev(inputs.uniform(100, 1))) as t:
        with pytest.raises(jz.JzError) as e:
            t.knn(257)
        assert e.value.status == jz.JZ_E_UNSUPPORTED
        with pytest.raises(jz.JzError) as e:
            t.fof(-1.0)
        assert e.value.status == jz.JZ_E_INVALID


def test_tree_against_plane_reference(jz):
    """Sorted order, Morton keys and every plane's splits against the
    oracle's plane construction (oracle.planes) on the same keys."""
    p = inputs.clustered(30000, 12, 41)
    opts = jz.default_opts(keep_keys=1, n_target=10, key_bits=21)
    with jz.jz_build(to_dev(p), opts) as t:
        st = t.stats()
        ex = t.export(order=True, keys=True)
        want_keys = planes.interleave(planes.quantize(p))
        order = np.argsort(want_keys, kind="stable")
        assert np.array_equal(ex["order"], order)
        assert np.array_equal(ex["keys"], want_keys[order])
        lv = planes.key_gap_levels(want_keys[order])
        nmax = [opts.leaf_max * opts.coarsen ** q for q in range(st["planes"])]
        ref = planes.planes(list(lv), nmax)
        for q in range(st["planes"]):
            got = t.export(plane=q)["spl"]
            assert np.array_equal(got, np.array(ref[q])), q


def test_forest_equals_standalone(jz):
    rng = np.random.default_rng(5)
    sizes = [0, 1, 5, 48, 49, 300, 1000, 4000, 0, 17, 2500]
    sets = [inputs.clustered(s, max(1, s // 500), seed=100 + i) if s else
            np.zeros((0, 3), np.float32) for i, s in enumerate(sizes)]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    allp = np.concatenate(sets)
    b = np.array([inputs.linking_length(max(s, 1), a) for s, a in
                  zip(sizes, rng.uniform(0.1, 0.8, len(sizes)))], dtype=np.float32)
    with jz.jz_forest_build(to_dev(allp), off) as f:
        idx, d2 = f.knn(9)
        lab = f.fof(b)
        torch.cuda.synchronize()
        idx, d2, lab = idx.cpu().numpy(), d2.cpu().numpy(), lab.cpu().numpy()
    for s, p in enumerate(sets):
        a, e = off[s], off[s + 1]
        if e == a:
            continue
        wi, wd = oracle.knn_bf(p, 9)
        assert_knn_equal(idx[a:e], d2[a:e], wi, wd, "set %d" % s)
        assert np.array_equal(lab[a:e], oracle.fof_bf(p, b[s])), s
        gi, gd, _ = gpu_knn(jz, p, 9)
        assert np.array_equal(gi, idx[a:e]) and np.array_equal(gd, d2[a:e])


def test_full_size_clustered(jz, fp64_log):
    """N = 2^24 clustered (the benchmark workload): kNN k=16 on 2^14 sampled
    rows against brute force and in full against the exact kd-tree oracle; FoF
    in full against the kd-tree oracle; the benchmark's concurrent call on its
    tree (node growth 16) gives the same; binary64 cross-checks of the sampled
    kNN rows and of every FoF pair (reported, not asserted)."""
    n = 2 ** 24
    p = inputs.clustered(n, 4096, 2)
    b = inputs.linking_length(n, 0.2)
    with jz.jz_build(to_dev(p)) as t:
        idx, d2 = t.knn(16)
        lab = t.fof(b)
        torch.cuda.synchronize()
        gi, gd, gl = idx.cpu().numpy(), d2.cpu().numpy(), lab.cpu().numpy()
        del idx, d2, lab
    # the benchmark's call: both halves concurrent, on a tree of node growth
    # 16 per plane; the same results
    with jz.jz_build(to_dev(p), jz.default_opts(coarsen=16)) as t:
        idx, d2, lab = t.knn_fof(16, b)
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), gi)
        assert np.array_equal(d2.cpu().numpy().view(np.uint32), gd.view(np.uint32))
        assert np.array_equal(lab.cpu().numpy(), gl)
        del idx, d2, lab
    rows = np.random.default_rng(9).choice(n, 2 ** 14, replace=False)
    wi, wd = oracle.knn_bf(p, 16, rows=rows)
    assert_knn_equal(gi[rows], gd[rows], wi, wd, "sampled rows")
    ki, kd = oracle.knn_kd(p, 16)
    assert_knn_equal(gi, gd, ki, kd, "full kd")
    assert np.array_equal(gl, oracle.fof_kd(p, b))
    flips = oracle.knn_f64_report(p, gi[rows], rows=rows)
    fp64_log.append("clustered N=2^24 k=16: %d of %d sampled kNN rows differ in binary64"
                    % (flips.size, rows.size))
    rep = oracle.fof_f64_report(p, b, labels=gl)
    fp64_log.append("clustered N=2^24 FoF alpha=0.2: pairs linked only in float32 %d, only in "
                    "binary64 %d, partition differs: %s (%d points relabelled)" % (
                        rep["pairs_f32_only"], rep["pairs_f64_only"], rep["partition_differs"],
                        rep["points_relabelled"]))


def test_regularization_same_results_smaller_nodes(jz):
    """A tight Gaussian with a few points far from the bulk (the paper's case
    for regularization): with reg_fmax = 50 the far points no longer share
    huge nodes (more leaves), and every result is still exact."""
    rng = np.random.default_rng(61)
    bulk = (0.5 + 0.01 * rng.standard_normal((30000, 3))).astype(np.float32)
    far = rng.random((40, 3)).astype(np.float32)
    p = np.concatenate([bulk, far])[rng.permutation(30040)]
    wi, wd = oracle.knn_bf(p, 16)
    b = inputs.linking_length(30040, 0.3) * 0.05
    wl = oracle.fof_bf(p, b)
    leaves = []
    for fmax in (0.0, 50.0):
        gi, gd, st = gpu_knn(jz, p, 16, reg_fmax=fmax)
        assert_knn_equal(gi, gd, wi, wd, "reg_fmax=%g" % fmax)
        lab, _ = gpu_fof(jz, p, b, reg_fmax=fmax)
        assert np.array_equal(lab, wl), fmax
        leaves.append(st["nodes"][0])
    assert leaves[1] > leaves[0], leaves


@pytest.mark.parametrize("key_bits", [1, 4, 10, 13, 21])
def test_key_width_never_changes_results(jz, key_bits):
    """Coarse Morton keys make many points share a key (equal keys are cut
    into aligned power-of-two runs of sorted positions); the automatic width
    and explicit widths must all give the exact result."""
    p = inputs.clustered(20000, 16, 71)
    wi, wd = oracle.knn_bf(p, 16)
    b = inputs.linking_length(20000, 0.2)
    wl = oracle.fof_bf(p, b)
    gi, gd, _ = gpu_knn(jz, p, 16, key_bits=key_bits)
    assert_knn_equal(gi, gd, wi, wd, "key_bits=%d" % key_bits)
    lab, _ = gpu_fof(jz, p, b, key_bits=key_bits)
    assert np.array_equal(lab, wl), key_bits


def test_knn_fof_in_one_call(jz):
    """jz_knn_fof (kNN on the given stream, FoF concurrently on a second one)
    gives the oracle's results and those of the two calls made one after the
    other, with the same kNN statistics; a call whose lists overflow reruns its
    half on its own; a stream that is not the default one is ordered
    before and after both halves; argument errors are those of jz_knn and
    jz_fof."""
    p = inputs.clustered(30000, 24, 91)
    b = inputs.linking_length(30000, 0.2)
    wi, wd = oracle.knn_bf(p, 16)
    wl = oracle.fof_bf(p, b)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        # (k = 11, so no capacity learned by other tests applies: the first call reruns)
        for k, lpn in ((11, 1.0), (16, None)):
            opts = jz.default_opts(list_per_node=lpn) if lpn else None
            dev = to_dev(p)  # queued on s: the call must wait for the copy
            with jz.jz_build(dev, opts, stream=s) as t:
                gi, gd, gl = t.knn_fof(k, b, stream=s)
                ks, fs = t.last_stats
                assert t.stats()["evaluations"] == ks["evaluations"]
                ri, rd = t.knn(k, stream=s)
                ks2 = t.stats()
                rl = t.fof(b, stream=s)
                fs2 = t.stats()
                s.synchronize()
                gi, gd, gl = gi.cpu().numpy(), gd.cpu().numpy(), gl.cpu().numpy()
                want_i, want_d = oracle.knn_bf(p, k) if k != 16 else (wi, wd)
                assert_knn_equal(gi, gd, want_i, want_d, "knn_fof k=%d" % k)
                assert np.array_equal(gl, wl)
                assert np.array_equal(gi, ri.cpu().numpy())
                assert np.array_equal(gd.view(np.uint32), rd.cpu().numpy().view(np.uint32))
                assert np.array_equal(gl, rl.cpu().numpy())
                for key in ("evaluations", "leaf_pairs", "list_entries", "nodes"):
                    assert ks[key] == ks2[key], key
                # (FoF's lists and evaluation counts depend on when unions
                # land: pairs found already connected are dropped)
                assert fs["nodes"] == fs2["nodes"] and fs["planes"] == fs2["planes"]
                assert fs["evaluations"] > 0 and fs["leaf_pairs"] > 0
                if lpn:  # (FoF capacities learned by earlier calls may spare its rerun)
                    assert ks["reruns"] >= 1, ks["reruns"]
    with jz.jz_build(to_dev(inputs.uniform(100, 1))) as t:
        with pytest.raises(jz.JzError) as e:
            t.knn_fof(257, 0.1)
        assert e.value.status == jz.JZ_E_UNSUPPORTED
        with pytest.raises(jz.JzError) as e:
            t.knn_fof(4, -1.0)
        assert e.value.status == jz.JZ_E_INVALID
    with jz.jz_build(torch.zeros((0, 3), dtype=torch.float32, device="cuda")) as t:
        gi, gd, gl = t.knn_fof(4, 0.1)
        assert gi.shape == (0, 4) and gl.shape == (0,)
    # lists too small and no regrow: the kNN half's error is returned (the
    # FoF half's, if it failed too, is not)
    q = inputs.uniform(8000, 23)
    opts = jz.default_opts(list_per_node=1.0, auto_regrow=0)
    with jz.jz_build(to_dev(q), opts) as t:
        with pytest.raises(jz.JzError) as e:
            t.knn_fof(16, inputs.linking_length(8000, 0.2))
        assert e.value.status == jz.JZ_E_CAPACITY
        assert "interaction list overflow" in str(e.value) and "FoF" not in str(e.value)
