"""The three ways a batch runs (host-driven rounds, the planned launch
sequence, a captured HIP graph) give bit-identical results and statistics,
and a replayed graph reads the current contents of the caller's buffers.

Every replay is checked against an eager search, with the program's own eager
work and synchronisations between replays.  Parity of the shared result with
the FP64 oracle is checked on the replayed output as well.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

COUNTS = ("leaves_scanned", "leaves_lb_pruned", "leaves_filter_pruned", "series_scanned", "fallback_items",
          "rounds", "scan_bytes")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    raw = W.random_walk(24000, 128, seed=611)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=800, n_segments=16)
    N = ix.info()["n_leaves"]
    h = 32
    w = W.mlp_weights(N, 128, h, seed=612, out_bias=4.0)
    offs = np.random.default_rng(613).uniform(0.0, 3.5, N).astype(np.float32)
    ix.set_filters(np.arange(N, dtype=np.int32), torch.from_numpy(w).cuda(), h)
    ix.set_offsets([1, 10], [0.9], np.stack([offs, offs]))
    nq = 300
    q = [W.noisy_queries(raw, nq, (0.05, 0.3), 614 + i, 714 + i)[0] for i in range(3)]
    rng = np.random.default_rng(615)
    ks = rng.choice([1, 10], nq).astype(np.int32)
    ts = rng.choice([0.9, 1.0], nq).astype(np.float32)
    # k and target stay in the same device buffers: a graph is replayed only
    # for the buffer addresses it was captured with
    kd, td = torch.from_numpy(ks).cuda(), torch.from_numpy(ts).cuda()
    return dict(pkg=pkg, raw=raw, ix=ix, w=w, h=h, offs=offs, q=q, ks=ks, ts=ts, kd=kd, td=td, N=N)


def _search(env, qd, flags, out=None, stats=True):
    r = env["ix"].search(qd, k=env["kd"], target=env["td"], k_max=10, schedule=(1, 0), with_stats=stats, out=out, flags=flags)
    torch.cuda.synchronize()
    return r


def test_paths_are_bit_identical(env):
    pkg = env["pkg"]
    qd = torch.from_numpy(env["q"][0]).cuda()
    i0, d0, s0 = _search(env, qd, pkg.SEARCH_HOST_ROUNDS)
    assert s0["path"] == 0
    i1, d1, s1 = _search(env, qd, pkg.SEARCH_NO_GRAPH)
    assert s1["path"] == 1
    out = (torch.empty_like(i0), torch.empty_like(d0))
    paths = []
    for rep in range(4):
        out[0].fill_(-7)
        out[1].fill_(-7.0)
        i2, d2, s2 = _search(env, qd, 0, out=out)
        paths.append(s2["path"])
        assert torch.equal(i2, i0) and torch.equal(d2, d0), rep
        for c in COUNTS:
            assert s2[c] == s0[c] == s1[c], (c, s0[c], s1[c], s2[c])
        assert s2["ms_scan"] > 0.0
    assert torch.equal(i1, i0) and torch.equal(d1, d0)
    assert 3 in paths and paths[-1] == 2, paths
    assert env["ix"].graph_note() == ""


def test_capacity_checked_plans_fall_back_on_overflow(env):
    """A planned batch whose item buffers are sized below the worst case
    (leafi_set_plan_capacity) checks every round's item count on the device.
    Sized for batch A, A runs planned, then captured and replayed, with the
    host-driven results.  The replayed graph then meets batch B (noisier
    queries, far more leaves per query) in the same buffers: its second round
    overflows, lays out nothing, and the call runs B again with host-driven
    rounds (path 4); later calls of that shape run host-driven rounds at once
    (path 0).  With room for the first round only, a planned call overflows
    as well.  The no-allocation search refuses a capacity-checked plan.  The
    capacity is forced from the host: every kernel still runs to its end."""
    pkg = env["pkg"]
    ix = env["ix"]
    qa = env["q"][1]
    qb = W.noisy_queries(env["raw"], len(qa), 1.5, 616, 716)[0]
    nq = len(qa)
    ra = _search(env, torch.from_numpy(qa).cuda(), pkg.SEARCH_HOST_ROUNDS)
    rb = _search(env, torch.from_numpy(qb).cuda(), pkg.SEARCH_HOST_ROUNDS)
    assert ra[2]["rounds"] == 2
    # B's second round alone holds more items than all of A's rounds
    assert rb[2]["leaves_scanned"] - nq > ra[2]["leaves_scanned"] + ra[2]["fallback_items"], (ra[2], rb[2])
    qd = torch.from_numpy(qa).cuda()
    out = (torch.empty_like(ra[0]), torch.empty_like(ra[1]))
    try:
        ix.set_plan_capacity(ra[2]["leaves_scanned"] + ra[2]["fallback_items"])
        paths = []
        for rep in range(3):
            out[0].fill_(-7)
            out[1].fill_(-7.0)
            i1, d1, s1 = _search(env, qd, 0, out=out)
            paths.append(s1["path"])
            assert torch.equal(i1, ra[0]) and torch.equal(d1, ra[1]), rep
            for c in COUNTS:
                assert s1[c] == ra[2][c], (c, ra[2][c], s1[c])
        assert paths == [1, 3, 2], paths
        qd.copy_(torch.from_numpy(qb).cuda())  # same buffer, batch B
        paths = []
        for rep in range(3):
            out[0].fill_(-7)
            out[1].fill_(-7.0)
            i2, d2, s2 = _search(env, qd, 0, out=out)
            paths.append(s2["path"])
            assert torch.equal(i2, rb[0]) and torch.equal(d2, rb[1]), rep
            for c in COUNTS:
                assert s2[c] == rb[2][c], (c, rb[2][c], s2[c])
        assert paths == [4, 0, 0], paths
        # room for the first round (one leaf per query) only, a shape of its
        # own (other output buffers), without statistics: the overflow is
        # read back all the same
        ix.set_plan_capacity(nq + 1)
        out2 = (torch.empty_like(ra[0]), torch.empty_like(ra[1]))
        qd.copy_(torch.from_numpy(qa).cuda())
        i3, d3 = _search(env, qd, pkg.SEARCH_NO_GRAPH, out=out2, stats=False)
        assert torch.equal(i3, ra[0]) and torch.equal(d3, ra[1])
        with pytest.raises(pkg.LeafiError):
            ix.search_noalloc(qd, env["kd"], env["td"], out2, k_max=10, schedule=(1, 0))
        with pytest.raises(pkg.LeafiError):
            ix.set_plan_capacity(-1)
        # room again: the overflow word does not linger
        ix.set_plan_capacity(0)
        i4, d4, s4 = _search(env, qd, pkg.SEARCH_NO_GRAPH)
        assert s4["path"] == 1 and torch.equal(i4, ra[0]) and torch.equal(d4, ra[1])
    finally:
        ix.set_plan_capacity(0)


def test_graph_replay_reads_current_buffers(env):
    pkg = env["pkg"]
    qd = torch.from_numpy(env["q"][0]).cuda()
    out = (torch.empty((len(env["ks"]), 10), dtype=torch.int64, device="cuda"),
           torch.empty((len(env["ks"]), 10), dtype=torch.float32, device="cuda"))
    for _ in range(3):  # make sure this shape is captured
        _search(env, qd, 0, out=out, stats=False)
    seen = []
    for rep in range(6):
        src = env["q"][rep % 3]
        qd.copy_(torch.from_numpy(src).cuda())          # same buffer, new contents
        ids, d = _search(env, qd, 0, out=out, stats=False)
        got = (ids.clone(), d.clone())
        # eager work in between: a host-driven search of the same queries on other buffers
        e_ids, e_d, st = _search(env, torch.from_numpy(src).cuda(), pkg.SEARCH_HOST_ROUNDS)
        assert st["path"] == 0
        assert torch.equal(got[0], e_ids) and torch.equal(got[1], e_d), rep
        seen.append(got[0].cpu().numpy())
    assert not np.array_equal(seen[0], seen[1])  # the batches really differ


def test_replayed_result_matches_oracle(env):
    qd = torch.from_numpy(env["q"][1]).cuda()
    out = (torch.empty((len(env["ks"]), 10), dtype=torch.int64, device="cuda"),
           torch.empty((len(env["ks"]), 10), dtype=torch.float32, device="cuda"))
    for _ in range(3):
        ids, d, st = _search(env, qd, 0, out=out)
    assert st["path"] == 2
    ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
    xs, qs = O.znorm(env["raw"]), O.znorm(env["q"][1])
    mu, sd = O.segment_stats(xs, 16)
    t = O.build_tree(mu, sd, 128, 800, "median")
    lb = O.lower_bound(*O.query_stats(qs, 16), O.leaf_boxes(mu, sd, t), 128)
    order = O.visit_order(lb)
    ld, li = O.leaf_knn(xs, t.leaves, qs, 10)
    df = np.stack([O.mlp_forward(env["w"][f], qs, 128, env["h"]) for f in range(env["N"])], 1)
    has = np.ones(env["N"], dtype=bool)
    for k in (1, 10):
        for tgt in (0.9, 1.0):
            sel = np.nonzero((env["ks"] == k) & (env["ts"] == tgt))[0]
            offs = env["offs"] if tgt < 1.0 else np.full(env["N"], np.inf)
            r = O.leafi_search(lb[sel], order[sel], ld[sel], li[sel], k, has, df[sel] - offs[None], (1, 0))
            fin = np.isfinite(r.dist)
            assert np.all(np.abs(d[sel, :k][fin] - r.dist[fin]) <= 1e-4 * r.dist[fin])
            for a, b in zip(*np.nonzero(ids[sel, :k] != r.ids)):
                x = xs[ids[sel][a, b]].astype(np.float64)
                dg = np.sqrt(((x - qs[sel[a]]) ** 2).sum())
                assert abs(dg - r.dist[a, b]) <= 3e-5 * r.dist[a, b]
            assert (ids[sel, k:] == -1).all()


def test_autotune_keeps_results_identical(env):
    """Every tile shape the tuner tries gives the same results; the chosen one
    is then used by later searches."""
    pkg = env["pkg"]
    qd = torch.from_numpy(env["q"][2]).cuda()
    before = _search(env, qd, pkg.SEARCH_NO_GRAPH)
    rep = env["ix"].autotune(qd, k=env["kd"], target=env["td"], k_max=10, schedule=(1, 0), repeats=2)
    # three tile heights times four query counts
    assert len(rep["candidates"]) == 12
    assert {c["chunk_rows"] for c in rep["candidates"]} == {512, 1024, 2048}
    assert {c["queries_per_tile"] for c in rep["candidates"]} == {16, 32, 48, 64}
    assert all(c["ms"] > 0 for c in rep["candidates"])
    assert rep["chosen"]["ms"] == min(c["ms"] for c in rep["candidates"])
    after = _search(env, qd, pkg.SEARCH_NO_GRAPH)
    assert torch.equal(before[0], after[0]) and torch.equal(before[1], after[1])
    for c in ("leaves_scanned", "leaves_filter_pruned", "fallback_items"):
        assert before[2][c] == after[2][c]
    # k = 1 (4 candidates): the same shapes
    k1 = torch.ones(len(env["ks"]), dtype=torch.int32, device="cuda")
    ids_a, d_a = env["ix"].search(qd, k=k1, target=env["td"], k_max=1, schedule=(1, 0), flags=pkg.SEARCH_NO_GRAPH)
    rep1 = env["ix"].autotune(qd, k=k1, target=env["td"], k_max=1, schedule=(1, 0), repeats=2)
    assert len(rep1["candidates"]) == 12
    ids_b, d_b = env["ix"].search(qd, k=k1, target=env["td"], k_max=1, schedule=(1, 0), flags=pkg.SEARCH_NO_GRAPH)
    assert torch.equal(ids_a, ids_b) and torch.equal(d_a, d_b)
    # every shape, set directly, for the mixed-k batch
    for chunk in (128, 512, 2048, 4096):
        for mq in (16, 32, 48, 64):
            env["ix"].set_tiling(chunk, mq)
            got = _search(env, qd, pkg.SEARCH_NO_GRAPH)
            assert torch.equal(got[0], before[0]) and torch.equal(got[1], before[1]), (chunk, mq)
    env["ix"].set_tiling(1024, 32)
    with pytest.raises(pkg.LeafiError):
        env["ix"].set_tiling(1000, 32)
    with pytest.raises(pkg.LeafiError):
        env["ix"].set_tiling(1024, 24)


def test_deferred_rescans_agree_and_stay_exact(env):
    """With k' = k every first-round item fails its certificate (its k'-th
    candidate is the k-th result itself), so the whole first round is rescanned
    by the second round's scan, and what fails again by the final FP32 pass.
    The three paths agree bit for bit, and the answer is the exact k-NN of the
    FP64 oracle."""
    pkg = env["pkg"]
    qd = torch.from_numpy(env["q"][1]).cuda()
    k = 10
    # a graph is replayed only for the buffer addresses it was captured with
    nq = len(env["ks"])
    kd = torch.full((nq,), k, dtype=torch.int32, device="cuda")
    td = torch.ones(nq, dtype=torch.float32, device="cuda")
    out = (torch.empty((nq, k), dtype=torch.int64, device="cuda"),
           torch.empty((nq, k), dtype=torch.float32, device="cuda"))
    res = []
    for flags in (pkg.SEARCH_HOST_ROUNDS, pkg.SEARCH_NO_GRAPH, 0, 0, 0):
        ids, d, st = env["ix"].search(qd, k=kd, target=td, k_max=k, use_filters=False, schedule=(1, 0), kprime=k,
                                      with_stats=True, flags=flags, out=out)
        torch.cuda.synchronize()
        res.append((ids.clone(), d.clone(), st))
    assert [r[2]["path"] for r in res][:2] == [0, 1] and res[-1][2]["path"] == 2
    for ids, d, st in res[1:]:
        assert torch.equal(ids, res[0][0]) and torch.equal(d, res[0][1])
        for c in COUNTS:
            assert st[c] == res[0][2][c], (c, st[c], res[0][2][c])
    assert res[0][2]["fallback_items"] >= len(env["ks"])  # every first-round item, at least
    xs, qs = O.znorm(env["raw"]), O.znorm(env["q"][1])
    want_ids, want_d = O.knn(xs, qs, k)
    got_ids, got_d = res[-1][0].cpu().numpy(), res[-1][1].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got_d - want_d) <= 1e-5 * want_d)
    for a, b in zip(*np.nonzero(got_ids != want_ids)):
        # a different id only where another row is (numerically) as close
        dg = np.sqrt(((xs[got_ids[a, b]].astype(np.float64) - qs[a]) ** 2).sum())
        assert abs(dg - want_d[a, b]) <= 1e-5 * want_d[a, b]
