"""Parity at the two larger configurations, on outputs the FP64 oracle can
compute one query at a time.

* 10,000,000 random walks of length 256 (precision case): batches of 1,024
  queries, k = 10, BF16 scan with FP32 rerank; per-query error against FP64
  brute force over all 10M series; filtered search with seeded filters
  against the oracle's Algorithm 2 at equal schedule.
* 25,000,000 Gaussian-mixture series of length 96 split at range midpoints
  (ragged leaves): 4,096 queries with k = 1, 10, 50 in one batch; filters
  with infinite offsets give the exact results.

At both sizes the buffers sized for a batch's worst case would exceed the
planned-sequence limit, so batches run as capacity-checked planned sequences
(statistics path 1 to 3): each round's item count is checked on the device,
and a round that overflows its buffers sends the batch to host-driven rounds
(path 4: forced at 10M by a small capacity; at 25M the exact search's second
round of 14M items overflows the planned buffers of the default limit, and
the next batches of that shape are planned for the size the rerun met, then
captured and replayed).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    return pkg


def _say(msg):
    print(f"[large] {msg}", file=sys.stderr, flush=True)


def _check(ids, d, want_ids, want_d, xs, qs):
    """ids equal except near-ties, distances within 1e-4 relative; returns the
    largest relative distance error per query."""
    fin = np.isfinite(want_d)
    assert np.array_equal(np.isfinite(d), fin)
    rel = np.where(fin, np.abs(d - want_d) / np.maximum(want_d, 1e-6), 0.0)
    assert rel.max() <= 1e-4, rel.max()
    for row, f in zip(ids, fin):
        assert len(np.unique(row[f])) == int(f.sum())
    for a, b in zip(*np.nonzero((ids != want_ids) & fin)):
        x = xs[ids[a, b]].astype(np.float64)
        dg = np.sqrt(((x - qs[a].astype(np.float64)) ** 2).sum())
        assert abs(dg - want_d[a, b]) <= 3e-5 * want_d[a, b], (a, b)
    return rel.max(axis=1)


def test_precision_10m_k10_exact_and_filtered():
    """10M random walks, batches of 1,024 queries at k = 10.  Exact search: 16
    sampled queries against FP64 brute force over all 10M series, per-query
    maximum relative distance error printed; the default execution (a
    capacity-checked planned sequence, then its captured graph), host-driven
    rounds and a planned sequence forced to overflow (path 4) give identical
    results.  Filtered search with seeded filters on every leaf:
    the same 16 queries against the oracle's Algorithm 2 at the same schedule
    (the oracle's own tree, bounds, visit order, per-leaf neighbours and FP64
    filter outputs)."""
    pkg = _pkg()
    wl = W.WORKLOADS["rw10m"]
    raw = W.random_walk(wl["n"], wl["m"], wl["seed"])
    _say("generated 10M x 256")
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16)
    torch.cuda.synchronize()
    N = ix.info()["n_leaves"]
    _say(f"built {N} leaves")
    parts = [W.noisy_queries(raw, n, s, wl["test_seed"] + i, wl["test_seed"] + 100 + i)[0]
             for i, (n, s) in enumerate(zip((342, 341, 341), wl["sigmas"]))]
    q = np.concatenate(parts)
    qd = torch.from_numpy(q).cuda()
    out = (torch.empty((len(q), 10), dtype=torch.int64, device="cuda"),
           torch.empty((len(q), 10), dtype=torch.float32, device="cuda"))
    # k and target in fixed device buffers: a graph is replayed only for the
    # buffer addresses it was captured with
    kd = torch.full((len(q),), 10, dtype=torch.int32, device="cuda")
    td = torch.ones(len(q), dtype=torch.float32, device="cuda")
    res = []
    for flags, cap, want in ((0, 0, 1), (0, 0, 3), (0, 0, 2), (pkg.SEARCH_HOST_ROUNDS, 0, 0),
                             (pkg.SEARCH_NO_GRAPH, len(q) + 1, 4)):
        ix.set_plan_capacity(cap)
        ids, d, st = ix.search(qd, k=kd, target=td, k_max=10, use_filters=False, schedule=(1, 0), with_stats=True,
                               out=out, flags=flags)
        res.append((ids.clone(), d.clone(), st))
        assert st["path"] == want, (want, st, ix.graph_note())
    ix.set_plan_capacity(0)
    for r in res[1:]:
        assert torch.equal(res[0][0], r[0]) and torch.equal(res[0][1], r[1])
        for c in ("leaves_scanned", "series_scanned", "fallback_items", "rounds", "scan_bytes"):
            assert r[2][c] == res[0][2][c], c
    st = res[0][2]
    _say(f"exact search stats {st}")
    assert st["fallback_items"] <= 0.02 * st["leaves_scanned"] + 1
    ids, d = res[0][0].cpu().numpy(), res[0][1].cpu().numpy().astype(np.float64)
    # filtered search: seeded filters on every leaf, seeded offsets for (k = 10, target 0.99)
    h = 64
    wts = W.mlp_weights(N, wl["m"], h, seed=3101, out_bias=8.0)
    offs = np.random.default_rng(3102).uniform(0.0, 6.0, size=N).astype(np.float32)
    ix.set_filters(np.arange(N, dtype=np.int32), torch.from_numpy(wts).cuda(), h)
    ix.set_offsets([10], [0.99], offs[None])
    fids, fd, fst = ix.search(qd, k=10, target=0.99, use_filters=True, schedule=(1, 0), with_stats=True)
    _say(f"filtered search stats {fst}")
    assert fst["leaves_filter_pruned"] > 0
    fids, fd = fids.cpu().numpy(), fd.cpu().numpy().astype(np.float64)
    xs = O.znorm(raw)
    del raw
    rows = np.random.default_rng(11).choice(len(q), 16, replace=False)
    qs = O.znorm(q[rows])
    want_ids, want_d = O.knn(xs, qs, 10)
    err = _check(ids[rows], d[rows], want_ids, want_d, xs, qs)
    _say(f"per-query max relative distance error vs FP64: {np.array2string(err, precision=2)}")
    # the oracle's Algorithm 2 with the same filters, at the same schedule
    mu, sd = O.segment_stats(xs, 16)
    tree = O.build_tree(mu, sd, wl["m"], wl["capacity"], "median")
    off_, mem_ = ix.leaves()
    assert len(tree.leaves) == N
    for L in range(N):
        assert np.array_equal(mem_[off_[L]:off_[L + 1]], tree.leaves[L])
    qmu, qsd = O.query_stats(qs, 16)
    lb = O.lower_bound(qmu, qsd, O.leaf_boxes(mu, sd, tree), wl["m"])
    ld, li = O.leaf_knn(xs, tree.leaves, qs, 10)
    dF = np.stack([O.mlp_forward(wts[f], qs, wl["m"], h) for f in range(N)], 1) - offs[None].astype(np.float64)
    r = O.leafi_search(lb, O.visit_order(lb), ld, li, 10, np.ones(N, dtype=bool), dF, (1, 0))
    assert r.f_pruned.sum() > 0
    _check(fids[rows], fd[rows], r.ids, r.dist, xs, qs)


def test_ragged_25m_k_mix():
    pkg = _pkg()
    wl = W.WORKLOADS["gm25m"]
    raw = W.gaussian_mixture(wl["n"], wl["m"], wl["n_comp"], wl["spread"], wl["seed_means"], wl["seed_members"])
    _say("generated 25M x 96")
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16,
                           split_rule="midpoint")
    torch.cuda.synchronize()
    off, _ = ix.leaves()
    sizes = np.diff(off)
    _say(f"built {len(sizes)} leaves, sizes {sizes.min()} .. {sizes.max()}")
    assert sizes.max() <= wl["capacity"] and sizes.min() < wl["capacity"] // 4  # ragged
    q, _, _ = W.noisy_queries(raw, wl["nq"], wl["sigma"], wl["q_seed"], wl["q_seed"] + 100)
    ks = np.array([wl["ks"][i % 3] for i in range(wl["nq"])], dtype=np.int32)
    qd, kd = torch.from_numpy(q).cuda(), torch.from_numpy(ks).cuda()
    td = torch.ones(len(q), dtype=torch.float32, device="cuda")
    out = (torch.empty((len(q), 50), dtype=torch.int64, device="cuda"),
           torch.empty((len(q), 50), dtype=torch.float32, device="cuda"))
    # The second round holds 14M items, more than the planned buffers of the
    # 16 GiB limit: the first planned batch overflows and runs again with
    # host-driven rounds (path 4), which record the round's size; the next
    # batch of that shape is planned for it (path 1), then captured (3) and
    # replayed (2), all with the same results.
    res = []
    for want in (4, 1, 3, 2):
        i_, d_, st = ix.search(qd, k=kd, target=td, k_max=50, use_filters=False, schedule=(1, 0), with_stats=True,
                               out=out)
        _say(f"search stats {st}")
        assert st["path"] == want, (want, st, ix.graph_note())
        res.append((i_.clone(), d_.clone(), st))
    for r in res[1:]:
        assert torch.equal(r[0], res[0][0]) and torch.equal(r[1], res[0][1])
        for c in ("leaves_scanned", "series_scanned", "fallback_items", "rounds", "scan_bytes"):
            assert r[2][c] == res[0][2][c], c
    ids, d, st = res[0]
    assert st["fallback_items"] <= 0.02 * st["leaves_scanned"] + 1
    # seeded filters on every leaf: with infinite offsets they never prune and
    # the results are the exact ones; finite offsets prune
    N = len(sizes)
    wts = W.mlp_weights(N, wl["m"], 32, seed=4101, out_bias=8.0)
    ix.set_filters(np.arange(N, dtype=np.int32), torch.from_numpy(wts).cuda(), 32)
    ix.set_offsets([1, 10, 50], [0.99], np.full((3, N), np.inf, dtype=np.float32))
    i2, d2, st2 = ix.search(qd, k=kd, target=0.99, k_max=50, use_filters=True, schedule=(1, 0), with_stats=True)
    assert st2["leaves_filter_pruned"] == 0 and st2["filter_evals"] > 0
    assert torch.equal(i2, ids) and torch.equal(d2, d)
    ix.set_offsets([1, 10, 50], [0.99], np.zeros((3, N), dtype=np.float32))
    i3, d3, st3 = ix.search(qd, k=kd, target=0.99, k_max=50, use_filters=True, schedule=(1, 0), with_stats=True)
    _say(f"filtered search stats {st3}")
    assert st3["leaves_filter_pruned"] > 0
    ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
    d3 = d3.cpu().numpy().astype(np.float64)
    kk = ks[:, None] > np.arange(50)
    assert np.all(d3[kk] >= d[kk] * (1 - 1e-6))  # a filtered search can only miss neighbours
    xs = O.znorm(raw)
    del raw
    rows = np.random.default_rng(12).choice(len(q), 24, replace=False)
    qs = O.znorm(q[rows])
    want_ids, want_d = O.knn(xs, qs, 50)
    for k in wl["ks"]:
        sel = ks[rows] == k
        if sel.any():
            _check(ids[rows][sel, :k], d[rows][sel, :k], want_ids[sel, :k], want_d[sel, :k], xs, qs[sel])
            assert (ids[rows][sel, k:] == -1).all()
