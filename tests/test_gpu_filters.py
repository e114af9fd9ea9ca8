"""Parity of the learned-filter steps with the FP64 oracle, through the C ABI:
leaf selection (Algorithm 3) with a measured size threshold and a memory
budget that binds, the training targets the scan computes for every example
(Algorithm 1, node-wise nearest-neighbour distances of global queries on every
filtered leaf and of local queries on their own leaf), and filtered search on
the 64-query inference tiles (forced, and chosen by batch size) against the
oracle's Algorithm 2 at equal schedule."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import workloads as W

from test_gpu_parity import assert_knn_parity

pytestmark = pytest.mark.gpu


def _pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    return pkg


@pytest.fixture(scope="module")
def ragged():
    """30k Gaussian-mixture series of length 96, midpoint splits: ragged leaves."""
    pkg = _pkg()
    raw = W.gaussian_mixture(30000, 96, 40, 0.3, 41, 42)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=2000, n_segments=16, split_rule="midpoint")
    off, _ = ix.leaves()
    return dict(pkg=pkg, raw=raw, ix=ix, sizes=np.diff(off))


def test_selection_matches_oracle_with_measured_threshold_and_budget(ragged):
    ix, sizes = ragged["ix"], ragged["sizes"]
    m = h = 96
    w = (h * m + 2 * h + 1) * 4.0
    assert sizes.min() < sizes.max()
    # measured th (t^F and t^S timed on this GPU), budget for 3 filters
    rep = ix.train_filters(n_global=40, n_local=8, noise_lo=0.05, noise_hi=0.2, max_epochs=1, mem_budget=int(3 * w),
                           seed=5)
    th = rep["th"]
    assert th > 0 and rep["t_filter_s"] > 0 and rep["t_series_s"] > 0
    got, _ = ix.get_filters()
    want = O.select_leaves(sizes, th, w, 3 * w)
    assert list(got) == list(want), (th, sizes)
    # th at the median leaf size, budget for 5 filters: the budget binds
    th2 = float(np.median(sizes))
    assert (sizes >= th2).sum() > 5
    rep = ix.train_filters(n_global=40, n_local=8, noise_lo=0.05, noise_hi=0.2, max_epochs=1, th_override=th2,
                           mem_budget=int(5 * w) + 100, seed=5)
    got, _ = ix.get_filters()
    want = O.select_leaves(sizes, th2, w, 5 * w + 100)
    assert len(want) == 5 and list(got) == list(want)
    # a budget below one filter selects nothing; th = 0 with room for all selects every leaf
    rep = ix.train_filters(n_global=40, n_local=8, max_epochs=1, th_override=0.0, mem_budget=int(w) - 1, seed=5)
    assert rep["n_filters"] == 0
    rep = ix.train_filters(n_global=40, n_local=8, max_epochs=1, th_override=0.0, mem_budget=int(w * len(sizes)),
                           seed=5)
    got, _ = ix.get_filters()
    assert list(got) == list(O.select_leaves(sizes, 0.0, w, w * len(sizes)))


def test_training_targets_match_oracle_node_distances():
    """Every example target is d^L(query, leaf of the filter): global queries on
    every filtered leaf, local queries on their own leaf (20k random walks,
    32 leaves, 30 filters selected by a budget)."""
    pkg = _pkg()
    wl = W.WORKLOADS["rw20k"]
    raw = W.random_walk(wl["n"], wl["m"], wl["seed"])
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16)
    m = h = 256
    w = (h * m + 2 * h + 1) * 4.0
    n_g, n_l = 150, 40
    rep = ix.train_filters(n_global=n_g, n_local=n_l, noise_lo=0.05, noise_hi=0.2, max_epochs=2, th_override=0.0,
                           mem_budget=int(30 * w), seed=9, keep_examples=1)
    F = rep["n_filters"]
    assert F == 30
    leaves, _ = ix.get_filters()
    q, exq, y, n_train = ix.examples()
    q, y = q.cpu().numpy(), y.cpu().numpy().astype(np.float64)
    assert q.shape == (n_g + F * n_l, m) and exq.shape == y.shape == (F, n_g + n_l)
    n_gv = int(round(0.2 * n_g))
    assert n_train == n_g - n_gv + n_l
    for f in range(F):
        e = exq[f]
        # [global training | local (this filter's own queries) | global validation]
        assert list(e[: n_g - n_gv]) == list(range(n_g - n_gv))
        assert list(e[n_g - n_gv: n_train]) == list(range(n_g + f * n_l, n_g + (f + 1) * n_l))
        assert list(e[n_train:]) == list(range(n_g - n_gv, n_g))
    xs = O.znorm(raw)
    mu, sd = O.segment_stats(xs, 16)
    tree = O.build_tree(mu, sd, m, wl["capacity"], "median")
    qs = O.znorm(q)
    dL, _ = O.leaf_knn(xs, tree.leaves, qs, 1)
    want = np.stack([dL[exq[f], leaves[f], 0] for f in range(F)])
    assert np.all(np.abs(y - want) <= 1e-4 * np.maximum(want, 1e-6)), np.abs(y - want).max()
    # local queries are their own leaf's series plus noise: their d^L is small
    local = np.stack([want[f, n_g - n_gv: n_train] for f in range(F)])
    assert np.median(local) < np.median(want[:, : n_g - n_gv])


@pytest.fixture(scope="module")
def rw20k_filtered():
    """rw20k with seeded filters on every leaf and 3,000 noisier queries (enough
    (query, filter) pairs after the first round for the batch-size switch to the
    64-query tiles: at least one 32-query tile per compute unit)."""
    pkg = _pkg()
    wl = W.WORKLOADS["rw20k"]
    raw = W.random_walk(wl["n"], wl["m"], wl["seed"])
    q, _, _ = W.noisy_queries(raw, 3000, 0.3, 1012, 1013)
    xs, qs = O.znorm(raw), O.znorm(q)
    m = wl["m"]
    mu, sd = O.segment_stats(xs, 16)
    tree = O.build_tree(mu, sd, m, wl["capacity"], "median")
    N = len(tree.leaves)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16)
    h = 64
    wts = W.mlp_weights(N, m, h, seed=99, out_bias=6.0)
    offs = np.random.default_rng(5).uniform(0.0, 5.0, size=N).astype(np.float32)
    ix.set_filters(np.arange(N, dtype=np.int32), torch.from_numpy(wts).cuda(), h)
    ix.set_offsets([1], [0.9], offs[None])
    qmu, qsd = O.query_stats(qs, 16)
    lb = O.lower_bound(qmu, qsd, O.leaf_boxes(mu, sd, tree), m)
    ld, li = O.leaf_knn(xs, tree.leaves, qs, 1)
    df = np.stack([O.mlp_forward(wts[f], qs, m, h) for f in range(N)], 1)
    return dict(pkg=pkg, ix=ix, q=q, xs=xs, qs=qs, lb=lb, order=O.visit_order(lb), ld=ld, li=li,
                dF=df - offs[None].astype(np.float64), N=N)


def test_filter_tiles_forced_and_automatic_are_identical_and_match_oracle(rw20k_filtered):
    s = rw20k_filtered
    pkg, ix = s["pkg"], s["ix"]
    qt = torch.from_numpy(s["q"]).cuda()
    res = {}
    for name, flags in [("auto", 0), ("small", pkg.SEARCH_FILTER_TILE_SMALL), ("large", pkg.SEARCH_FILTER_TILE_LARGE),
                        ("large-host", pkg.SEARCH_FILTER_TILE_LARGE | pkg.SEARCH_HOST_ROUNDS)]:
        ids, d, st = ix.search(qt, k=1, target=0.9, use_filters=True, schedule=(1, 0), with_stats=True, flags=flags)
        res[name] = (ids.cpu().numpy(), d.cpu().numpy(), st)
    for name in ("small", "large", "large-host"):
        assert np.array_equal(res[name][0], res["auto"][0]) and np.array_equal(res[name][1], res["auto"][1]), name
        for key in ("leaves_scanned", "leaves_filter_pruned", "filter_evals"):
            assert res[name][2][key] == res["auto"][2][key], (name, key)
    st = res["auto"][2]
    # enough pairs for the automatic switch to the large tiles: at least one
    # 32-query tile per compute unit (sum of ceil(pairs / 32) >= 256)
    assert st["filter_evals"] >= 256 * 32, st
    r = O.leafi_search(s["lb"], s["order"], s["ld"], s["li"], 1, np.ones(s["N"], dtype=bool), s["dF"], (1, 0))
    assert r.f_pruned.sum() > 0
    assert_knn_parity(res["large"][0], res["large"][1], r.ids, r.dist, s["xs"], s["qs"])
    if not r.near_tie.any():
        assert st["leaves_filter_pruned"] == int(r.f_pruned.sum())
        assert st["leaves_scanned"] == int(r.scanned.sum())


def test_training_schedule_follows_the_plateau_rule_and_keeps_the_best_weights():
    """The learning-rate schedule (divide by 10 after `patience` epochs without a
    1e-4 relative validation improvement, stop below lr_min) re-simulated from
    the recorded validation losses stops at the recorded epoch for every
    filter; the kept weights are those of the best epoch: their validation MSE
    under the FP64 oracle's forward pass equals the smallest recorded loss.  The
    best loss at each learning-rate drop is non-increasing."""
    pkg = _pkg()
    wl = W.WORKLOADS["rw20k"]
    raw = W.random_walk(wl["n"], wl["m"], wl["seed"])
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16)
    m = h = 256
    w = (h * m + 2 * h + 1) * 4.0
    lr0, lr_min, patience = 0.01, 1e-4, 3
    rep = ix.train_filters(n_global=200, n_local=60, noise_lo=0.05, noise_hi=0.2, max_epochs=60, th_override=0.0,
                           mem_budget=int(12 * w), seed=21, keep_examples=1, lr0=lr0, lr_min=lr_min,
                           patience=patience)
    F = rep["n_filters"]
    assert F == 12
    epochs, trace = ix.train_trace()
    q, exq, y, n_train = ix.examples()
    leaves, wts = ix.get_filters()
    wts = wts.cpu().numpy().astype(np.float64)
    qs, y = O.znorm(q.cpu().numpy()), y.cpu().numpy().astype(np.float64)
    stops = 0
    for f in range(F):
        n = int(epochs[f])
        assert 1 <= n <= 60 and np.isfinite(trace[f, :n]).all() and np.isnan(trace[f, n:]).all()
        best, bad, lr, stop_at, drops = np.inf, 0, lr0, None, []
        for e in range(n):
            v = float(trace[f, e])
            if v < best * (1 - 1e-4):
                best, bad = v, 0
            else:
                bad += 1
                if bad >= patience:
                    lr *= 0.1
                    bad = 0
                    drops.append(best)
            if lr < lr_min * (1 - 1e-3):
                stop_at = e + 1
                break
        assert (stop_at or 60) == n, (f, stop_at, n)
        stops += stop_at is not None
        assert all(b2 <= b1 for b1, b2 in zip(drops, drops[1:]))
        # the kept weights: validation MSE in FP64 = the best recorded loss
        e_val = exq[f, n_train:]
        pred = O.mlp_forward(wts[f], qs[e_val], m, h)
        mse = float(np.mean((pred - y[f, n_train:]) ** 2))
        assert abs(mse - np.nanmin(trace[f])) <= 2e-3 * np.nanmin(trace[f]), (f, mse, np.nanmin(trace[f]))
    assert stops > 0  # the stopping rule was reached by some filter
