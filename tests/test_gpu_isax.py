"""The iSAX (MESSI) backbone on the GPU, against the FP64 oracle.

The library builds the iSAX tree on the host and gives each leaf its SAX
intervals as the summary box; the lower bound, filters, scan and rounds are
the same kernels as for the DSTree-style tree.  Checked: partition, leaf
boxes and lower bounds equal the oracle's; exact search equals brute force;
and a filtered search over more than 10,000 leaves, each with a seeded
filter (so more than 10,000 filters are evaluated per batch), equals the
oracle's Algorithm 2 at the same schedule on sampled queries.
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
    print(f"[isax] {msg}", file=sys.stderr, flush=True)


def _check(ids, d, want_ids, want_d, xs, qs):
    """ids equal except near-ties (distinct per row), distances within 1e-4 relative."""
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


@pytest.fixture(scope="module")
def small():
    pkg = _pkg()
    raw = W.random_walk(20000, 64, seed=1301)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=100, n_segments=16, split_rule="isax")
    xs = O.znorm(raw)
    mu, _ = O.segment_stats(xs, 16)
    tree = O.build_isax_tree(mu, 64, 100)
    q = W.noisy_queries(raw, 64, (0.05, 0.3), 1302, 1303)[0]
    return dict(pkg=pkg, raw=raw, ix=ix, xs=xs, tree=tree, q=q)


def test_isax_partition_boxes_and_bounds_match_oracle(small):
    ix, tree = small["ix"], small["tree"]
    off, mem = ix.leaves()
    assert len(off) - 1 == len(tree.leaves)
    for L, want in enumerate(tree.leaves):
        assert np.array_equal(mem[off[L]:off[L + 1]], want)
    assert np.array_equal(ix.boxes(), O.isax_boxes(tree))
    lb = ix.lower_bounds(torch.from_numpy(small["q"]).cuda()).cpu().numpy()
    qs = O.znorm(small["q"])
    qmu, qsd = O.query_stats(qs, 16)
    want = O.lower_bound(qmu, qsd, O.isax_boxes(tree), 64)
    assert np.allclose(lb, want, rtol=1e-5, atol=1e-5)
    # the bound never exceeds the distance to the leaf's nearest member
    ld, _ = O.leaf_knn(small["xs"], tree.leaves, qs, 1)
    assert np.all(lb <= ld[:, :, 0] * (1 + 1e-5) + 1e-5)


@pytest.mark.parametrize("k,schedule", [(1, (1, 0)), (5, (1, 0)), (5, (1,))])
def test_isax_exact_search_matches_bruteforce(small, k, schedule):
    ix = small["ix"]
    ids, d, st = ix.search(torch.from_numpy(small["q"]).cuda(), k=k, use_filters=False, schedule=schedule,
                           with_stats=True)
    qs = O.znorm(small["q"])
    want_ids, want_d = O.knn(small["xs"], qs, k)
    _check(ids.cpu().numpy(), d.cpu().numpy().astype(np.float64), want_ids, want_d, small["xs"], qs)
    assert st["leaves_lb_pruned"] > 0


def test_isax_filtered_search_over_10k_filters_matches_oracle():
    """150,000 random walks of length 64 in an iSAX tree of capacity 100:
    more than 10,000 leaves (most of them root children), every leaf with a
    seeded filter (h = 32) and seeded offsets for (k = 5, target 0.99).  A
    batch of 256 queries; 24 sampled queries against the oracle's Algorithm 2
    at schedule (1, 0) with the oracle's own tree, bounds, visit order,
    per-leaf neighbours and FP64 filter outputs."""
    pkg = _pkg()
    m, h, k = 64, 32, 5
    raw = W.random_walk(150000, m, seed=1311)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=100, n_segments=16, split_rule="isax")
    N = ix.info()["n_leaves"]
    _say(f"{N} leaves")
    assert 10000 <= N <= 16384
    wts = W.mlp_weights(N, m, h, seed=1312, out_bias=4.0)
    offs = np.random.default_rng(1313).uniform(0.0, 3.0, size=N).astype(np.float32)
    ix.set_filters(np.arange(N, dtype=np.int32), torch.from_numpy(wts).cuda(), h)
    ix.set_offsets([k], [0.99], offs[None])
    q = W.noisy_queries(raw, 256, (0.05, 0.3), 1314, 1315)[0]
    ids, d, st = ix.search(torch.from_numpy(q).cuda(), k=k, target=0.99, use_filters=True, schedule=(1, 0),
                           with_stats=True)
    _say(f"filtered search stats {st}")
    assert st["filter_evals"] >= 10000 and st["leaves_filter_pruned"] > 0
    ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
    xs = O.znorm(raw)
    mu, _ = O.segment_stats(xs, 16)
    tree = O.build_isax_tree(mu, m, 100)
    off_, mem_ = ix.leaves()
    assert len(tree.leaves) == N
    for L in range(N):
        assert np.array_equal(mem_[off_[L]:off_[L + 1]], tree.leaves[L])
    rows = np.random.default_rng(1316).choice(len(q), 24, replace=False)
    qs = O.znorm(q[rows])
    qmu, qsd = O.query_stats(qs, 16)
    lb = O.lower_bound(qmu, qsd, O.isax_boxes(tree), m)
    ld, li = O.leaf_knn(xs, tree.leaves, qs, k)
    dF = np.stack([O.mlp_forward(wts[f], qs, m, h) for f in range(N)], 1) - offs[None].astype(np.float64)
    r = O.leafi_search(lb, O.visit_order(lb), ld, li, k, np.ones(N, dtype=bool), dF, (1, 0))
    assert r.f_pruned.sum() > 0
    _check(ids[rows], d[rows], r.ids, r.dist, xs, qs)
