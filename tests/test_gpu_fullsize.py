"""Parity at the benchmark's full size (1,000,000 random walks of length 256,
leaf capacity 10,000), in the launch configuration bench.py times, on outputs
the oracle can compute one query at a time."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw1m():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    wl = W.WORKLOADS["rw1m"]
    raw = W.random_walk(wl["n"], wl["m"], wl["seed"])
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16)
    xs = O.znorm(raw)
    q = []
    for s, sd in zip(wl["sigmas"], wl["test_seeds"]):
        q.append(W.noisy_queries(raw, wl["nq"], s, sd, sd + 100)[0])
    q = np.concatenate(q)
    mu, sd = O.segment_stats(xs, 16)
    tree = O.build_tree(mu, sd, 256, wl["capacity"], "median")
    return dict(pkg=pkg, raw=raw, xs=xs, ix=ix, q=q, wl=wl, tree=tree)


def test_full_size_tree_partition(rw1m):
    t = rw1m["tree"]
    off, mem = rw1m["ix"].leaves()
    assert len(off) - 1 == len(t.leaves) == 128
    for L, want in enumerate(t.leaves):
        assert np.array_equal(mem[off[L]:off[L + 1]], want)


def test_full_size_exact_search_sampled(rw1m):
    """The bench's batch of 1,000 queries (schedule (1, 0), BF16 scan); 24
    sampled rows checked against FP64 brute force over all 1M series."""
    ix, q = rw1m["ix"], rw1m["q"]
    batch = q[1000:2000]
    ids, d, st = ix.search(torch.from_numpy(batch).cuda(), k=10, use_filters=False, schedule=(1, 0),
                           with_stats=True)
    ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(7).choice(1000, 24, replace=False)
    qs = O.znorm(batch[rows])
    want_ids, want_d = O.knn(rw1m["xs"], qs, 10)
    assert np.all(np.abs(d[rows] - want_d) <= 1e-4 * want_d)
    for row in ids[rows]:
        assert len(np.unique(row)) == len(row)
    for a, b in zip(*np.nonzero(ids[rows] != want_ids)):
        x = rw1m["xs"][ids[rows][a, b]].astype(np.float64)
        dg = np.sqrt(((x - qs[a]) ** 2).sum())
        assert abs(dg - want_d[a, b]) <= 3e-5 * want_d[a, b]
    # the certificate spares nearly every item an exact rescan
    assert st["fallback_items"] <= 0.02 * st["leaves_scanned"] + 1


def test_full_size_leaf_nn_sampled(rw1m):
    """d^L of 8 queries against every leaf (the training-target computation)."""
    ix, q = rw1m["ix"], rw1m["q"]
    sub = q[::375][:8]
    d, ids = ix.leaf_knn(torch.from_numpy(sub).cuda(), 1)
    d, ids = d.cpu().numpy()[:, :, 0].astype(np.float64), ids.cpu().numpy()[:, :, 0]
    wd, wi = O.leaf_knn(rw1m["xs"], rw1m["tree"].leaves, O.znorm(sub), 1)
    assert np.all(np.abs(d - wd[:, :, 0]) <= 1e-4 * wd[:, :, 0])
    # ids equal except near-ties: a different id must be exactly as close in FP64
    qs = O.znorm(sub)
    for a, L in zip(*np.nonzero(ids != wi[:, :, 0])):
        x = rw1m["xs"][ids[a, L]].astype(np.float64)
        dg = np.sqrt(((x - qs[a]) ** 2).sum())
        assert abs(dg - wd[a, L, 0]) <= 3e-5 * wd[a, L, 0], (a, L, dg, wd[a, L, 0])
