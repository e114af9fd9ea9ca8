"""Serving engine (continuous batching): results do not depend on the mix.

A trace of requests with mixed k and recall targets arrives while others are
on the GPU.  Each result must be bitwise identical to the same query searched
alone (and to the batched search at the same schedule), and must match the
FP64 oracle's Algorithm 2 at that schedule up to near-ties.
"""
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


@pytest.fixture(scope="module")
def served():
    pkg = _pkg()
    raw = W.random_walk(20000, 128, seed=501)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=700, n_segments=16)
    N = ix.info()["n_leaves"]
    h = 32
    w = W.mlp_weights(N, 128, h, seed=502, out_bias=4.0)
    offs = np.random.default_rng(503).uniform(0.0, 3.5, N).astype(np.float32)
    ix.set_filters(np.arange(N, dtype=np.int32), torch.from_numpy(w).cuda(), h)
    ix.set_offsets([1, 5], [0.9], np.stack([offs, offs]))
    n = 160
    q, _, _ = W.noisy_queries(raw, n, (0.05, 0.3), 504, 505)
    rng = np.random.default_rng(506)
    ks = rng.choice([1, 5], n).astype(np.int32)
    targets = rng.choice([0.9, 1.0], n).astype(np.float32)
    arrivals = np.cumsum(rng.exponential(1.0 / 20000.0, n))  # 20k requests/s
    return dict(pkg=pkg, raw=raw, ix=ix, w=w, h=h, offs=offs, q=q, ks=ks, targets=targets, arrivals=arrivals, N=N)


def test_mix_equals_batched_search_and_alone(served):
    s = served
    pkg, ix = s["pkg"], s["ix"]
    # batched search of the same requests (no server running on the index)
    qd = torch.from_numpy(s["q"]).cuda()
    b_ids, b_d = ix.search(qd, k=torch.from_numpy(s["ks"]).cuda(), target=torch.from_numpy(s["targets"]).cuda(),
                           k_max=5, schedule=(1, 0))
    b_ids, b_d = b_ids.cpu().numpy(), b_d.cpu().numpy()
    sv = pkg.Server(ix, k_max=5, max_slots=48, schedule=(1, 0))
    try:
        ids, d, lat, rep = sv.replay(s["q"], s["arrivals"], s["ks"], s["targets"])
        assert rep["completed"] == len(s["q"])
        assert rep["max_active"] > 1            # requests really overlapped on the GPU
        assert np.array_equal(ids, b_ids)
        assert np.array_equal(d, b_d)
        assert np.all(lat > 0)
        # the same requests one at a time on an idle server
        for i in range(0, len(s["q"]), 8):
            t = sv.submit(s["q"][i], int(s["ks"][i]), float(s["targets"][i]))
            while (res := sv.poll(t)) is None:
                pass
            a_ids, a_d, _ = res
            assert np.array_equal(a_ids, ids[i]) and np.array_equal(a_d, d[i])
    finally:
        sv.close()


def test_mix_matches_oracle_at_equal_schedule(served):
    s = served
    pkg, ix = s["pkg"], s["ix"]
    sv = pkg.Server(ix, k_max=5, max_slots=32, schedule=(1, 0))
    try:
        ids, d, lat, rep = sv.replay(s["q"], s["arrivals"], s["ks"], s["targets"])
    finally:
        sv.close()
    xs, qs = O.znorm(s["raw"]), O.znorm(s["q"])
    mu, sd = O.segment_stats(xs, 16)
    t = O.build_tree(mu, sd, 128, 700, "median")
    lb = O.lower_bound(*O.query_stats(qs, 16), O.leaf_boxes(mu, sd, t), 128)
    order = O.visit_order(lb)
    ld, li = O.leaf_knn(xs, t.leaves, qs, 5)
    df = np.stack([O.mlp_forward(s["w"][f], qs, 128, s["h"]) for f in range(s["N"])], 1)
    has = np.ones(s["N"], dtype=bool)
    for k in (1, 5):
        for tgt in (0.9, 1.0):
            sel = np.nonzero((s["ks"] == k) & (s["targets"] == tgt))[0]
            if len(sel) == 0:
                continue
            offs = s["offs"] if tgt < 1.0 else np.full(s["N"], np.inf)
            r = O.leafi_search(lb[sel], order[sel], ld[sel], li[sel], k, has, df[sel] - offs[None], (1, 0))
            got_ids, got_d = ids[sel, :k], d[sel, :k].astype(np.float64)
            fin = np.isfinite(r.dist)
            assert np.all(np.abs(got_d[fin] - r.dist[fin]) <= 1e-4 * r.dist[fin])
            for a, b in zip(*np.nonzero(got_ids != r.ids)):
                x = xs[got_ids[a, b]].astype(np.float64)
                dg = np.sqrt(((x - qs[sel[a]]) ** 2).sum())
                assert abs(dg - r.dist[a, b]) <= 3e-5 * r.dist[a, b]
            assert (ids[sel, k:] == -1).all()


def test_admission_under_tiny_memory_budget(served):
    s = served
    pkg, ix = s["pkg"], s["ix"]
    with pytest.raises(pkg.LeafiError, match="admits no query"):
        pkg.Server(ix, k_max=5, max_slots=0, mem_budget=1000)
    # slots = floor(budget / per-slot bytes): linear in the budget
    big = pkg.Server(ix, k_max=5, max_slots=0, mem_budget=300_000)
    s_big = big.slots
    big.close()
    sv = pkg.Server(ix, k_max=5, max_slots=0, mem_budget=30_000)
    try:
        assert 1 <= sv.slots <= 8
        assert 10 * sv.slots <= s_big <= 10 * (sv.slots + 1)
        n = 40
        ids, d, lat, rep = sv.replay(s["q"][:n], s["arrivals"][:n] * 0.0, s["ks"][:n], s["targets"][:n])
        assert rep["completed"] == n and rep["max_active"] <= sv.slots
    finally:
        sv.close()
    # results under the small budget equal the unconstrained batch
    b_ids, b_d = ix.search(torch.from_numpy(s["q"][:n]).cuda(), k=torch.from_numpy(s["ks"][:n]).cuda(),
                           target=torch.from_numpy(s["targets"][:n]).cuda(), k_max=5, schedule=(1, 0))
    assert np.array_equal(ids, b_ids.cpu().numpy()) and np.array_equal(d, b_d.cpu().numpy())
