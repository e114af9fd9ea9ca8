"""Pins for the FP64 oracle: each test checks it against something other than
itself (closed forms, textbook routines, brute force, hand-computed cases,
invariants the paper's definitions imply)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


# ---------------------------------------------------------------- z-normalisation

def test_znorm_closed_forms():
    x = W.random_walk(300, 128, seed=11)
    z = O.znorm(x).astype(np.float64)
    # mean 0 and squared norm m (population std); fp32 storage bounds the error
    assert np.abs(z.mean(axis=1)).max() < 1e-6
    assert np.abs((z ** 2).sum(axis=1) / 128 - 1.0).max() < 1e-6
    # affine invariance: z(a x + b) == z(x) for a > 0
    z2 = O.znorm((3.0 * x.astype(np.float64) + 7.0).astype(np.float32)).astype(np.float64)
    assert np.abs(z2 - z).max() < 1e-5


def test_znorm_constant_series_and_c_matches_numpy():
    x = W.random_walk(50, 64, seed=12)
    x[3] = 5.0
    x[7] = 0.0
    z = O.znorm(x)
    assert not z[3].any() and not z[7].any()
    assert np.array_equal(z, O.znorm_py(x))


# ---------------------------------------------------------------- distances and k-NN

def _direct(data_s, q_s):
    return np.sqrt(((q_s[:, None, :].astype(np.float64) - data_s[None].astype(np.float64)) ** 2).sum(-1))


def test_distance_expansion_identity():
    x = O.znorm(W.random_walk(400, 96, seed=13))
    q = O.znorm(W.noisy_queries(W.random_walk(400, 96, seed=13), 20, 0.2, 1, 2)[0])
    ids, d = O.knn(x, q, 400)
    x64, q64 = x.astype(np.float64), q.astype(np.float64)
    # ||q||^2 + ||x||^2 - 2 q.x, a different route to the same squared distance
    d2 = (q64 ** 2).sum(1)[:, None] + (x64 ** 2).sum(1)[None] - 2 * q64 @ x64.T
    got = np.take_along_axis(d2, ids, axis=1)
    assert np.allclose(d ** 2, got, rtol=1e-9, atol=1e-9)
    # z-normalised inputs: d^2 = 2m - 2 q.x up to the fp32 storage of ||x||^2 = m
    approx = 2 * 96 - 2 * np.take_along_axis(q64 @ x64.T, ids, axis=1)
    assert np.abs(d ** 2 - approx).max() < 1e-3


def test_knn_matches_stable_argsort_with_planted_ties():
    x = W.random_walk(1500, 32, seed=14)
    x[900] = x[100]          # exact duplicates: equal distances, smaller id first
    x[1400] = x[100]
    x[50] = x[1200]
    xs = O.znorm(x)
    q = xs[[100, 1200, 7, 300]].copy()
    q[2] += np.float32(0.01)
    ids, d = O.knn(xs, q, 10)
    ref = _direct(xs, q)
    want = np.argsort(ref, axis=1, kind="stable")[:, :10]
    assert np.array_equal(ids, want)
    assert np.allclose(d, np.take_along_axis(ref, want, axis=1), rtol=1e-12)
    assert list(ids[0, :3]) == [100, 900, 1400] and d[0, 0] == 0.0
    assert list(ids[1, :2]) == [50, 1200]


def test_knn_stream_equals_knn_over_the_whole_collection():
    """Chunked brute force (for collections too large for the host) = brute force
    over everything, including ties split across chunks and short chunks."""
    raw = W.random_walk(2300, 32, seed=17)
    raw[1500] = raw[40] * 3.0 + 2.0     # exact tie (same z-normalised series) in another chunk
    raw[2299] = raw[41]
    q, _, _ = W.noisy_queries(raw, 25, 0.2, 18, 19)
    q[0] = raw[40]
    qs = O.znorm(q)
    want_i, want_d = O.knn(O.znorm(raw), qs, 9)
    chunks = [(lo, raw[lo:lo + 700]) for lo in range(0, len(raw), 700)]  # last chunk 200 rows
    got_i, got_d = O.knn_stream(chunks, qs, 9)
    assert np.array_equal(got_i, want_i) and np.array_equal(got_d, want_d)
    assert list(got_i[0, :2]) == [40, 1500]
    # chunks shorter than k
    got_i, got_d = O.knn_stream([(lo, raw[lo:lo + 5]) for lo in range(0, 40, 5)], qs, 9)
    w_i, w_d = O.knn(O.znorm(raw[:40]), qs, 9)
    assert np.array_equal(got_i, w_i) and np.array_equal(got_d, w_d)


def test_knn_fewer_series_than_k():
    xs = O.znorm(W.random_walk(5, 16, seed=15))
    ids, d = O.knn(xs, xs[:2], 8)
    assert (ids[:, 5:] == -1).all() and np.isinf(d[:, 5:]).all()
    assert sorted(ids[0, :5]) == [0, 1, 2, 3, 4]


def test_leaf_knn_is_restricted_bruteforce():
    xs = O.znorm(W.random_walk(900, 48, seed=16))
    q = O.znorm(W.noisy_queries(W.random_walk(900, 48, seed=16), 7, 0.3, 3, 4)[0])
    rng = np.random.default_rng(0)
    perm = rng.permutation(900)
    leaves = [np.sort(perm[:100]), np.sort(perm[100:650]), np.sort(perm[650:])]
    d, ids = O.leaf_knn(xs, leaves, q, 4)
    full = _direct(xs, q)
    for L, mem in enumerate(leaves):
        sub = full[:, mem]
        o = np.argsort(sub, axis=1, kind="stable")[:, :4]
        assert np.array_equal(ids[:, L], mem[o])
        assert np.allclose(d[:, L], np.take_along_axis(sub, o, axis=1), rtol=1e-12)


# ---------------------------------------------------------------- tree and lower bounds

def test_median_tree_sizes_and_partition():
    xs = O.znorm(W.random_walk(20000, 256, seed=1001))
    mu, sd = O.segment_stats(xs, 16)
    t = O.build_tree(mu, sd, 256, 1000, "median")
    sizes = [len(l) for l in t.leaves]
    assert sizes == [625] * 32            # 20000 halves exactly five times
    allm = np.sort(np.concatenate(t.leaves))
    assert np.array_equal(allm, np.arange(20000))
    for l in t.leaves:
        assert np.all(np.diff(l) > 0)


def test_tree_split_choice_hand_case():
    # m = 4, S = 2: segment means/stds chosen by hand.  Member stats
    # (seg0 mu, seg1 mu) = (0,0) (0,3) (0,1) (0,2): segment 1's mean has the
    # largest range, so the median split sends ids {0, 2} (values 0, 1) left.
    mu = np.array([[0, 0], [0, 3], [0, 1], [0, 2]], dtype=np.float32)
    sd = np.array([[1, 1], [1, 1], [1, 1], [1, 1]], dtype=np.float32)
    t = O.build_tree(mu, sd, 4, 2, "median")
    assert [list(l) for l in t.leaves] == [[0, 2], [1, 3]]
    assert t.root.split[:2] == (1, 0)
    # now a std range wins: sd of segment 0 spans 0..2 (score 2*4 = 8) while
    # mu of segment 1 spans 0..1.5 (score 2*2.25 = 4.5)
    mu2 = np.array([[0, 0], [0, 1.5], [0, 1], [0, 0.5]], dtype=np.float32)
    sd2 = np.array([[2, 1], [0, 1], [1, 1], [0.5, 1]], dtype=np.float32)
    t2 = O.build_tree(mu2, sd2, 4, 2, "median")
    assert t2.root.split[:2] == (0, 1)
    assert [list(l) for l in t2.leaves] == [[1, 3], [0, 2]]
    # midpoint rule: values 0, 0.1, 0.2, 10 split at 5 -> 3 left, 1 right
    mu3 = np.array([[0, 0], [0, 0.1], [0, 0.2], [0, 10]], dtype=np.float32)
    t3 = O.build_tree(mu3, sd, 4, 3, "midpoint")
    assert [list(l) for l in t3.leaves] == [[0, 1, 2], [3]]


def _piecewise_constant(vals, seglen):
    return np.repeat(np.asarray(vals, dtype=np.float32), seglen, axis=-1)


def test_lower_bound_is_exact_for_piecewise_constant_single_member():
    # For piecewise-constant series the within-segment deviations vanish, so
    # d^2 = sum_s l_s (mu_q - mu_x)^2 and the bound is tight (up to the one-ulp
    # widening of the stored box).
    S, l = 4, 5
    x = _piecewise_constant([[0.3, -1.0, 2.0, 0.5]], l)
    q = _piecewise_constant([[1.0, 0.0, -0.5, 0.25]], l)
    mu, sd = O.segment_stats(x, S)
    box = O.node_box(mu, sd, np.array([0]))[None]
    qmu, qsd = O.query_stats(q, S)
    lb = O.lower_bound(qmu, qsd, box, S * l)[0, 0]
    d = math.sqrt(((q.astype(np.float64) - x) ** 2).sum())
    assert lb <= d
    assert abs(lb - d) < 1e-5 * d
    assert abs(d - math.sqrt(5 * (0.7 ** 2 + 1.0 + 2.5 ** 2 + 0.25 ** 2))) < 1e-6


def test_lower_bound_hand_box():
    # one segment of length 4 with box mu in [0, 1], sd in [2, 3]; query mu 1.5, sd 1
    box = np.array([[[0.0, 1.0, 2.0, 3.0]]], dtype=np.float32)
    lb = O.lower_bound(np.array([[1.5]]), np.array([[1.0]]), box, 4)
    assert abs(lb[0, 0] - math.sqrt(4 * (0.25 + 1.0))) < 1e-12
    lb_in = O.lower_bound(np.array([[0.5]]), np.array([[2.5]]), box, 4)
    assert lb_in[0, 0] == 0.0


@pytest.mark.parametrize("rule", ["median", "midpoint"])
def test_lower_bound_never_exceeds_node_distance(rule):
    raw = W.random_walk(3000, 64, seed=21) if rule == "median" else W.gaussian_mixture(3000, 64, 20, 0.3, 5, 6)
    xs = O.znorm(raw)
    mu, sd = O.segment_stats(xs, 8)
    t = O.build_tree(mu, sd, 64, 200, rule)
    qraw = np.concatenate([W.noisy_queries(raw, 20, 0.1, 1, 2)[0], W.random_walk(10, 64, seed=99)])
    q = O.znorm(qraw)
    boxes = O.leaf_boxes(mu, sd, t)
    qmu, qsd = O.query_stats(q, 8)
    lb = O.lower_bound(qmu, qsd, boxes, 64)
    d, _ = O.leaf_knn(xs, t.leaves, q, 1)
    assert np.all(lb <= d[:, :, 0] * (1 + 1e-12))
    assert (lb > 0).mean() > 0.3          # the bound is not trivially zero
    # parent bound <= child bound
    def walk(node):
        if node.left is None:
            return
        bp = O.lower_bound(qmu, qsd, O.node_box(mu, sd, node.members)[None], 64)
        for ch in (node.left, node.right):
            bc = O.lower_bound(qmu, qsd, O.node_box(mu, sd, ch.members)[None], 64)
            assert np.all(bp <= bc + 1e-12)
            walk(ch)
    walk(t.root)


def test_visit_order_ties_by_leaf_id():
    lb = np.array([[0.5, 0.1, 0.5, 0.0, 0.1]])
    assert list(O.visit_order(lb)[0]) == [3, 1, 4, 0, 2]


# ---------------------------------------------------------------- MLP filter

def test_mlp_identity_special_case():
    m = h = 8
    w = np.zeros(m * h + 2 * h + 1)
    w[: m * h] = np.eye(m).reshape(-1)
    w[m * h + h: m * h + 2 * h] = 1.0
    q = np.random.default_rng(3).standard_normal((5, m)).astype(np.float32)
    got = O.mlp_forward(w, q, m, h)
    assert np.allclose(got, np.maximum(q.astype(np.float64), 0).sum(1), rtol=1e-15)


def test_mlp_matches_explicit_loops_and_layout():
    m, h = 5, 3
    w = W.mlp_weights(1, m, h, seed=4)[0].astype(np.float64)
    q = np.random.default_rng(5).standard_normal((4, m))
    out = O.mlp_forward(w, q, m, h)
    for r in range(4):
        acc = w[m * h + 2 * h]
        for j in range(h):
            z = w[m * h + j]
            for i in range(m):
                z += w[i * h + j] * q[r, i]       # input-major W1
            acc += w[m * h + h + j] * max(z, 0.0)
        assert abs(acc - out[r]) < 1e-12


def test_mlp_gradient_central_differences():
    m = h = 4
    w = W.mlp_weights(1, m, h, seed=8)[0].astype(np.float64)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((6, m))
    y = rng.uniform(1, 3, 6)
    loss, g = O.mlp_mse_grad(w, X, y, m, h)
    eps = 1e-6
    for p in range(len(w)):
        wp, wm = w.copy(), w.copy()
        wp[p] += eps
        wm[p] -= eps
        fd = (O.mlp_mse_grad(wp, X, y, m, h)[0] - O.mlp_mse_grad(wm, X, y, m, h)[0]) / (2 * eps)
        assert abs(fd - g[p]) < 1e-6 * max(1.0, abs(fd))
    assert abs(loss - ((O.mlp_forward(w, X, m, h) - y) ** 2).mean()) < 1e-12


# ---------------------------------------------------------------- search (Algorithm 2)

@pytest.fixture(scope="module")
def small_index():
    raw = W.random_walk(6000, 64, seed=31)
    xs = O.znorm(raw)
    mu, sd = O.segment_stats(xs, 8)
    t = O.build_tree(mu, sd, 64, 400, "median")
    q = O.znorm(W.noisy_queries(raw, 40, (0.05, 0.3), 7, 8)[0])
    qmu, qsd = O.query_stats(q, 8)
    lb = O.lower_bound(qmu, qsd, O.leaf_boxes(mu, sd, t), 64)
    order = O.visit_order(lb)
    kmax = 5
    ld, li = O.leaf_knn(xs, t.leaves, q, kmax)
    return dict(xs=xs, t=t, q=q, lb=lb, order=order, ld=ld, li=li, kmax=kmax)


@pytest.mark.parametrize("schedule", [(1,), (2,), (1, 0), (0,), (1, 3)])
@pytest.mark.parametrize("k", [1, 5])
def test_plain_tree_search_is_exact(small_index, schedule, k):
    s = small_index
    r = O.leafi_search(s["lb"], s["order"], s["ld"], s["li"], k, schedule=schedule)
    ids, d = O.knn(s["xs"], s["q"], k)
    assert np.array_equal(r.ids, ids)
    assert np.allclose(r.dist, d, rtol=1e-12)
    if schedule == (1,):
        assert r.lb_pruned.sum() > 0      # the bound prunes something


def test_infinite_offsets_give_exact_results(small_index):
    s = small_index
    N = s["lb"].shape[1]
    has = np.ones(N, dtype=bool)
    dF = np.full_like(s["lb"], -np.inf)   # d^f - (+inf)
    for sched in [(1,), (1, 0)]:
        r = O.leafi_search(s["lb"], s["order"], s["ld"], s["li"], 3, has, dF, sched)
        ids, _ = O.knn(s["xs"], s["q"], 3)
        assert np.array_equal(r.ids, ids)
        assert r.f_pruned.sum() == 0


def test_minus_infinite_offsets_prune_every_filtered_leaf_after_first_results(small_index):
    s = small_index
    N = s["lb"].shape[1]
    has = np.ones(N, dtype=bool)
    dF = np.full_like(s["lb"], np.inf)    # d^f - (-inf)
    r = O.leafi_search(s["lb"], s["order"], s["ld"], s["li"], 1, has, dF, (1,))
    # only the first leaf in visit order is searched; all others are pruned
    assert np.array_equal(r.scanned.sum(1), np.ones(len(s["q"])))
    first = s["order"][:, 0]
    assert np.all(r.scanned[np.arange(len(first)), first])
    assert np.all(r.lb_pruned | r.f_pruned | r.scanned)


def test_search_strictness_hand_case():
    # Two leaves, k = 1.  Leaf 0 (visited first) holds distances 2.0 and 5.0;
    # leaf 1 holds 1.0.  With tau = 2.0 after leaf 0: a bound or prediction
    # equal to tau does not prune (prune only when strictly greater).
    lb = np.array([[0.0, 2.0]])
    order = np.array([[0, 1]])
    ld = np.array([[[2.0, 5.0], [1.0, np.inf]]])
    li = np.array([[[10, 11], [20, -1]]])
    r = O.leafi_search(lb, order, ld, li, 1)
    assert r.ids[0, 0] == 20 and r.scanned[0, 1]
    has = np.array([False, True])
    r = O.leafi_search(lb, order, ld, li, 1, has, np.array([[0.0, 2.0]]))
    assert r.ids[0, 0] == 20
    r = O.leafi_search(lb, order, ld, li, 1, has, np.array([[0.0, 2.0000001]]))
    assert r.ids[0, 0] == 10 and r.f_pruned[0, 1]
    r = O.leafi_search(np.array([[0.0, 2.0000001]]), order, ld, li, 1)
    assert r.ids[0, 0] == 10 and r.lb_pruned[0, 1]
    # k = 3: tau stays +inf until three results are held, so nothing is pruned
    r = O.leafi_search(np.array([[0.0, 9.0]]), order, ld, li, 3, has, np.array([[0.0, 9.0]]))
    assert list(r.ids[0]) == [20, 10, 11]


def test_bsf_before_bruteforce(small_index):
    s = small_index
    xs, q, t = s["xs"], s["q"], s["t"]
    full = _direct(xs, q)
    leaf_of = np.empty(len(xs), dtype=np.int64)
    for L, mem in enumerate(t.leaves):
        leaf_of[mem] = L
    for k in (1, 3):
        got = O.bsf_before(s["ld"], s["order"], k)
        for c in range(0, len(q), 7):
            for pos in range(len(t.leaves)):
                L = s["order"][c, pos]
                prev = s["order"][c, :pos]
                pool = np.sort(full[c, np.isin(leaf_of, prev)])
                want = pool[k - 1] if len(pool) >= k else np.inf
                assert got[c, L] == pytest.approx(want, rel=1e-12)
        if k == 1:
            # prefix minimum of d^L along the visit order
            dl = np.take_along_axis(s["ld"][:, :, 0], s["order"], axis=1)
            pm = np.concatenate([np.full((len(q), 1), np.inf), np.minimum.accumulate(dl, axis=1)[:, :-1]], 1)
            assert np.allclose(np.take_along_axis(got, s["order"], axis=1), pm)


def _true_nbr_leaf(s, k):
    ids, _ = O.knn(s["xs"], s["q"], k)
    leaf_of = np.empty(len(s["xs"]), dtype=np.int64)
    for L, mem in enumerate(s["t"].leaves):
        leaf_of[mem] = L
    return leaf_of[ids], ids


@pytest.mark.parametrize("k", [1, 3])
def test_simulated_recall_is_conservative(small_index, k):
    s = small_index
    N = s["lb"].shape[1]
    rng = np.random.default_rng(41)
    has = rng.random(N) < 0.8
    dfilt = s["ld"][:, :, 0] + rng.normal(0, 0.5, size=s["lb"].shape)
    dbsf = O.bsf_before(s["ld"], s["order"], k)
    nbr_leaf, ids = _true_nbr_leaf(s, k)
    _, true_d = O.knn(s["xs"], s["q"], k)
    for trial in range(6):
        offs = np.where(has, rng.uniform(-0.5, 1.0, N), np.inf)
        sim = O.simulated_recall(dfilt, dbsf, nbr_leaf, has, offs)
        for sched in [(1,), (2,), (1, 0)]:
            r = O.leafi_search(s["lb"], s["order"], s["ld"], s["li"], k, has, dfilt - offs[None], sched)
            ret_d = np.where(r.ids >= 0, r.dist, np.inf)
            ach = O.recall_at_k(r.ids, ret_d, true_d).mean()
            assert ach >= sim - 1e-12


def test_calibration_hand_example():
    # Two filtered leaves, four calibration queries, k = 1 (values chosen by hand).
    dL = np.array([[1.0, 3.0], [2.0, 1.5], [1.2, 2.5], [4.0, 0.5]])
    df = np.array([[1.5, 2.0], [2.5, 2.6], [3.0, 2.0], [3.5, 1.0]])
    order = np.array([[0, 1], [0, 1], [1, 0], [1, 0]])
    dbsf = O.bsf_before(dL[:, :, None], order, 1)
    assert np.array_equal(dbsf, np.array([[np.inf, 1.0], [np.inf, 2.0], [2.5, np.inf], [0.5, np.inf]]))
    nbr_leaf = np.array([[0], [1], [0], [1]])
    has = np.array([True, True])
    offs, q = O.autotune_curve(df, dL, dbsf, nbr_leaf, has)
    # alpha sorted per filter: leaf 0 -> 0.5 0.5 0.5 1.8; leaf 1 -> 0.5 0.5 1.0 1.1
    assert np.allclose(offs[:4, 0], [0.5, 0.5, 0.5, 1.8])
    assert np.allclose(offs[:4, 1], [0.5, 0.5, 1.0, 1.1])
    assert np.isinf(offs[4]).all()
    # query 1's neighbour needs o_1 >= 0.6; query 2's is kept at equality (2.5 <= 2.5)
    assert np.allclose(q, [0.75, 0.75, 1.0, 1.0, 1.0])
    j, o = O.step_offsets(offs, q, 0.99, 4)
    assert j == 2 and np.allclose(o, [0.5, 1.0])
    j, o = O.step_offsets(offs, q, 0.7, 4, corrected=False)
    assert j == 0
    j, _ = O.step_offsets(offs, q, 0.7, 4)          # ceil(5 * 0.7) / 4 = 1
    assert j == 2
    j, _ = O.step_offsets(offs, q, 0.5, 4)          # ceil(2.5) / 4 = 0.75
    assert j == 0


def test_conformal_target_values():
    assert O.conformal_target(0.99, 500) == pytest.approx(0.992)
    assert O.conformal_target(0.95, 500) == pytest.approx(0.952)
    assert O.conformal_target(0.99, 99) == pytest.approx(1.0)
    assert O.conformal_target(1.0, 10) == 1.0


def test_calibration_reaches_target_on_calibration_set(small_index):
    s = small_index
    N = s["lb"].shape[1]
    rng = np.random.default_rng(44)
    has = np.ones(N, dtype=bool)
    dfilt = s["ld"][:, :, 0] * rng.uniform(0.7, 1.4, size=s["lb"].shape)
    dbsf = O.bsf_before(s["ld"], s["order"], 1)
    nbr_leaf, _ = _true_nbr_leaf(s, 1)
    _, true_d = O.knn(s["xs"], s["q"], 1)
    offs, q = O.autotune_curve(dfilt, s["ld"][:, :, 0], dbsf, nbr_leaf, has)
    assert np.all(np.diff(q) >= 0)                   # larger offsets never lower recall
    for tgt in (0.8, 0.9, 0.99):
        j, o = O.step_offsets(offs, q, tgt, len(q) - 1)
        r = O.leafi_search(s["lb"], s["order"], s["ld"], s["li"], 1, has, dfilt - o[None], (1,))
        ach = O.recall_at_k(r.ids, np.where(r.ids >= 0, r.dist, np.inf), true_d).mean()
        assert ach >= O.conformal_target(tgt, len(q) - 1) - 1e-12


# ---------------------------------------------------------------- Steffen interpolant

def test_steffen_hand_case_and_linear():
    fit = O.steffen_fit(np.array([0.0, 1.0, 2.0]), np.array([0.0, 1.0, 4.0]))
    # slopes: y'0 = 0 (one-sided parabola slope 0), y'1 = 2, y'2 = 4 -> both cubics are t^2
    for t in (0.0, 0.25, 0.5, 1.0, 1.5, 2.0):
        assert O.steffen_eval(fit, t) == pytest.approx(t * t, abs=1e-12)
    xl = np.array([0.0, 0.3, 1.0, 2.5])
    lin = O.steffen_fit(xl, 2 * xl + 1)
    for t in np.linspace(0, 2.5, 11):
        assert O.steffen_eval(lin, t) == pytest.approx(2 * t + 1, abs=1e-12)


def test_steffen_knots_and_monotone():
    rng = np.random.default_rng(51)
    x = np.cumsum(rng.uniform(0.01, 1.0, 12))
    y = np.cumsum(rng.exponential(1.0, 12) * (rng.random(12) < 0.7))
    fit = O.steffen_fit(x, y)
    for xi, yi in zip(x, y):
        assert O.steffen_eval(fit, xi) == pytest.approx(yi, abs=1e-10)
    grid = np.linspace(x[0], x[-1], 2000)
    vals = np.array([O.steffen_eval(fit, t) for t in grid])
    assert np.all(np.diff(vals) >= -1e-12)
    # no overshoot: values stay within each interval's endpoint range
    for i in range(len(x) - 1):
        seg = vals[(grid >= x[i]) & (grid <= x[i + 1])]
        assert seg.min() >= min(y[i], y[i + 1]) - 1e-10 and seg.max() <= max(y[i], y[i + 1]) + 1e-10


def test_steffen_offsets_hand_cases():
    """The offset mapping's own rules, by hand: equal recalls keep the largest
    offset, a target at or below the first recall takes that offset, a target
    above the largest finite-offset recall turns the filter off, two knots
    interpolate linearly, and a filter-less leaf stays +inf."""
    inf = np.inf
    # nc = 4 positions + the appended +inf row (recall 1)
    q = np.array([0.5, 0.5, 0.75, 0.75, 1.0])
    offs = np.array([[1.0, inf, 1.0],
                     [2.0, inf, 1.5],
                     [3.0, inf, 2.0],
                     [5.0, inf, 4.0],
                     [inf, inf, inf]])
    # knots after dedupe: filter 0 (0.5, 2), (0.75, 5); filter 2 (0.5, 1.5), (0.75, 4)
    got = O.steffen_offsets(offs, q, 0.5, 4, corrected=False)
    assert got[0] == 2.0 and got[2] == 1.5          # largest offset at the repeated recall, not 1.0
    assert np.isinf(got[1])                          # no filter on that leaf
    got = O.steffen_offsets(offs, q, 0.3, 4, corrected=False)
    assert got[0] == 2.0 and got[2] == 1.5          # below the first recall: first knot
    got = O.steffen_offsets(offs, q, 0.8, 4, corrected=False)
    assert np.isinf(got).all()                       # above the largest finite recall: filters off
    got = O.steffen_offsets(offs, q, 0.625, 4, corrected=False)
    assert got[0] == pytest.approx(3.5, abs=1e-12)  # 2 + 0.5 * (5 - 2)
    assert got[2] == pytest.approx(2.75, abs=1e-12)  # 1.5 + 0.5 * (4 - 1.5)
    got = O.steffen_offsets(offs, q, 0.75, 4, corrected=False)
    assert got[0] == pytest.approx(5.0, abs=1e-12) and got[2] == pytest.approx(4.0, abs=1e-12)


def test_steffen_offsets_collinear_and_corrected_target():
    """Three collinear knots interpolate linearly (every Steffen slope equals the
    common secant), and the corrected level ceil((nc + 1) t) / nc is what is
    looked up."""
    inf = np.inf
    q = np.array([0.2, 0.4, 0.6, 1.0])               # nc = 3
    offs = np.array([[1.0], [2.0], [3.0], [inf]])
    assert O.steffen_offsets(offs, q, 0.5, 3, corrected=False)[0] == pytest.approx(2.5, abs=1e-12)
    assert O.steffen_offsets(offs, q, 0.3, 3, corrected=False)[0] == pytest.approx(1.5, abs=1e-12)
    # corrected: 0.3 -> ceil(1.2) / 3 = 2/3 > 0.6, the filter is switched off
    assert np.isinf(O.steffen_offsets(offs, q, 0.3, 3, corrected=True)[0])
    # corrected: 0.1 -> ceil(0.4) / 3 = 1/3, between the first two knots
    assert O.steffen_offsets(offs, q, 0.1, 3, corrected=True)[0] == pytest.approx(1.0 + (1 / 3 - 0.2) / 0.2,
                                                                                abs=1e-12)


# ---------------------------------------------------------------- leaf selection (Algorithm 3)

def test_select_leaves_cases():
    sizes = np.array([5, 10, 10, 3])
    assert list(O.select_leaves(sizes, 4, 1.0, 2.0)) == [1, 2]
    assert list(O.select_leaves(sizes, 0, 1.0, 100.0)) == [1, 2, 0, 3]
    assert list(O.select_leaves(sizes, 0, 1.0, 0.5)) == []
    assert list(O.select_leaves(sizes, 10, 1.0, 100.0)) == [1, 2]
    assert O.size_threshold(2.0, 46.0, 0.16) == pytest.approx(575.0)


# ---------------------------------------------------------------- CNN filter (two correlations, kernel 3)

def _cnn_pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def test_cnn_hand_case_fixes_tap_order_and_padding():
    # tap 0 reads position p - 1, tap 2 reads p + 1; one zero pad at each end
    w = _cnn_pack([[1.0, 0.0, 0.0]], [0.0], [[[0.0, 0.0, 1.0]]], [0.0], [2.0], 0.5)
    assert len(w) == O.cnn_param_count(1)
    # z1 = x[p-1] = [0, 1, 2]; z2 = h1[p+1] = [1, 2, 0]; mean 1; 2 * 1 + 0.5
    assert O.cnn_forward(w, np.array([[1.0, 2.0, 3.0]]), 1)[0] == pytest.approx(2.5, abs=1e-15)


def test_cnn_linear_regime_matches_numpy_correlate():
    """With biases that keep every pre-activation positive the network is two
    zero-padded cross-correlations and a mean; numpy's correlate computes them."""
    rng = np.random.default_rng(41)
    C, m = 5, 17
    W1, W2 = rng.normal(0, 0.3, (C, 3)), rng.normal(0, 0.3, (C, C, 3))
    b1, b2, w3, b3 = rng.uniform(20, 30, C), rng.uniform(200, 300, C), rng.normal(0, 1, C), 0.7
    w = _cnn_pack(W1, b1, W2, b2, w3, b3)
    X = rng.normal(0, 1, (4, m))
    got = O.cnn_forward(w, X, C)
    for i, x in enumerate(X):
        h1 = np.stack([b1[c] + np.correlate(np.pad(x, 1), W1[c], "valid") for c in range(C)])
        assert h1.min() > 0
        z2 = np.stack([b2[o] + sum(np.correlate(np.pad(h1[c], 1), W2[o, c], "valid") for c in range(C))
                       for o in range(C)])
        assert z2.min() > 0
        assert got[i] == pytest.approx(b3 + w3 @ z2.mean(axis=1), rel=1e-12)


def test_cnn_center_taps_are_a_per_position_network():
    """Outer taps zero: each position runs the same two-layer network on its
    own value, and the readout averages it over the positions."""
    rng = np.random.default_rng(42)
    C, m = 6, 11
    W1, W2 = rng.normal(0, 1, (C, 3)), rng.normal(0, 1, (C, C, 3))
    W1[:, [0, 2]] = 0.0
    W2[:, :, [0, 2]] = 0.0
    b1, b2, w3 = rng.normal(0, 1, C), rng.normal(0, 1, C), rng.normal(0, 1, C)
    w = _cnn_pack(W1, b1, W2, b2, w3, -0.3)
    X = rng.normal(0, 1, (5, m))
    h1 = np.maximum(X[:, :, None] * W1[:, 1] + b1, 0.0)          # [B, m, C]
    h2 = np.maximum(h1 @ W2[:, :, 1].T + b2, 0.0)               # [B, m, C]
    want = h2.mean(axis=1) @ w3 - 0.3
    assert np.allclose(O.cnn_forward(w, X, C), want, rtol=1e-12, atol=1e-12)


def test_cnn_output_is_shift_invariant_inside_a_zero_border():
    """With b1, b2 <= 0 a zero input region maps to zero activations, so moving
    the series by one position inside a zero border leaves the mean unchanged."""
    rng = np.random.default_rng(43)
    C, m = 4, 20
    W1, W2 = rng.normal(0, 1, (C, 3)), rng.normal(0, 1, (C, C, 3))
    w = _cnn_pack(W1, -np.abs(rng.normal(0, 0.2, C)), W2, -np.abs(rng.normal(0, 0.2, C)), rng.normal(0, 1, C), 0.1)
    x = np.zeros((1, m))
    x[0, 4:14] = rng.normal(0, 1, 10)
    y = np.roll(x, 2, axis=1)
    assert O.cnn_forward(w, x, C)[0] == pytest.approx(O.cnn_forward(w, y, C)[0], rel=1e-12)
    # a non-zero bias breaks it (the border activations are then not zero)
    w2 = w.copy()
    w2[3 * C: 4 * C] = 1.0
    assert abs(O.cnn_forward(w2, x, C)[0] - O.cnn_forward(w2, np.roll(x, 5, axis=1), C)[0]) > 1e-6


def test_cnn_gradient_central_differences():
    rng = np.random.default_rng(44)
    C, m, B = 3, 7, 4
    w = rng.normal(0, 0.6, O.cnn_param_count(C))
    X, y = rng.normal(0, 1, (B, m)), rng.normal(0, 1, B)
    loss, g = O.cnn_mse_grad(w, X, y, C)
    assert loss == pytest.approx(float(((O.cnn_forward(w, X, C) - y) ** 2).mean()), rel=1e-12)
    eps = 1e-6
    num = np.empty_like(w)
    for i in range(len(w)):
        e = np.zeros_like(w)
        e[i] = eps
        num[i] = (O.cnn_mse_grad(w + e, X, y, C)[0] - O.cnn_mse_grad(w - e, X, y, C)[0]) / (2 * eps)
    assert np.allclose(g, num, rtol=1e-5, atol=1e-7)


# ---------------------------------------------------------------- leaf selection as a knapsack (Equations 1-2)

def test_knapsack_textbook_case():
    # the classic three-item instance: the two heavier items beat the lightest pair
    assert list(O.knapsack_01([60, 100, 120], [10, 20, 30], 50)) == [1, 2]
    assert list(O.knapsack_01([60, 100, 120], [10, 20, 30], 0)) == []
    assert list(O.knapsack_01([60, 100, 120], [10, 20, 30], 10)) == [0]
    assert list(O.knapsack_01([5.0], [7], 6)) == []


def test_knapsack_matches_brute_force():
    rng = np.random.default_rng(21)
    for _ in range(300):
        n = int(rng.integers(1, 9))
        v = rng.normal(1.0, 1.5, n)
        wt = rng.integers(0, 7, n)
        C = int(rng.integers(0, 16))
        got = O.knapsack_01(v, wt, C)
        assert wt[got].sum() <= C
        best = max(sum(v[i] for i in range(n) if mask >> i & 1)
                   for mask in range(1 << n) if sum(wt[i] for i in range(n) if mask >> i & 1) <= C)
        assert v[got].sum() == pytest.approx(best, abs=1e-12)


def test_knapsack_equal_weights_takes_the_largest_values():
    rng = np.random.default_rng(22)
    v = rng.normal(0.0, 1.0, 40)
    for cap in (0, 1, 5, 17, 40):
        got = O.knapsack_01(v, np.ones(40, dtype=np.int64), cap)
        pos = np.flatnonzero(v > 0)
        want = pos[np.argsort(-v[pos])][:cap]
        assert set(got) == set(want)


def test_selection_estimates_hand_case():
    # two queries, three leaves; lb <= d^L everywhere
    lb = np.array([[0.0, 1.0, 3.0], [0.5, 2.5, 0.1]])
    dL = np.array([[2.0, 1.5, 4.0], [1.0, 3.0, 0.8]])
    order = np.array([[0, 1, 2], [2, 0, 1]])
    # query 0: leaf 0 (bsf inf) -> 2.0; leaf 1 reached (1.5 < 2.0) -> 1.5; leaf 2 pruned (3.0 > 1.5)
    # query 1: leaf 2 (bsf inf) -> 0.8; leaf 0 reached, nothing below 0.8 (ideal prune); leaf 1 pruned
    p_lb, p_f = O.selection_estimates(lb, dL, order)
    assert list(p_lb) == [0.0, 0.5, 0.5]
    assert list(p_f) == [0.5, 0.0, 0.0]


def test_selection_estimates_equal_the_search_simulation():
    """p^lb is the share of queries whose exact sequential search (Algorithm 2,
    no filters) prunes the leaf by its bound; the ideal filter rate is the
    share of its visits that Algorithm 2 with exact filters (d^F = d^L)
    prunes by the filter: exact filters prune only leaves holding nothing
    better, so the best-so-far sequence is unchanged."""
    rng = np.random.default_rng(23)
    nq, N = 30, 12
    dL = rng.uniform(1.0, 10.0, (nq, N))
    lb = dL * rng.uniform(0.0, 1.0, (nq, N))
    order = O.visit_order(lb)
    p_lb, p_f = O.selection_estimates(lb, dL, order)
    ids = np.arange(nq * N, dtype=np.int64).reshape(nq, N, 1)
    plain = O.leafi_search(lb, order, dL[:, :, None], ids, 1, schedule=(1,))
    assert np.array_equal(p_lb, plain.lb_pruned.mean(axis=0))
    filt = O.leafi_search(lb, order, dL[:, :, None], ids, 1, has_filter=np.ones(N, dtype=bool), dF=dL,
                          schedule=(1,))
    assert np.array_equal(filt.lb_pruned, plain.lb_pruned)
    assert np.array_equal(filt.ids, plain.ids)
    reach = (~plain.lb_pruned).sum(axis=0)
    want = np.where(reach > 0, filt.f_pruned.sum(axis=0) / np.maximum(reach, 1), 0.0)
    assert np.array_equal(p_f, want)


def test_leaf_benefit_hand_case():
    # (1 - 0.25) * (0.5 * 2 * 100 - 30) = 52.5; a tiny leaf loses time
    b = O.leaf_benefit([100, 10], [0.25, 0.0], [0.5, 0.5], 2.0, 30.0)
    assert b[0] == pytest.approx(52.5) and b[1] == pytest.approx(-20.0)


def test_select_knapsack_reduces_to_algorithm3_under_uniform_rates():
    """With the same p^lb everywhere and ideal filters everywhere (p^F = 1/a),
    b_i > 0 is |N_i| > a t^F / t^S and b grows with |N_i|: the knapsack picks
    Algorithm 3's leaves, in its order (sizes kept off the threshold)."""
    rng = np.random.default_rng(24)
    for trial in range(20):
        N = 60
        sizes = rng.choice(np.arange(1, 400), N, replace=False)
        sizes = sizes[sizes != 100]
        a, tS, tF = 2.0, 1e-3, 0.05        # th = a tF / tS = 100
        w, cM = 10, int(rng.integers(0, 400))
        sel, b = O.select_knapsack(sizes, np.full(len(sizes), 0.3), np.ones(len(sizes)), a, tS, tF, w, cM)
        want = O.select_leaves(sizes, O.size_threshold(a, tF, tS), w, cM)
        assert list(sel) == list(want)


def test_select_knapsack_uses_per_leaf_rates():
    # the largest leaf is always pruned by its bound (no benefit); the filter
    # of leaf 2 would prune nothing; the budget holds two filters
    sizes = np.array([1000, 500, 800, 300])
    p_lb = np.array([1.0, 0.2, 0.1, 0.1])
    p_f = np.array([1.0, 1.0, 0.0, 0.9])
    sel, b = O.select_knapsack(sizes, p_lb, p_f, 2.0, 1.0, 10.0, 4, 8)
    assert b[0] == 0.0 and b[2] < 0
    assert list(sel) == [1, 3]


# ---------------------------------------------------------------- recall

def test_recall_at_k_hand_cases():
    true_d = np.array([[1.0, 2.0, 3.0]])
    assert O.recall_at_k(np.array([[4, 5, 6]]), np.array([[1.0, 2.0, 3.0]]), true_d)[0] == 1.0
    assert O.recall_at_k(np.array([[4, 5, 6]]), np.array([[1.0, 2.0, 3.5]]), true_d)[0] == pytest.approx(2 / 3)
    assert O.recall_at_k(np.array([[4, -1, -1]]), np.array([[1.0, np.inf, np.inf]]), true_d)[0] == pytest.approx(1 / 3)


# ---------------------------------------------------------------- iSAX backbone (MESSI)

def _phi(x: float) -> float:
    """Standard normal CDF from the complementary error function (math.erfc),
    independent of the quantile routine the breakpoints come from."""
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def test_isax_breakpoints_closed_forms_and_nesting():
    assert list(O.isax_breakpoints(1)) == [0.0]
    b2 = O.isax_breakpoints(2).astype(np.float64)
    # Phi^-1(3/4) = 0.6744897501960817 (textbook quartile of N(0, 1))
    assert np.allclose(b2, [-0.6744897501960817, 0.0, 0.6744897501960817], rtol=0, atol=1e-7)
    b8 = O.isax_breakpoints(8)
    assert len(b8) == 255 and np.all(np.diff(b8) > 0)
    assert np.array_equal(b8, -b8[::-1])               # symmetric about 0
    for j, v in enumerate(b8.astype(np.float64), start=1):
        # within the fp32 rounding of the quantile: |Phi(v) - j/256| <= density * |v| * 2^-23
        dens = math.exp(-v * v / 2) / math.sqrt(2 * math.pi)
        assert abs(_phi(v) - j / 256.0) <= dens * max(abs(v), 1e-30) * 2.0 ** -23 + 1e-15, j
    for b in range(1, 8):
        bb = O.isax_breakpoints(b)
        assert np.array_equal(bb, b8[(np.arange(1, 2 ** b) << (8 - b)) - 1]), b


def test_sax_symbols_hand_cases_and_prefixes():
    b8 = O.isax_breakpoints(8)
    v = np.array([-10.0, 10.0, 0.0, -1e-7, b8[10], np.nextafter(b8[10], np.float32(-np.inf))], dtype=np.float32)
    assert list(O.sax_symbols(v)) == [0, 255, 128, 127, 11, 10]
    rng = np.random.default_rng(5)
    mu = rng.standard_normal((500, 4)).astype(np.float32)
    s8 = O.sax_symbols(mu)
    for b in range(1, 8):
        assert np.array_equal(s8 >> (8 - b), O.sax_symbols(mu, b)), b


def test_isax_tree_partition_words_and_sizes():
    raw = W.random_walk(8000, 64, seed=33)
    xs = O.znorm(raw)
    mu, _ = O.segment_stats(xs, 16)
    cap = 60
    t = O.build_isax_tree(mu, 64, cap)
    allids = np.sort(np.concatenate(t.leaves))
    assert np.array_equal(allids, np.arange(len(xs)))
    s8 = O.sax_symbols(mu)
    words = []
    for L, ids in enumerate(t.leaves):
        bits, sym = t.isax[L]
        assert np.all(np.diff(ids) > 0)
        assert np.all(bits >= 1) and np.all(bits <= 8)
        # every member's symbols start with the leaf's word
        assert np.array_equal(s8[ids] >> (8 - bits)[None, :], np.broadcast_to(sym, (len(ids), 16)))
        if len(ids) > cap:
            assert np.all(bits == 8) and np.all(s8[ids] == s8[ids[0]])
        words.append(int("".join(str(int(x)) for x in (sym >> (bits - 1))), 2))
    # depth-first order: root words never decrease along the leaves
    assert all(a <= b for a, b in zip(words, words[1:]))
    assert len(t.leaves) > 100


def test_isax_lower_bound_hand_case():
    # m = 4, two segments of length 2; the leaf holds one series whose
    # segment means are 0.3 and -1.2, at one bit per segment: [0, +inf) and
    # (-inf, 0).  Query means 0.5 (inside) and 0.4 (0.4 above the interval).
    t = O.Tree(root=O.Node(members=np.array([0])), S=2, m=4)
    t.leaves = [np.array([0])]
    mu = np.array([[0.3, -1.2]], dtype=np.float32)
    t.isax = [(np.array([1, 1]), O.sax_symbols(mu, 1)[0])]
    box = O.isax_boxes(t)
    lb = O.lower_bound(np.array([[0.5, 0.4]]), np.array([[3.0, 0.0]]), box, 4)
    # 2 * (0^2 + gap^2) with gap = 0.4 - (0 widened by one ulp)
    assert lb[0, 0] == pytest.approx(math.sqrt(2 * 0.4 ** 2), rel=1e-6)


@pytest.fixture(scope="module")
def isax_index():
    raw = W.random_walk(6000, 64, seed=37)
    xs = O.znorm(raw)
    mu, _ = O.segment_stats(xs, 16)
    t = O.build_isax_tree(mu, 64, 50)
    q = O.znorm(W.noisy_queries(raw, 30, (0.05, 0.3), 9, 10)[0])
    qmu, qsd = O.query_stats(q, 16)
    lb = O.lower_bound(qmu, qsd, O.isax_boxes(t), 64)
    ld, li = O.leaf_knn(xs, t.leaves, q, 5)
    return dict(xs=xs, t=t, q=q, lb=lb, ld=ld, li=li)


def test_isax_lower_bound_never_exceeds_node_distance(isax_index):
    s = isax_index
    assert np.all(s["lb"] <= s["ld"][:, :, 0] * (1 + 1e-12) + 1e-12)


@pytest.mark.parametrize("schedule", [(1,), (1, 0)])
def test_plain_isax_tree_search_is_exact(isax_index, schedule):
    s = isax_index
    r = O.leafi_search(s["lb"], O.visit_order(s["lb"]), s["ld"], s["li"], 5, schedule=schedule)
    ids, d = O.knn(s["xs"], s["q"], 5)
    assert np.array_equal(r.ids, ids)
    assert np.allclose(r.dist, d, rtol=1e-12)
    assert r.lb_pruned.sum() > 0
