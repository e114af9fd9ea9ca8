"""CNN learned filters through the C ABI against the FP64 oracle: inference
(dense, and listed pairs inside a filtered search against the oracle's
Algorithm 2 at equal schedule), one SGD step against the FP64 gradient, and
training with the measured inference cost, whose size threshold exceeds the
MLP filters' on the same index."""
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


@pytest.mark.parametrize("F,m,C,nq", [(3, 32, 32, 50), (2, 96, 96, 20), (2, 64, 16, 33), (1, 8, 4, 7),
                                      (2, 36, 8, 5)])
def test_cnn_infer_matches_oracle(F, m, C, nq):
    pkg = _pkg()
    w = W.cnn_weights(F, C, seed=F + m + C, out_bias=0.5)
    x = O.znorm(W.random_walk(nq, m, seed=m + 1))
    got = pkg.cnn_infer(torch.from_numpy(w).cuda(), m, C, torch.from_numpy(x).cuda()).cpu().numpy()
    for f in range(F):
        want = O.cnn_forward(w[f], x, C)
        # FP32 sums of 3C terms per second-layer output, m outputs per channel
        assert np.allclose(got[:, f], want, rtol=1e-4, atol=1e-4 * np.abs(want).max()), \
            np.abs(got[:, f] - want).max()


def test_cnn_shape_limits_are_enforced():
    pkg = _pkg()
    w = torch.zeros((1, 3 * 128 * 128 + 6 * 128 + 1), device="cuda")
    x = torch.zeros((2, 128), device="cuda")
    with pytest.raises(pkg.LeafiError):
        pkg.cnn_infer(w, 128, 128, x)      # conv2 weights and activations exceed the LDS
    with pytest.raises(pkg.LeafiError):
        pkg.cnn_infer(w[:, :3 * 36 + 6 * 6 + 1].contiguous(), 36, 6, x[:, :36].contiguous())  # 6 channels


@pytest.mark.parametrize("F,m,C,B", [(2, 16, 8, 5), (2, 32, 32, 9), (1, 40, 12, 3)])
def test_cnn_sgd_step_matches_fp64_gradient(F, m, C, B):
    pkg = _pkg()
    lr = 0.05
    w = W.cnn_weights(F, C, seed=7)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((F, B, m)).astype(np.float32)
    y = rng.uniform(1, 4, (F, B)).astype(np.float32)
    wt = torch.from_numpy(w.copy()).cuda()
    loss = pkg.cnn_sgd_step(wt, m, C, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), lr).cpu().numpy()
    got = wt.cpu().numpy().astype(np.float64)
    for f in range(F):
        l64, g = O.cnn_mse_grad(w[f].astype(np.float64), x[f], y[f].astype(np.float64), C)
        assert abs(loss[f] - l64) <= 1e-5 * l64
        step_got = got[f] - w[f]
        step_want = -lr * g
        assert np.max(np.abs(step_got - step_want)) <= 1e-4 * np.abs(step_want).max() + 1e-7


@pytest.fixture(scope="module")
def gm64():
    """30k Gaussian-mixture series of length 64 (median splits, capacity 1,500),
    1,000 noisy queries, and the oracle's tree, bounds and per-leaf 1-NN."""
    pkg = _pkg()
    m = 64
    raw = W.gaussian_mixture(30000, m, 30, 0.4, 51, 52)
    q, _, _ = W.noisy_queries(raw, 1000, 0.2, 53, 54)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=1500, n_segments=8)
    xs, qs = O.znorm(raw), O.znorm(q)
    mu, sd = O.segment_stats(xs, 8)
    tree = O.build_tree(mu, sd, m, 1500, "median")
    off, mem = ix.leaves()
    assert len(tree.leaves) == len(off) - 1
    for L, members in enumerate(tree.leaves):
        assert np.array_equal(mem[off[L]:off[L + 1]], members)
    qmu, qsd = O.query_stats(qs, 8)
    lb = O.lower_bound(qmu, qsd, O.leaf_boxes(mu, sd, tree), m)
    ld, li = O.leaf_knn(xs, tree.leaves, qs, 1)
    return dict(pkg=pkg, ix=ix, m=m, raw=raw, q=q, xs=xs, qs=qs, lb=lb, order=O.visit_order(lb), ld=ld, li=li,
                N=len(tree.leaves))


def test_cnn_filtered_search_matches_oracle_algorithm2(gm64):
    """Seeded CNN filters on every leaf (listed-pair inference inside the
    search) against the oracle's Algorithm 2 with the oracle's FP64 CNN
    outputs, at schedule (1, 0)."""
    s = gm64
    ix, m, N = s["ix"], s["m"], s["N"]
    C = 32
    wts = W.cnn_weights(N, C, seed=61, out_bias=4.0)
    offs = np.random.default_rng(62).uniform(0.0, 3.0, size=N).astype(np.float32)
    ix.set_cnn_filters(np.arange(N, dtype=np.int32), torch.from_numpy(wts).cuda(), C)
    inf = ix.info()
    assert inf["filter_arch"] == 1 and inf["hidden"] == C and inf["n_filters"] == N
    ids_f, w_back = ix.get_filters()
    assert np.array_equal(w_back.cpu().numpy(), wts)
    ix.set_offsets([1], [0.9], offs[None])
    qt = torch.from_numpy(s["q"]).cuda()
    res = []
    for flags in (0, s["pkg"].SEARCH_HOST_ROUNDS):
        ids, d, st = ix.search(qt, k=1, target=0.9, use_filters=True, schedule=(1, 0), with_stats=True, flags=flags)
        res.append((ids.cpu().numpy(), d.cpu().numpy(), st))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    df = np.stack([O.cnn_forward(wts[f], s["qs"], C) for f in range(N)], 1)
    r = O.leafi_search(s["lb"], s["order"], s["ld"], s["li"], 1, np.ones(N, dtype=bool),
                       df - offs[None].astype(np.float64), (1, 0))
    assert r.f_pruned.sum() > 0 and r.scanned.sum() > 0
    assert_knn_parity(res[0][0], res[0][1], r.ids, r.dist, s["xs"], s["qs"])
    st = res[0][2]
    if not r.near_tie.any():
        assert st["leaves_filter_pruned"] == int(r.f_pruned.sum())
        assert st["leaves_scanned"] == int(r.scanned.sum())


def test_train_cnn_filters_and_threshold(gm64):
    """Training CNN filters (channels = m): the measured t^F and hence
    Algorithm 3's threshold exceed the MLP filters' on the same index; the
    trained filters predict the node-wise distances of their validation
    queries no worse than their mean target does; calibration and a
    filtered search run through them."""
    s = gm64
    ix, m = s["ix"], s["m"]
    w_bytes = (3 * m * m + 6 * m + 1) * 4
    rep_mlp = ix.train_filters(n_global=60, n_local=10, noise_lo=0.05, noise_hi=0.3, max_epochs=2, seed=3,
                               mem_budget=1 << 30)
    rep = ix.train_filters(n_global=100, n_local=20, noise_lo=0.05, noise_hi=0.3, max_epochs=30, seed=3, arch="cnn",
                           th_override=0.0, mem_budget=3 * w_bytes + 100, keep_examples=1)
    assert rep["n_filters"] == 3
    inf = ix.info()
    assert inf["filter_arch"] == 1 and inf["hidden"] == m
    ep, tr = ix.train_trace()
    assert np.all(ep >= 1)
    # validation MSE of the kept weights below that of the constant mean target
    q, exq, y, n_train = ix.examples()
    y = y.cpu().numpy().astype(np.float64)
    for f in range(3):
        base = float(((y[f, n_train:] - y[f, :n_train].mean()) ** 2).mean())
        assert np.nanmin(tr[f]) <= base * 1.05, (f, np.nanmin(tr[f]), base)
    # the kept weights' predictions equal the oracle's forward on the same queries
    ids_f, wk = ix.get_filters()
    qs = O.znorm(q.cpu().numpy())
    dev = s["pkg"].cnn_infer(wk, m, m, torch.from_numpy(qs.astype(np.float32)).cuda()).cpu().numpy()
    for f in range(3):
        want = O.cnn_forward(wk[f].cpu().numpy(), qs, m)
        assert np.allclose(dev[:, f], want, rtol=1e-4, atol=1e-4 * np.abs(want).max())
    # measured costs: the CNN's threshold is far above the MLP's
    rep_c = ix.train_filters(n_global=60, n_local=10, max_epochs=1, seed=3, arch="cnn", mem_budget=w_bytes + 100)
    assert rep_c["t_filter_s"] > 5 * rep_mlp["t_filter_s"]
    assert rep_c["th"] > 5 * rep_mlp["th"]
    # calibration and search through trained CNN filters
    rep = ix.train_filters(n_global=100, n_local=20, max_epochs=5, seed=3, arch="cnn", th_override=0.0,
                           mem_budget=3 * w_bytes + 100)
    calib, _, _ = W.noisy_queries(s["raw"], 200, (0.05, 0.3), 71, 72)
    ix.calibrate(torch.from_numpy(calib).cuda(), [1], [0.95])
    ids, d = ix.search(torch.from_numpy(s["q"]).cuda(), k=1, target=0.95, use_filters=True)
    assert (ids.cpu().numpy() >= 0).all()
