"""Leaf selection as a knapsack (Equations 1-2) through the C ABI, against
the FP64 oracle: the per-leaf rates p^lb and ideal p^F estimated by following
each training query's exact 1-NN search, the benefit b_i, the knapsack's
choice, and leafi_train_filters with that selection rule."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

M = 96
W_BYTES = (M * M + 2 * M + 1) * 4


def _pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    return pkg


@pytest.fixture(scope="module")
def ragged():
    """30k Gaussian-mixture series of length 96, midpoint splits (ragged
    leaves), 400 training-like queries at noise 0.05-0.2, and the oracle's
    bounds, visit orders and node-wise 1-NN distances for them."""
    pkg = _pkg()
    raw = W.gaussian_mixture(30000, M, 40, 0.3, 41, 42)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=2000, n_segments=16, split_rule="midpoint")
    q, _, _ = W.noisy_queries(raw, 400, (0.05, 0.2), 61, 62)
    xs, qs = O.znorm(raw), O.znorm(q)
    mu, sd = O.segment_stats(xs, 16)
    tree = O.build_tree(mu, sd, M, 2000, "midpoint")
    off, mem = ix.leaves()
    assert len(tree.leaves) == len(off) - 1
    for L, members in enumerate(tree.leaves):
        assert np.array_equal(mem[off[L]:off[L + 1]], members)
    qmu, qsd = O.query_stats(qs, 16)
    lb = O.lower_bound(qmu, qsd, O.leaf_boxes(mu, sd, tree), M)
    ld, _ = O.leaf_knn(xs, tree.leaves, qs, 1)
    return dict(pkg=pkg, ix=ix, raw=raw, q=q, sizes=np.diff(off), lb=lb, order=O.visit_order(lb), dL=ld[:, :, 0])


def test_knapsack_estimates_and_choice_match_oracle(ragged):
    ix, sizes = ragged["ix"], ragged["sizes"]
    nq = len(ragged["q"])
    p_lb, p_f = O.selection_estimates(ragged["lb"], ragged["dL"], ragged["order"])
    reach = np.round((1.0 - p_lb) * nq)
    a, tS, tF = 2.0, 1e-9, 1.5e-7
    for K in (0, 3, 6, 1000):
        r = ix.select_knapsack(torch.from_numpy(ragged["q"]).cuda(), a=a, t_filter=tF, t_series=tS, hidden=M,
                               mem_budget=K * W_BYTES + W_BYTES // 2)
        # rates: the library's bounds (fp32) and distances decide the same
        # comparisons as the oracle's except at near-ties (a query or two)
        assert np.abs(r["p_lb"] - p_lb).max() <= 2.0 / nq
        assert np.all(np.abs(r["p_f"] - p_f) <= 2.0 / np.maximum(reach, 1) + 1e-12)
        # Equation 2 on the library's own rates, and the knapsack's choice on them
        b_want = O.leaf_benefit(sizes, r["p_lb"], r["p_f"] / a, tS, tF)
        assert np.allclose(r["benefit"], b_want, rtol=1e-12, atol=1e-18)
        sel_want, _ = O.select_knapsack(sizes, r["p_lb"], r["p_f"], a, tS, tF, W_BYTES, K * W_BYTES + W_BYTES // 2)
        assert list(r["leaves"]) == list(sel_want)
        # against the oracle's own rates: optimal up to what the near-ties move
        sel_or, b_or = O.select_knapsack(sizes, p_lb, p_f, a, tS, tF, W_BYTES, K * W_BYTES + W_BYTES // 2)
        slack = len(sel_or) * np.abs(r["benefit"] - b_or).max() * 2 + 1e-18
        assert len(r["leaves"]) == len(sel_or)
        assert b_or[r["leaves"]].sum() >= b_or[sel_or].sum() - slack
    # a cost ratio t^F / t^S at the median of p^F |N| / a: with room for all,
    # exactly the leaves above it (and not always pruned by their bounds) are taken
    v = r["p_f"] * sizes / a
    ratio = float(np.median(v[v > 0]))
    r = ix.select_knapsack(torch.from_numpy(ragged["q"]).cuda(), a=a, t_filter=ratio * tS, t_series=tS, hidden=M,
                           mem_budget=1000 * W_BYTES)
    out = np.setdiff1d(np.arange(len(sizes)), r["leaves"])
    assert len(r["leaves"]) > 0 and len(out) > 0
    assert np.all(r["benefit"][out] <= 0) and np.all(r["benefit"][r["leaves"]] > 0)
    assert set(r["leaves"]) == set(np.flatnonzero((v > ratio) & (r["p_lb"] < 1.0)))


def test_knapsack_argument_errors(ragged):
    pkg, ix = ragged["pkg"], ragged["ix"]
    qd = torch.from_numpy(ragged["q"][:4]).cuda()
    with pytest.raises(pkg.LeafiError):
        ix.select_knapsack(qd, a=0.0, t_filter=1e-7, t_series=1e-9)
    with pytest.raises(pkg.LeafiError):
        ix.select_knapsack(qd, a=2.0, t_filter=1e-7, t_series=1e-9, mem_budget=-1)
    with pytest.raises(pkg.LeafiError):
        ix.train_filters(n_global=8, n_local=2, max_epochs=1, selection=7)


def test_train_filters_with_knapsack_selection(ragged):
    """leafi_train_filters(selection=KNAPSACK) installs exactly what
    leafi_select_knapsack picks on its global training queries (t^F / t^S
    fixed through th_override = a t^F / t^S), and trains them; with measured
    costs it reports them and installs only leaves of positive benefit."""
    ix = ragged["ix"]
    n_g = 200
    th = 600.0
    rep = ix.train_filters(n_global=n_g, n_local=20, noise_lo=0.05, noise_hi=0.2, max_epochs=2, selection="knapsack",
                           th_override=th, mem_budget=4 * W_BYTES + 100, seed=7, keep_examples=1)
    got, _ = ix.get_filters()
    assert rep["n_filters"] == len(got) == 4
    q, _, _, _ = ix.examples()
    r = ix.select_knapsack(q[:n_g].contiguous(), a=2.0, t_filter=th / 2.0, t_series=1.0, hidden=M,
                           mem_budget=4 * W_BYTES + 100)
    assert list(got) == list(r["leaves"])
    assert np.all(r["benefit"][got] > 0)
    # a budget of one filter takes the leaf of largest benefit
    rep = ix.train_filters(n_global=n_g, n_local=20, noise_lo=0.05, noise_hi=0.2, max_epochs=1, selection="knapsack",
                           th_override=th, mem_budget=W_BYTES, seed=7)
    got1, _ = ix.get_filters()
    assert list(got1) == [got[0]]
    # measured costs
    rep = ix.train_filters(n_global=n_g, n_local=20, max_epochs=1, selection="knapsack", mem_budget=4 * W_BYTES,
                           seed=7)
    assert rep["t_filter_s"] > 0 and rep["t_series_s"] > 0
    assert rep["th"] == pytest.approx(2.0 * rep["t_filter_s"] / rep["t_series_s"])
    assert rep["n_filters"] <= 4
