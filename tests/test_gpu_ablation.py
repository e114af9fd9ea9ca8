"""Ablation and target sweep as a regression suite for the calibrator
(paper: Section "Without Local Training Data" and its table of query time
and recall without and with local training data; Section "Varying Recall
Target"), on 1M random walks of length 256 (capacity 10,000) with k = 1.

For training without (n_local = 0) and with local queries, calibration for
targets 0.95 ... 0.999 on 500 held-out queries must give, on 3,000 test
queries at noise 0.05 / 0.1 / 0.2:
  * offsets that never decrease with the target (every filter);
  * with schedule (1, 0) (the filters decide once, with the first round's
    best-so-far, which the target does not change) series scanned and
    recall that never decrease with the target;
  * recall against the exact search within a finite-sample band below each
    target (three standard errors of a calibration set and a test set).
The exact search is the library's filters-off search, itself matched to
the FP64 oracle by the parity tests; a sample of it is checked here too."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TARGETS = (0.95, 0.97, 0.99, 0.995, 0.999)


def _pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    return pkg


@pytest.fixture(scope="module")
def rw1m():
    pkg = _pkg()
    wl = W.WORKLOADS["rw1m"]
    raw = W.random_walk(wl["n"], wl["m"], wl["seed"])
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16)
    c, _, _ = W.noisy_queries(raw, wl["n_calib"], tuple(wl["train_sigma"]), wl["calib_seed"], wl["calib_seed"] + 100)
    tests = [W.noisy_queries(raw, 1000, s, sd, sd + 100)[0] for s, sd in zip(wl["sigmas"], wl["test_seeds"])]
    q = np.concatenate(tests)
    qd = torch.from_numpy(q).cuda()
    ids, d = ix.search(qd, k=1, use_filters=False)
    return dict(pkg=pkg, wl=wl, raw=raw, ix=ix, calib=torch.from_numpy(c).cuda(), q=q, qd=qd,
                exact=(ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)))


def test_exact_search_sample_matches_oracle(rw1m):
    rows = np.random.default_rng(31).choice(len(rw1m["q"]), 24, replace=False)
    xs = O.znorm(rw1m["raw"])
    want_ids, want_d = O.knn(xs, O.znorm(rw1m["q"][rows]), 1)
    got_ids, got_d = rw1m["exact"][0][rows], rw1m["exact"][1][rows]
    assert np.all(np.abs(got_d[:, 0] - want_d[:, 0]) <= 1e-4 * np.maximum(want_d[:, 0], 1e-6))
    assert np.all((got_ids[:, 0] == want_ids[:, 0]) | (np.abs(got_d[:, 0] - want_d[:, 0]) <= 1e-5 * want_d[:, 0]))


@pytest.mark.parametrize("n_local", [0, 500])
def test_target_sweep(rw1m, n_local):
    ix, wl, qd = rw1m["ix"], rw1m["wl"], rw1m["qd"]
    rep = ix.train_filters(n_global=1500, n_local=n_local, noise_lo=wl["train_sigma"][0],
                           noise_hi=wl["train_sigma"][1], max_epochs=200, th_override=0.0, seed=wl["train_seed"])
    assert rep["n_filters"] > 0
    ix.calibrate(rw1m["calib"], [1], list(TARGETS))
    offs = ix.offsets().astype(np.float64)          # [targets, filters]
    assert np.all(np.diff(offs, axis=0) >= 0), "offsets must not decrease with the target"
    ex_ids, ex_d = rw1m["exact"]
    nc, nt = wl["n_calib"], len(rw1m["q"])
    rows = []
    for t, o in zip(TARGETS, offs):
        ids, d, st = ix.search(qd, k=1, target=t, use_filters=True, schedule=(1, 0), with_stats=True)
        ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
        hit = (ids[:, 0] == ex_ids[:, 0]) | (d[:, 0] <= ex_d[:, 0] * (1 + 3e-5))
        rec = float(hit.mean())
        band = 3.0 * np.sqrt(t * (1 - t)) * (1 / np.sqrt(nc) + 1 / np.sqrt(nt)) + 1.0 / nc
        rows.append((t, rec, st["series_scanned"], st["leaves_filter_pruned"]))
        assert rec >= t - band, (n_local, t, rec, band)
    print(f"\nn_local={n_local}: " + "; ".join(f"t={t}: recall {r:.4f}, series {s}, filter-pruned {f}"
                                             for t, r, s, f in rows))
    for (t0, r0, s0, f0), (t1, r1, s1, f1) in zip(rows, rows[1:]):
        assert s1 >= s0 and f1 <= f0 and r1 >= r0, (t0, t1)
