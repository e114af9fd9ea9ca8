"""The library's host algorithms -- tree build and leaf boxes (the DSTree-style
backbone), Algorithm 3's leaf selection and Algorithm 4's calibration -- built
for the CPU with AddressSanitizer and UndefinedBehaviorSanitizer (g++, no GPU
code) and run on seeded inputs whose expected results come from the oracle.

Inputs are computed by the oracle (segment statistics, visit orders, per-leaf
neighbours, filter predictions of seeded weights); the harness runs the
library's own C++ on them, so a memory error or undefined behaviour in that
code fails the test, and so does any disagreement with the oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_01836_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host", "harness.cpp")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    d = tmp_path_factory.mktemp("host")
    exe = d / "harness"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", CSRC, HARNESS, os.path.join(CSRC, "tree.cpp"), os.path.join(CSRC, "calib.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe, d


def _run(harness, mode, payload: bytes) -> bytes:
    exe, d = harness
    inp, outp = d / f"{mode}.in", d / f"{mode}.out"
    inp.write_bytes(payload)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe), mode, str(inp), str(outp)], capture_output=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr.decode(errors="replace")[-4000:]
    assert b"runtime error" not in r.stderr, r.stderr.decode(errors="replace")[-4000:]
    return outp.read_bytes()


def _tree(harness, mu, sd, m, cap, rule):
    n, S = mu.shape
    payload = (np.array([n], np.int64).tobytes() + np.array([S, m, cap, rule], np.int32).tobytes() +
               np.ascontiguousarray(mu, np.float32).tobytes() + np.ascontiguousarray(sd, np.float32).tobytes())
    out = _run(harness, "tree", payload)
    N = int(np.frombuffer(out[:8], np.int64)[0])
    off = np.frombuffer(out[8:8 + 8 * (N + 1)], np.int64)
    mem = np.frombuffer(out[8 + 8 * (N + 1): 8 + 8 * (N + 1) + 8 * n], np.int64)
    boxes = np.frombuffer(out[8 + 8 * (N + 1) + 8 * n:], np.float32).reshape(N, S, 4)
    return [mem[off[L]:off[L + 1]] for L in range(N)], boxes


@pytest.mark.parametrize("kind", ["median_rw", "midpoint_mixture"])
def test_tree_and_boxes_match_oracle(harness, kind):
    if kind == "median_rw":
        raw, m, cap, rule = W.random_walk(20000, 256, 1001), 256, 1000, "median"
    else:
        raw, m, cap, rule = W.gaussian_mixture(30000, 96, 40, 0.3, 41, 42), 96, 2000, "midpoint"
    xs = O.znorm(raw)
    mu, sd = O.segment_stats(xs, 16)
    leaves, boxes = _tree(harness, mu, sd, m, cap, {"median": 0, "midpoint": 1}[rule])
    want = O.build_tree(mu, sd, m, cap, rule)
    assert len(leaves) == len(want.leaves)
    for got, w in zip(leaves, want.leaves):
        assert np.array_equal(got, w)
    assert np.array_equal(boxes, O.leaf_boxes(mu, sd, want))


@pytest.mark.parametrize("n,m,cap", [(20000, 64, 100), (12000, 256, 40), (300000, 64, 200)])
def test_isax_tree_and_boxes_match_oracle(harness, n, m, cap):
    """The iSAX (MESSI) tree: partition, depth-first order and each leaf's
    SAX-interval box equal the oracle's (the library computes its own
    breakpoints from the normal CDF; the oracle takes scipy's quantiles)."""
    xs = O.znorm(W.random_walk(n, m, 1201))
    mu, sd = O.segment_stats(xs, 16)
    leaves, boxes = _tree(harness, mu, sd, m, cap, 2)
    want = O.build_isax_tree(mu, m, cap)
    assert len(leaves) == len(want.leaves)
    for got, w in zip(leaves, want.leaves):
        assert np.array_equal(got, w)
    assert np.array_equal(boxes, O.isax_boxes(want))


def test_tree_with_heavy_ties_matches_oracle(harness):
    """Quantised statistics (many equal values): the median split's (value, id)
    order decides; a capacity of 1 splits down to single series."""
    rng = np.random.default_rng(3)
    mu = (np.round(rng.normal(size=(3000, 4)) * 4) / 4).astype(np.float32)
    sd = (np.round(np.abs(rng.normal(size=(3000, 4))) * 2) / 2).astype(np.float32)
    for cap, rule in [(7, "median"), (100, "midpoint"), (1, "median")]:
        leaves, _ = _tree(harness, mu, sd, 32, cap, {"median": 0, "midpoint": 1}[rule])
        want = O.build_tree(mu, sd, 32, cap, rule)
        assert [list(x) for x in leaves] == [list(x) for x in want.leaves], (cap, rule)


def test_selection_matches_oracle(harness):
    rng = np.random.default_rng(8)
    sizes = rng.integers(1, 50, 300).astype(np.int64)   # many equal sizes: ties by leaf id
    for th, w, cM in [(0.0, 1.0, 1e9), (20.0, 3.0, 100.0), (25.5, 1.0, 40.0), (60.0, 1.0, 1e9), (0.0, 5.0, 4.0)]:
        payload = np.array([len(sizes)], np.int64).tobytes() + np.array([th, w, cM], np.float64).tobytes() + \
            sizes.tobytes()
        out = _run(harness, "select", payload)
        c = int(np.frombuffer(out[:8], np.int64)[0])
        got = np.frombuffer(out[8:8 + 4 * c], np.int32)
        assert list(got) == list(O.select_leaves(sizes, th, w, cM)), (th, w, cM)


@pytest.fixture(scope="module")
def calib_case():
    """Oracle inputs of Algorithm 4 on 20k random walks (32 leaves), seeded
    filters on 24 of the leaves, 120 calibration queries."""
    raw = W.random_walk(20000, 256, 1001)
    xs = O.znorm(raw)
    mu, sd = O.segment_stats(xs, 16)
    tree = O.build_tree(mu, sd, 256, 1000, "median")
    N = len(tree.leaves)
    cq, _, _ = W.noisy_queries(raw, 120, (0.05, 0.2), 61, 62)
    cqs = O.znorm(cq)
    qmu, qsd = O.query_stats(cqs, 16)
    order = O.visit_order(O.lower_bound(qmu, qsd, O.leaf_boxes(mu, sd, tree), 256))
    ld, li = O.leaf_knn(xs, tree.leaves, cqs, 3)
    leaves = np.arange(0, N, 4).tolist() + np.arange(1, N, 2).tolist()[:16]  # 24 filtered leaves
    h = 32
    w = W.mlp_weights(len(leaves), 256, h, seed=99, out_bias=6.0)
    df32 = np.stack([O.mlp_forward(w[f], cqs, 256, h) for f in range(len(leaves))], 1).astype(np.float32)
    leaf_of = np.empty(len(xs), dtype=np.int64)
    for L, mem in enumerate(tree.leaves):
        leaf_of[mem] = L
    return dict(N=N, order=order, ld=ld, li=li, leaves=np.array(leaves, np.int32), df32=df32, leaf_of=leaf_of,
                xs=xs, cqs=cqs)


@pytest.mark.parametrize("mapping", ["step", "steffen"])
@pytest.mark.parametrize("corrected", [True, False])
def test_calibration_matches_oracle(harness, calib_case, mapping, corrected):
    c = calib_case
    nc, N, F, kmax = len(c["cqs"]), c["N"], len(c["leaves"]), 3
    targets = np.array([0.5, 0.8, 0.9, 0.95, 0.99, 1.0], np.float32)
    # the oracle's curve over all leaves (+inf where a leaf has no filter)
    has = np.zeros(N, dtype=bool)
    has[c["leaves"]] = True
    dfull = np.zeros((nc, N))
    dfull[:, c["leaves"]] = c["df32"].astype(np.float64)
    for k in (1, 3):
        payload = (np.array([nc, N, F, kmax, k, len(targets), {"step": 0, "steffen": 1}[mapping], int(corrected)],
                            np.int32).tobytes() +
                   np.ascontiguousarray(c["order"], np.int32).tobytes() +
                   np.ascontiguousarray(c["ld"], np.float64).tobytes() +
                   np.ascontiguousarray(c["li"], np.int64).tobytes() + c["df32"].tobytes() + c["leaves"].tobytes() +
                   targets.tobytes())
        got = np.frombuffer(_run(harness, "calib", payload), np.float32).reshape(len(targets), F)
        dbsf = O.bsf_before(c["ld"], c["order"], k)
        ids, _ = O.knn(c["xs"], c["cqs"], k)
        offs, q = O.autotune_curve(dfull, c["ld"][:, :, 0], dbsf, c["leaf_of"][ids], has)
        for b, t in enumerate(targets):
            if mapping == "step":
                _, want = O.step_offsets(offs, q, float(t), nc, corrected)
            else:
                want = O.steffen_offsets(offs, q, float(t), nc, corrected)
            want = want[c["leaves"]]
            assert np.array_equal(np.isinf(got[b]), np.isinf(want)), (k, t)
            fin = np.isfinite(want)
            assert np.allclose(got[b][fin], want[fin], rtol=1e-6, atol=1e-7), (k, t)
