"""Benchmark of the LeaFi hot path on one MI355X.

Default workload (the serving configuration, rw50m): 50,000,000 random-walk
series of length 256 generated on the GPU (fp32; the library keeps them
z-normalised as fp32 plus a bf16 copy, about 77 GB resident), leaf capacity
10,000 (8,192 leaves), one 256->256->1 ReLU MLP filter per selected leaf
trained on 1,500 global + 500 local noisy queries per filter, conformal
calibration on 500 held-out queries for k in {1, 10, 100} x recall targets
{0.90, 0.95, 0.99}.  Test queries are collection series plus N(0, 0.1^2)
noise (relative to the z-normalised series), each with its own k and target
drawn uniformly from those classes.

A step is one batched search of 1,024 such queries (mixed k and targets)
through the whole search path: z-normalisation, summary bounds, visit order,
filter inference, the round schedule of prune / leaf scan (BF16 MFMA) /
rerank (FP32, FP64 band) / merge, and the output.  Index build, training and
calibration happen before the timed region; inputs are resident in HBM when
timing starts.  Beside the steps: the serving engine under Poisson arrivals
(p50/p99 from arrival to completion per offered rate), the same batches with
filters off (exact search), the plain FP32 per-query path, and the FP64 CPU
oracle on a bounded sample, whose exact answers also give recall per class.

Other workloads (`--workload`): rw1m, the 1M x 256 learned-filter
configuration (k = 1, target 0.99, three batches of 1,000 queries at noise
0.05/0.1/0.2); rw10m, the 10M x 256 precision configuration (k = 10, target
0.99, three batches of 1,024 queries at those noise levels); gm25m, 25M
length-96 Gaussian-mixture series with ragged leaves (four batches of 4,096
queries at noise 0.1, k in {1, 10, 50}, target 0.99); rw50m_isax, the default
collection and queries in an iSAX tree.  Those are generated on the host.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/sec + p50/p99 latency at recall@k≥0.99; leaf-scan HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense bf16 matrix-core peak of one MI355X


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


SCAN_SOURCES = ("k_scan.hip", "scan_bounds.h")


def scan_source_digest():
    """SHA-256 over the BF16 scan kernel's own sources, in order."""
    h = hashlib.sha256()
    for name in SCAN_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2502_01836_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per scan dispatch from the committed counter summary of this
    workload, if it was taken with the scan sources as they are now (else None)."""
    summ = os.path.join(ROOT, "profiles", f"scan_bf16_{workload}_traffic.md")
    try:
        text = open(summ).read()
        digest = scan_source_digest()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_", "k_scan_")))
    if vals.get("k_scan_sha256", "").strip() != digest:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def make_collection(wl, dev):
    """Raw collection on the device, and a factory of host chunks (first row,
    raw fp32 rows) for the CPU oracle."""
    import torch
    import workloads as W
    n, m = wl["n"], wl["m"]
    if wl["kind"] == "random_walk_device":
        raw_d = W.random_walk_device(n, m, wl["seed"], device=dev)

        def chunks(gen_time):
            for lo, hi, x in W.random_walk_device_chunks(n, m, wl["seed"], device=dev):
                t = time.perf_counter()
                h = x.cpu().numpy()
                gen_time[0] += time.perf_counter() - t
                yield lo, h
        return raw_d, None, chunks
    if wl["kind"] == "gaussian_mixture":
        raw = W.gaussian_mixture(n, m, wl["n_comp"], wl["spread"], wl["seed_means"], wl["seed_members"])
    else:
        raw = W.random_walk(n, m, wl["seed"])

    def chunks(gen_time):
        step = 1 << 20
        for lo in range(0, n, step):
            yield lo, raw[lo:lo + step]
    return torch.from_numpy(raw).to(dev), raw, chunks


def make_queries(wl, raw_d, raw):
    """Calibration queries, the test batches and each test query's (k, target)."""
    import torch
    import workloads as W
    dev = raw_d.device
    ks = tuple(wl.get("ks", (wl.get("k", 1),)))
    targets = tuple(wl.get("targets", (wl.get("target", 0.99),)))
    nq = wl["nq"]
    if raw is None:
        calib, _, _ = W.noisy_queries_device(raw_d, wl["n_calib"], tuple(wl["train_sigma"]), wl["calib_seed"])
        n_batches = 4
        pool, _, _ = W.noisy_queries_device(raw_d, n_batches * nq, wl["sigma"], wl["test_seed"])
        batches = [pool[i * nq:(i + 1) * nq].contiguous() for i in range(n_batches)]
        sig_desc = f"noise {wl['sigma']}"
    else:
        c, _, _ = W.noisy_queries(raw, wl["n_calib"], tuple(wl["train_sigma"]), wl["calib_seed"], wl["calib_seed"] + 100)
        calib = torch.from_numpy(c).to(dev)
        batches = []
        if "sigmas" in wl:
            # one batch per noise level
            seeds = wl.get("test_seeds") or tuple(wl["test_seed"] + i for i in range(len(wl["sigmas"])))
            for s, sd in zip(wl["sigmas"], seeds):
                q, _, _ = W.noisy_queries(raw, nq, s, sd, sd + 100)
                batches.append(torch.from_numpy(q).to(dev))
            sig_desc = "noise " + "/".join(str(s) for s in wl["sigmas"])
        else:
            # four batches at one noise level
            for i in range(4):
                sd = wl["q_seed"] + 1000 * i
                q, _, _ = W.noisy_queries(raw, nq, wl["sigma"], sd, sd + 100)
                batches.append(torch.from_numpy(q).to(dev))
            sig_desc = f"noise {wl['sigma']}"
    rng = np.random.default_rng(wl.get("mix_seed", 0))
    classes = [(k, t) for k in ks for t in targets]
    cls = [rng.integers(0, len(classes), nq) for _ in batches]
    kb = [np.array([classes[c][0] for c in cb], dtype=np.int32) for cb in cls]
    tb = [np.array([classes[c][1] for c in cb], dtype=np.float32) for cb in cls]
    return calib, batches, kb, tb, ks, targets, sig_desc


def recall_rows(got_ids, got_d, want_ids, want_d, k):
    """recall@k per query against exact answers (ids, FP64 or exact distances):
    a returned item is a hit if it is one of the k exact ids or exactly as
    close as the k-th (a tie, within 3e-5 relative)."""
    out = np.empty(len(got_ids))
    for a in range(0, len(got_ids), 2048):
        g, gd = got_ids[a:a + 2048, :k], got_d[a:a + 2048, :k]
        w = want_ids[a:a + 2048, :k]
        kth = want_d[a:a + 2048, k - 1:k]
        hit = (g[:, :, None] == w[:, None, :]).any(-1) | (np.isfinite(gd) & (gd <= kth * (1 + 3e-5)))
        out[a:a + 2048] = hit.sum(1) / k
    return out


ABLATION_TARGETS = (0.95, 0.97, 0.99, 0.995, 0.999)


def ablation(workloads, a):
    """Local training data off and on (n_local 0 / 500) x recall targets
    0.95 ... 0.999, per workload: training and calibration as in the
    benchmark, then every test batch searched at one target for all its
    queries (k = the workload's first k).  Per row: queries/s (best of three
    passes over the batches), recall against the exact (filters-off) search,
    series pruned and leaves pruned by filters.  One JSON line."""
    import torch
    import workloads as W
    import paper_2502_01836_amd as pkg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pkg.load()
    dev = torch.device("cuda:0")
    sched = tuple(int(x) for x in a.schedule.split(","))
    out = []
    for name in workloads:
        wl = W.WORKLOADS[name]
        n, m = wl["n"], wl["m"]
        t0 = time.time()
        raw_d, raw, _ = make_collection(wl, dev)
        calib, batches, _, _, ks, _, sig_desc = make_queries(wl, raw_d, raw)
        ix = pkg.Index()
        ix.build(raw_d, leaf_capacity=wl["capacity"], n_segments=wl.get("segments", 16),
                 split_rule=wl.get("split", "median"))
        del raw_d, raw
        torch.cuda.empty_cache()
        k = int(ks[0])
        exact = []
        for q in batches:
            ids, d = ix.search(q, k=k, use_filters=False, schedule=sched)
            exact.append((ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)))
        log(f"ablation {name}: data, index and exact answers in {time.time() - t0:.1f}s")
        for n_local in (0, 500):
            rep = ix.train_filters(n_global=1500, n_local=n_local, noise_lo=wl["train_sigma"][0],
                                   noise_hi=wl["train_sigma"][1], a=2.0, max_epochs=a.max_epochs,
                                   seed=wl["train_seed"])
            ix.calibrate(calib, [k], list(ABLATION_TARGETS))
            for t in ABLATION_TARGETS:
                got, st_all = [], []
                for q in batches:
                    ids, d, st = ix.search(q, k=k, target=t, use_filters=True, schedule=sched, with_stats=True)
                    got.append((ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)))
                    st_all.append(st)
                best = None
                for _ in range(3):
                    torch.cuda.synchronize()
                    s0 = time.perf_counter()
                    for q in batches:
                        ix.search(q, k=k, target=t, use_filters=True, schedule=sched)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - s0
                    best = dt if best is None else min(best, dt)
                nq_all = sum(len(q) for q in batches)
                rec = float(np.concatenate([recall_rows(g[0], g[1], e[0], e[1], k)
                                            for g, e in zip(got, exact)]).mean())
                pruned = 1.0 - sum(s["series_scanned"] for s in st_all) / (nq_all * n)
                row = {"workload": name, "local": n_local > 0, "n_local": n_local, "n_filters": rep["n_filters"],
                       "k": k, "target": t, "recall_vs_exact_search": rec, "target_met": rec >= t,
                       "queries_per_s": nq_all / best, "series_pruning_ratio": pruned,
                       "leaves_filter_pruned": int(sum(s["leaves_filter_pruned"] for s in st_all)),
                       "queries": nq_all}
                out.append(row)
                log(f"ablation {name} {'+' if n_local else '-'}Local target {t}: recall {rec:.4f}, "
                    f"{row['queries_per_s']:.0f} queries/s, series pruned {pruned:.4f}")
        del ix
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "recall and queries/s per recall target, without and with local training data",
                      "unit": "queries/s", "data": "synthetic", "n_gpus": 1, "schedule": list(sched),
                      "rows": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rw50m")
    ap.add_argument("--cpu-sample", type=int, default=48, help="queries timed on the CPU oracle (0 = skip)")
    ap.add_argument("--fp32-sample", type=int, default=256, help="queries of the plain FP32 per-query path (0 = skip)")
    ap.add_argument("--schedule", default="1,0")
    ap.add_argument("--max-epochs", type=int, default=1000)
    ap.add_argument("--serve-rates", default=None,
                    help="offered request rates (per second) of the serving leg; empty = skip")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-mem-gb", type=float, default=32.0, help="serving engine's memory budget for request slots")
    ap.add_argument("--tiling", default="",
                    help="BF16 scan tile shape 'rows,queries' to use instead of the tuner's pick")
    ap.add_argument("--cpu-one-core-rows", type=int, default=4_000_000,
                    help="collection rows the one-thread oracle sample scans (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy first (reference for hardware byte counters)")
    ap.add_argument("--ablation", default="",
                    help="instead of the benchmark: the local-data ablation and recall-target sweep on these "
                         "workloads (comma-separated, e.g. rw1m,rw10m); prints its own JSON line")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU layout is a design "
              "note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if a.ablation:
        ablation([w for w in a.ablation.split(",") if w], a)
        return

    import torch
    import workloads as W
    import paper_2502_01836_amd as pkg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pkg.load()
    wl = W.WORKLOADS[a.workload]
    n, m = wl["n"], wl["m"]
    dev = torch.device("cuda:0")
    if a.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t0 = time.time()
    raw_d, raw, host_chunks = make_collection(wl, dev)
    calib, batches, kb, tb, ks, targets, sig_desc = make_queries(wl, raw_d, raw)
    torch.cuda.synchronize()
    log(f"generated {n}x{m} and {len(batches)} batches of {wl['nq']} queries in {time.time() - t0:.1f}s")

    ix = pkg.Index()
    t0 = time.time()
    ix.build(raw_d, leaf_capacity=wl["capacity"], n_segments=wl.get("segments", 16),
             split_rule=wl.get("split", "median"))
    torch.cuda.synchronize()
    t_build = time.time() - t0
    info = ix.info()
    log(f"built index: {info['n_leaves']} leaves, {info['device_bytes'] / 1e9:.1f} GB resident, in {t_build:.1f}s")
    del raw_d
    torch.cuda.empty_cache()
    t0 = time.time()
    rep = ix.train_filters(n_global=1500, n_local=500, noise_lo=wl["train_sigma"][0], noise_hi=wl["train_sigma"][1],
                           a=2.0, max_epochs=a.max_epochs, seed=wl["train_seed"])
    t_train = time.time() - t0
    log(f"trained {rep['n_filters']} filters in {t_train:.1f}s (th={rep['th']:.1f}, collect {rep['ms_collect']:.0f} ms, "
        f"sgd {rep['ms_train']:.0f} ms, epochs<={rep['epochs_max_run']}, val mse {rep['mean_val_mse']:.3f})")
    t0 = time.time()
    ix.calibrate(calib, list(ks), list(targets))
    torch.cuda.synchronize()
    t_cal = time.time() - t0
    log(f"calibrated {len(ks)}x{len(targets)} (k, target) pairs in {t_cal:.1f}s")
    del calib

    sched = tuple(int(x) for x in a.schedule.split(","))
    nq = wl["nq"]
    k_max = max(ks)
    kd = [torch.from_numpy(k).to(dev) for k in kb]
    td = [torch.from_numpy(t).to(dev) for t in tb]
    out = (torch.empty((nq, k_max), dtype=torch.int64, device=dev),
           torch.empty((nq, k_max), dtype=torch.float32, device=dev))

    # exact answers (filters off, the same batches): the library's exact search,
    # itself checked against the FP64 oracle by the parity tests and below
    exact, exact_st = [], []
    for q, k_, t_ in zip(batches, kd, td):
        ids, d, st = ix.search(q, k=k_, target=t_, k_max=k_max, use_filters=False, schedule=sched, with_stats=True)
        exact.append((ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)))
        exact_st.append(st)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for q, k_, t_ in zip(batches, kd, td):
        ix.search(q, k=k_, target=t_, k_max=k_max, use_filters=False, schedule=sched, out=out)
    torch.cuda.synchronize()
    exact_qps = len(batches) * nq / (time.perf_counter() - s0)
    log(f"exact search (filters off): {exact_qps:.0f} queries/s")

    # scan tile shape: the library's tuner on each batch, smallest summed time
    # kept (or the shape given on the command line)
    t0 = time.time()
    if a.tiling:
        best = tuple(int(v) for v in a.tiling.split(","))
        ix.set_tiling(*best)
        tune = {"candidates": [], "chosen": {"chunk_rows": best[0], "queries_per_tile": best[1]}, "given": True}
        log(f"scan tiles set to {best}")
    else:
        tot = {}
        for q, k_, t_ in zip(batches, kd, td):
            rep_t = ix.autotune(q, k=k_, target=t_, k_max=k_max, use_filters=True, schedule=sched, repeats=3)
            for c in rep_t["candidates"]:
                key = (c["chunk_rows"], c["queries_per_tile"])
                tot[key] = tot.get(key, 0.0) + c["ms"]
        best = min(tot, key=tot.get)
        ix.set_tiling(*best)
        tune = {"candidates": [{"chunk_rows": c, "queries_per_tile": q_, "ms_sum_of_batches": v}
                               for (c, q_), v in sorted(tot.items())],
                "chosen": {"chunk_rows": best[0], "queries_per_tile": best[1], "ms_sum_of_batches": tot[best]}}
        log(f"tuned scan tiles in {time.time() - t0:.1f}s: {best} of "
            f"{[(c, q_, round(v, 3)) for (c, q_), v in sorted(tot.items())]}")

    # bound searches (arguments marshalled once); the timed steps use the
    # library's default execution (a repeated plannable batch shape replays a
    # captured graph, else host-driven rounds); the roofline pass asks for
    # statistics (scan kernels timed by HIP events on their stream)
    gbound = [ix.searcher(q, k_, t_, out, k_max=k_max, use_filters=True, schedule=sched)
              for q, k_, t_ in zip(batches, kd, td)]
    sbound = [ix.searcher(q, k_, t_, out, k_max=k_max, use_filters=True, schedule=sched, flags=1, with_stats=True)
              for q, k_, t_ in zip(batches, kd, td)]
    nb = len(batches)
    for i in range(2 * nb):
        gbound[i % nb]()
    for i in range(a.warmup):
        gbound[i % nb]()
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for i in range(a.steps):
        s0 = time.perf_counter()
        gbound[i % nb]()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
    t_total = time.perf_counter() - t_start
    qps = a.steps * nq / t_total
    ms_per_step = 1e3 * t_total / a.steps
    log(f"timed {a.steps} steps: {qps:.0f} queries/s, {ms_per_step:.2f} ms per batch")

    t_scan_ms, t_scan_bytes, t_scans, t_series, paths, stats_all = 0.0, 0.0, 0, 0, set(), []
    for i in range(a.warmup):
        sbound[i % nb]()
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for i in range(a.steps):
        st = sbound[i % nb]()
        t_scan_ms += st["ms_scan"]
        t_scan_bytes += st["scan_bytes"]
        t_scans += st["rounds"]
        t_series += st["series_scanned"]
        paths.add(st["path"])
        if i < nb:
            stats_all.append(st)
    stats_qps = a.steps * nq / (time.perf_counter() - p0)
    achieved = t_scan_bytes / (t_scan_ms * 1e-3) / 1e9 if t_scan_ms > 0 else 0.0
    # the same launches as matrix-core work: 2m flops per (query, series)
    # pair the regular rounds scanned
    t_scan_flops = 2.0 * m * t_series
    scan_tflops = t_scan_flops / (t_scan_ms * 1e-3) / 1e12 if t_scan_ms > 0 else 0.0
    log(f"roofline pass: {stats_qps:.0f} queries/s, scan {achieved:.0f} GB/s and {scan_tflops:.0f} TFLOP/s, "
        f"paths {sorted(paths)}")

    # results of each batch (filters on) and recall against the exact search
    got = []
    for i in range(nb):
        ids, d = ix.search(batches[i], k=kd[i], target=td[i], k_max=k_max, use_filters=True, schedule=sched)
        got.append((ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)))
    rec_exact = {}
    for k_ in ks:
        for t_ in targets:
            vals = []
            for i in range(nb):
                sel = (kb[i] == k_) & (tb[i] == np.float32(t_))
                if sel.any():
                    vals.append(recall_rows(got[i][0][sel], got[i][1][sel], exact[i][0][sel], exact[i][1][sel], k_))
            if vals:
                rec_exact[f"k{k_}_t{t_:.2f}"] = float(np.concatenate(vals).mean())
    n_series = n * nq
    pruned = 1.0 - sum(s["series_scanned"] for s in stats_all) / (len(stats_all) * n_series)
    pruned_exact = 1.0 - sum(s["series_scanned"] for s in exact_st) / (len(exact_st) * n_series)
    st0 = stats_all[0]
    log(f"batch 0: leaves scanned {st0['leaves_scanned']}, bound-pruned {st0['leaves_lb_pruned']}, "
        f"filter-pruned {st0['leaves_filter_pruned']}, filters evaluated {st0['filter_evals']}, "
        f"rescans {st0['fallback_items']}; series pruned {pruned:.4f} (exact search {pruned_exact:.4f})")

    # plain FP32 per-query path: one query per launch sequence (the library
    # loops over the queries), same filters, calibration and query mix; a
    # warm-up call over the whole sample first, then the timed call
    fp32 = None
    if a.fp32_sample > 0:
        ns = min(a.fp32_sample, nq)
        qs, ks_, ts_ = batches[1][:ns].contiguous(), kd[1][:ns].contiguous(), td[1][:ns].contiguous()
        ix.search(qs, k=ks_, target=ts_, k_max=k_max, use_filters=True, schedule=sched, scan="fp32")
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        ix.search(qs, k=ks_, target=ts_, k_max=k_max, use_filters=True, schedule=sched, scan="fp32")
        torch.cuda.synchronize()
        fp32 = ns / (time.perf_counter() - s0)
        log(f"plain FP32 per-query path: {fp32:.0f} queries/s ({ns} queries)")

    # serving leg: Poisson arrivals of single requests with mixed k and targets
    serving = []
    rates = [float(r) for r in (a.serve_rates if a.serve_rates is not None else
                                ",".join(str(r) for r in wl.get("rates", (50000, 100000, 200000, 400000)))).split(",")
             if r.strip()]
    pool = np.concatenate([b.cpu().numpy() for b in batches])
    pool_k, pool_t = np.concatenate(kb), np.concatenate(tb)
    served = {}  # pool index -> (ids, dists) of its last served request with the pool's own (k, target)
    if rates:
        ex_ids = np.concatenate([e[0] for e in exact])
        ex_d = np.concatenate([e[1] for e in exact])
        sv = pkg.Server(ix, k_max=k_max, max_slots=4096, schedule=sched, mem_budget=int(a.serve_mem_gb * 2 ** 30))
        log(f"serving engine: {sv.slots} request slots")
        try:
            rng = np.random.default_rng(wl.get("mix_seed", 0) + 1)
            for lam in rates:
                nreq = int(min(lam * a.serve_seconds, 200_000))
                pick = rng.integers(0, len(pool), nreq)
                arr = np.cumsum(rng.exponential(1.0 / lam, nreq))
                ids_r, d_r, lat_r, rep_r = sv.replay(pool[pick], arr, pool_k[pick], pool_t[pick])
                rec = {}
                for k_ in ks:
                    for t_ in targets:
                        sel = (pool_k[pick] == k_) & (pool_t[pick] == np.float32(t_))
                        if sel.any():
                            r_ = recall_rows(ids_r[sel], d_r[sel].astype(np.float64), ex_ids[pick[sel]],
                                             ex_d[pick[sel]], k_)
                            rec[f"k{k_}_t{t_:.2f}"] = float(r_.mean())
                for j, p in enumerate(pick):
                    served[int(p)] = (ids_r[j], d_r[j].astype(np.float64))
                serving.append({"offered_qps": lam, "requests": nreq,
                                "achieved_qps": nreq / rep_r["wall_s"],
                                "p50_ms": float(np.percentile(lat_r, 50)), "p99_ms": float(np.percentile(lat_r, 99)),
                                "mean_active": rep_r["mean_active"], "max_active": rep_r["max_active"],
                                "rounds": rep_r["rounds"], "recall_vs_exact_search": rec})
                log(f"serving {lam:.0f}/s: {serving[-1]['achieved_qps']:.0f}/s p50 {serving[-1]['p50_ms']:.2f} ms "
                    f"p99 {serving[-1]['p99_ms']:.2f} ms, mean active {rep_r['mean_active']:.0f}")
        finally:
            sv.close()

    # CPU oracle (FP64 brute force, all host threads) on a bounded sample; its
    # exact answers give the recall of the batched and the served results
    cpu, rec_oracle = None, None
    if a.cpu_sample > 0:
        import oracle as O
        rs = np.random.default_rng(17).choice(len(pool), a.cpu_sample, replace=False)
        gen_time = [0.0]
        s0 = time.perf_counter()
        o_ids, o_d = O.knn_stream(host_chunks(gen_time), O.znorm(pool[rs]), k_max)
        dt = time.perf_counter() - s0 - gen_time[0]
        cpu = {"value": a.cpu_sample / dt, "unit": "queries/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"{a.cpu_sample} test queries, FP64 brute-force exact {k_max}-NN over all {n} series "
                         f"(z-normalised chunk by chunk)",
               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        log(f"CPU oracle: {cpu['value']:.2f} queries/s on {cpu['cores']} threads ({dt:.1f}s)")
        if a.cpu_one_core_rows > 0:
            # the same oracle on one thread, over the collection's first rows;
            # its time scales linearly with the rows scanned, so the rate over
            # the whole collection is the sample's rate times rows / n
            rows = min(a.cpu_one_core_rows, n)
            n1 = min(4, a.cpu_sample)
            threads = O.num_threads()
            O.set_num_threads(1)
            try:
                gen1 = [0.0]

                def first_rows(gt):
                    for lo, h in host_chunks(gt):
                        if lo >= rows:
                            break
                        yield lo, h[:rows - lo]
                s1 = time.perf_counter()
                O.knn_stream(first_rows(gen1), O.znorm(pool[rs[:n1]]), k_max)
                dt1 = time.perf_counter() - s1 - gen1[0]
            finally:
                O.set_num_threads(threads)
            cpu["one_core"] = {"value": n1 / dt1 * rows / n, "unit": "queries/s", "cores": 1,
                               "sample": f"{n1} of those queries over the first {rows} series ({dt1:.1f} s), "
                                         f"rate scaled by {rows}/{n} to the whole collection"}
            log(f"CPU oracle on one thread: {cpu['one_core']['value']:.3f} queries/s ({dt1:.1f}s for {rows} rows)")
        g_ids = np.concatenate([g[0] for g in got])[rs]
        g_d = np.concatenate([g[1] for g in got])[rs]
        rec_oracle = {"batched": {}, "served": {}}
        for k_ in ks:
            for t_ in targets:
                sel = (pool_k[rs] == k_) & (pool_t[rs] == np.float32(t_))
                if sel.any():
                    key = f"k{k_}_t{t_:.2f}"
                    r_ = recall_rows(g_ids[sel], g_d[sel], o_ids[sel], o_d[sel], k_)
                    rec_oracle["batched"][key] = {"recall": float(r_.mean()), "queries": int(sel.sum())}
                    sv_rows = [(i, served[int(p)]) for i, p in enumerate(rs) if sel[i] and int(p) in served]
                    if sv_rows:
                        si = np.array([i for i, _ in sv_rows])
                        r_s = recall_rows(np.stack([v[0] for _, v in sv_rows]), np.stack([v[1] for _, v in sv_rows]),
                                          o_ids[si], o_d[si], k_)
                        rec_oracle["served"][key] = {"recall": float(r_s.mean()), "queries": len(si)}
        # the exact search (filters off) against the oracle: largest relative
        # distance error over each sampled query's k results
        e_d = np.concatenate([e[1] for e in exact])[rs]
        errs = [np.max(np.abs(e_d[i, :pool_k[r]] - o_d[i, :pool_k[r]]) / o_d[i, :pool_k[r]])
                for i, r in enumerate(rs)]
        rec_oracle["exact_search_max_rel_err"] = float(np.max(errs))

    lat_ms = np.array(lat) * 1e3
    kind_desc = ("Gaussian-mixture series ({} components, spread {})".format(wl["n_comp"], wl["spread"])
                 if wl["kind"] == "gaussian_mixture" else "random walks")
    line = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {n} {kind_desc} x {m}, "
                               f"{'iSAX tree of ' + str(wl['segments']) + ' segments, ' if wl.get('split') == 'isax' else ''}"
                               f"leaf capacity {wl['capacity']}, "
                               f"{info['n_leaves']} leaves, {rep['n_filters']} MLP filters {m}->{m}->1; batches of "
                               f"{nq} queries ({sig_desc}), each with k in {list(ks)} and recall target in "
                               f"{list(targets)}",
                   "schedule": list(sched), "n_leaves": info["n_leaves"], "resident_gb": info["device_bytes"] / 1e9},
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "latency_of": "one batch of the timed steps (the serving entries give request latencies)",
        "recall_vs_exact_search": rec_exact,
        "recall_vs_oracle": rec_oracle,
        "series_pruning_ratio": pruned,
        "series_pruning_ratio_exact_search": pruned_exact,
        "exact_search_qps": exact_qps,
        "speedup_vs_exact_search": qps / exact_qps,
        "fp32_plain_qps": fp32,
        "speedup_vs_fp32_plain": (qps / fp32) if fp32 else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(a.workload),
                     "kernel": "k_scan_bf16", "launches": t_scans,
                     "avg_launch_us": 1e3 * t_scan_ms / max(t_scans, 1),
                     "bytes_per_launch": t_scan_bytes / max(t_scans, 1),
                     "bytes_are": "unique leaf rows (real series, no padding) x (2m + 4) per round",
                     "scan_ms_per_step": t_scan_ms / a.steps, "scan_bytes_per_step": t_scan_bytes / a.steps},
        "scan_mfma": {"achieved": scan_tflops, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": scan_tflops / BF16_MFMA_PEAK_TFLOPS, "kernel": "k_scan_bf16",
                      "flops_are": "2m per (query, series) pair the regular rounds scanned (real series)",
                      "flops_per_step": t_scan_flops / a.steps},
        "search_paths": {"timed_steps": "default execution", "roofline_pass": sorted(paths)},
        "roofline_pass_qps": stats_qps,
        "scan_tiling": tune,
        "cpu_baseline": cpu,
        "serving": serving,
        "setup_s": {"build": t_build, "train": t_train, "calibrate": t_cal,
                    "collect_ms": rep["ms_collect"], "sgd_ms": rep["ms_train"]},
        "train": {"n_filters": rep["n_filters"], "th": rep["th"], "epochs_max_run": rep["epochs_max_run"],
                  "mean_val_mse": rep["mean_val_mse"]},
        "search_stats": st0,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
