"""leafi_search_knn_noalloc (the search for callers that cannot allocate)
against leafi_search_knn through the C ABI: bit-identical results on two calls
in a row, the second with a smaller batch; nothing allocated by the call;
an oversized batch rejected before anything runs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu


def _pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    return pkg


def test_noalloc_search_equals_search_on_two_calls():
    pkg = _pkg()
    wl = W.WORKLOADS["rw20k"]
    raw = W.random_walk(wl["n"], wl["m"], wl["seed"])
    alloc = pkg.TorchAllocator()
    ix = pkg.Index(allocator=alloc).build(torch.from_numpy(raw).cuda(), leaf_capacity=wl["capacity"], n_segments=16)
    N, m, h = ix.info()["n_leaves"], wl["m"], 64
    wts = W.mlp_weights(N, m, h, seed=99, out_bias=6.0)
    offs = np.random.default_rng(5).uniform(0.0, 5.0, size=(2, N)).astype(np.float32)
    ix.set_filters(np.arange(N, dtype=np.int32), torch.from_numpy(wts).cuda(), h)
    ix.set_offsets([3, 10], [0.9], offs)
    q, _, _ = W.noisy_queries(raw, 300, 0.2, 31, 32)
    for nq, k_max, sched in [(300, 10, (1, 0)), (37, 3, (2, 0))]:
        qd = torch.from_numpy(q[:nq]).cuda()
        # k cycles over 1, 3, 10 (clamped to k_max): k = 1 is not calibrated and runs exact
        kd = torch.from_numpy(np.minimum(np.resize(np.array([1, 3, 10], dtype=np.int32), nq), k_max)).cuda()
        td = torch.full((nq,), 0.9, dtype=torch.float32, device="cuda")
        ids, d = ix.search(qd, k=kd, target=td, k_max=k_max, use_filters=True, schedule=sched)
        out = (torch.full((nq, k_max), -7, dtype=torch.int64, device="cuda"),
               torch.full((nq, k_max), -7.0, dtype=torch.float32, device="cuda"))
        torch.cuda.synchronize()
        live, torch_bytes = alloc.live_bytes, torch.cuda.memory_allocated()
        ix.search_noalloc(qd, kd, td, out, k_max=k_max, use_filters=True, schedule=sched)
        torch.cuda.synchronize()
        assert alloc.live_bytes == live and torch.cuda.memory_allocated() == torch_bytes  # nothing allocated
        assert torch.equal(out[0], ids) and torch.equal(out[1], d), (nq, k_max)
    # the handle's own workspace is intact: the ordinary search still runs
    ids2, d2 = ix.search(qd, k=kd, target=td, k_max=k_max, use_filters=True, schedule=sched)
    assert torch.equal(ids2, ids) and torch.equal(d2, d)


def test_noalloc_rejects_what_does_not_fit_or_plan():
    pkg = _pkg()
    raw = W.random_walk(20000, 256, 1001)
    ix = pkg.Index().build(torch.from_numpy(raw).cuda(), leaf_capacity=1000, n_segments=16)
    nq = 50000  # its candidate lists alone need more than the fixed scratch area
    qd = torch.zeros((nq, 256), dtype=torch.float32, device="cuda")
    kd = torch.full((nq,), 10, dtype=torch.int32, device="cuda")
    td = torch.ones((nq,), dtype=torch.float32, device="cuda")
    out = (torch.empty((nq, 10), dtype=torch.int64, device="cuda"),
           torch.empty((nq, 10), dtype=torch.float32, device="cuda"))
    with pytest.raises(pkg.LeafiError) as e:
        ix.search_noalloc(qd, kd, td, out, k_max=10, use_filters=False)
    assert e.value.code == -1 and "bytes of scratch" in str(e.value)
    with pytest.raises(pkg.LeafiError) as e:  # an open-ended schedule cannot be planned
        ix.search_noalloc(qd[:8], kd[:8], td[:8], (out[0][:8], out[1][:8]), k_max=10, use_filters=False,
                          schedule=(1,))
    assert e.value.code == -1
