"""The caller's allocator behind the C ABI: torch's caching allocator owns the
handle's device memory, a refused allocation is LEAFI_ENOMEM and leaves the
handle usable, and calls out of order are LEAFI_ESTATE."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

ENOMEM, ESTATE = -2, -3


def _pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_01836_amd as pkg
    pkg.load()
    return pkg


def test_torch_allocator_owns_the_handle_memory():
    pkg = _pkg()
    raw = W.random_walk(6000, 128, seed=21)
    alloc = pkg.TorchAllocator()
    ix = pkg.Index(allocator=alloc)
    before = torch.cuda.memory_allocated()
    ix.build(torch.from_numpy(raw).cuda(), leaf_capacity=500, n_segments=16)
    torch.cuda.synchronize()
    info = ix.info()
    # the resident store is in torch's pool and counted by the allocator
    assert alloc.live_bytes >= info["device_bytes"] > 0
    assert torch.cuda.memory_allocated() - before >= info["device_bytes"]
    q, _, _ = W.noisy_queries(raw, 20, 0.1, 22, 23)
    ids, d = ix.search(torch.from_numpy(q).cuda(), k=3, use_filters=False)
    want_ids, want_d = O.knn(O.znorm(raw), O.znorm(q), 3)
    assert np.allclose(d.cpu().numpy(), want_d, rtol=1e-4)
    ix.close()
    assert alloc.live_bytes == 0


def test_refused_allocation_is_enomem_and_handle_stays_valid():
    pkg = _pkg()
    raw = torch.from_numpy(W.random_walk(6000, 128, seed=24)).cuda()
    alloc = pkg.TorchAllocator(limit=1 << 20)  # far below the 6000 x 128 store
    ix = pkg.Index(allocator=alloc)
    with pytest.raises(pkg.LeafiError) as e:
        ix.build(raw, leaf_capacity=500, n_segments=16)
    assert e.value.code == ENOMEM and "refused" in str(e.value)
    assert alloc.live_bytes == 0          # nothing leaked by the failed build
    assert ix.info()["n_leaves"] == 0     # the handle answers, unbuilt
    with pytest.raises(pkg.LeafiError) as e:
        ix.search(raw[:4].contiguous(), k=1, use_filters=False)
    assert e.value.code == ESTATE
    alloc.limit = None                    # the same handle builds once memory is there
    ix.build(raw, leaf_capacity=500, n_segments=16)
    ids, d = ix.search(raw[:4].contiguous(), k=1, use_filters=False)
    assert list(ids.cpu().numpy()[:, 0]) == [0, 1, 2, 3]
    # a search whose workspace is refused fails cleanly, and the next one works
    alloc.limit = alloc.live_bytes
    with pytest.raises(pkg.LeafiError) as e:
        ix.search(raw[:600].contiguous(), k=5, use_filters=False)
    assert e.value.code == ENOMEM
    alloc.limit = None
    ids, d = ix.search(raw[:600].contiguous(), k=5, use_filters=False)
    assert (ids.cpu().numpy()[:, 0] == np.arange(600)).all()


def test_calls_out_of_order_are_estate():
    pkg = _pkg()
    ix = pkg.Index()
    q = torch.zeros((2, 64), device="cuda")
    for call in (lambda: ix.search(q, k=1), lambda: ix.lower_bounds(q), lambda: ix.leaf_knn(q, 1),
                 lambda: ix.calibrate(q, [1], [0.9]), lambda: ix.train_filters(max_epochs=1)):
        with pytest.raises(pkg.LeafiError) as e:
            call()
        assert e.value.code == ESTATE
    raw = W.random_walk(3000, 64, seed=25)
    ix.build(torch.from_numpy(raw).cuda(), leaf_capacity=500, n_segments=8)
    with pytest.raises(pkg.LeafiError) as e:   # calibration needs filters
        ix.calibrate(torch.from_numpy(raw[:10]).cuda(), [1], [0.9])
    assert e.value.code == ESTATE
    with pytest.raises(pkg.LeafiError) as e:
        ix.set_offsets([1], [0.9], np.zeros((1, 1), dtype=np.float32))
    assert e.value.code == ESTATE
    with pytest.raises(pkg.LeafiError) as e:   # no training set kept
        ix.examples()
    assert e.value.code == ESTATE
