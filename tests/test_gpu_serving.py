"""Serving with micro-batches whose work overlaps on the device (pi_serve
with more than one micro-batch in flight: the ordering of a micro-batch runs
on a side stream beside the descent and updates of the one before it).  Each
micro-batch's results are the same alone and in the mix: the served answers
equal the serial replay of the whole stream (the map oracle), and equal what
the same micro-batches give one call at a time on a fresh index.  Batches
large enough for the multi-kernel path, keys that later micro-batches read
after earlier ones wrote them, and rebuilds between micro-batches."""
import numpy as np
import pytest
import torch

from oracle import mapref
from paper_1601_00159_amd.index import Index, to_numpy_u64

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.node.name}", flush=True)


def _stream(rng, lk, n):
    """60/25/15 search/insert/delete; a quarter of the keys from a small hot
    set, so that micro-batches read what the ones before them wrote."""
    ops = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=n, p=[0.6, 0.25, 0.15])
    hot = np.concatenate([lk[:300], rng.integers(0, 1 << 63, size=300, dtype=np.uint64)])
    keys = lk[rng.integers(0, lk.size, n)]
    fresh = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
    keys = np.where(ops == 1, fresh, keys)
    h = rng.random(n) < 0.25
    keys[h] = hot[rng.integers(0, hot.size, int(h.sum()))]
    vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
    return ops, keys, vals


@pytest.mark.parametrize("policy,inflight", [("never", 2), ("threshold", 2), ("threshold", 4), ("background", 3),
                                             ("slices", 2)])
def test_overlapped_micro_batches_same_alone_and_in_the_mix(policy, inflight):
    rng = np.random.default_rng({"never": 1, "threshold": 2, "background": 3, "slices": 4}[policy] * 10 + inflight)
    lk = np.unique(rng.integers(0, 1 << 63, size=1 << 18, dtype=np.uint64))
    lv = rng.integers(0, 1 << 64, size=lk.size, dtype=np.uint64, endpoint=False)
    n = 420_000
    ops, keys, vals = _stream(rng, lk, n)
    # everything has arrived at once: micro-batches of up to 60,000 queries
    # leave back to back, so each is ordered while the one before it runs
    arrival = np.zeros(n, dtype=np.float64)
    ms = mapref.MapState(lk, lv)
    wv, ws = ms.apply_batch(ops, keys, vals)
    kw = dict(rebuild_policy=policy)
    if policy in ("threshold", "slices"):
        kw.update(rebuild_fraction=0.01, rebuild_min=1)  # a rebuild between most micro-batches
    with Index(**kw) as ix:
        ix.bulk_load(lk, lv)
        gv, gs, done, ends = ix.serve(arrival, ops, keys, vals, deadline_us=0.0, max_batch=60_000,
                                      max_inflight=inflight)
        torch.cuda.synchronize()
        gv, gs = to_numpy_u64(gv), gs.cpu().numpy()
        st = ix.stats()
        print(f"  {ends.size} micro-batches, rebuilds {st['repairs']}, slice rounds {st['slice_rounds']}",
              flush=True)
        assert ends.size >= 7 and ends[-1] == n
        assert np.array_equal(gs, ws) and np.array_equal(gv, wv), "served answers vs the serial replay"
        ek, ev = ix.export()
        assert np.array_equal(to_numpy_u64(ek), ms.keys) and np.array_equal(to_numpy_u64(ev), ms.vals)
        if policy in ("threshold", "slices"):
            assert st["repairs"] + st["slice_rounds"] >= 2
    # the same micro-batches alone, one call each
    with Index(**kw) as ix:
        ix.bulk_load(lk, lv)
        b = 0
        for e in ends:
            av, as_ = ix.execute(ops[b:e], keys[b:e], vals[b:e])
            torch.cuda.synchronize()
            assert np.array_equal(as_.cpu().numpy(), gs[b:e]) and np.array_equal(to_numpy_u64(av), gv[b:e]), (b, e)
            b = int(e)


def test_overlapped_serving_with_growing_micro_batches():
    """Micro-batch sizes that grow from one to the next (each buffer set
    grows while the other may still be in use), and the one-workgroup path
    between multi-kernel micro-batches."""
    rng = np.random.default_rng(77)
    lk = np.unique(rng.integers(0, 1 << 63, size=100_000, dtype=np.uint64))
    ms = mapref.MapState(lk, lk)
    # arrival bursts of growing size, 1 ms apart
    sizes = [500, 3000, 20_000, 700, 90_000, 200_000, 900]
    n = sum(sizes)
    ops, keys, vals = _stream(rng, lk, n)
    arrival = np.repeat(np.arange(len(sizes), dtype=np.float64) * 1000.0, sizes)
    wv, ws = ms.apply_batch(ops, keys, vals)
    with Index() as ix:
        ix.bulk_load(lk, lk)
        gv, gs, done, ends = ix.serve(arrival, ops, keys, vals, deadline_us=5.0, max_batch=0, max_inflight=2)
        torch.cuda.synchronize()
        print(f"  micro-batch ends {ends.tolist()}", flush=True)
        assert np.array_equal(gs.cpu().numpy(), ws) and np.array_equal(to_numpy_u64(gv), wv)
        ek, ev = ix.export()
        assert np.array_equal(to_numpy_u64(ek), ms.keys) and np.array_equal(to_numpy_u64(ev), ms.vals)
