"""Device-side evidence of the single-writer invariant (Section 3.2.4): in
checked mode every storage write of a batch records its writer per node, and
a node written by two different writers in one phase would fail the handle.
The batches here are the ones that stress ownership -- one hot key hit by
every query type, long chains of new keys behind one predecessor, deletes
followed by revives of the same keys -- on the multi-kernel path, the
one-workgroup path and the many-index launch.  The answers must equal the
oracle's and the check must stay silent."""
import numpy as np
import pytest
import torch

from oracle.skiplist import SkipList
from paper_1601_00159_amd.index import Group, Index, to_device_u64, to_device_u8, to_numpy_u64

pytestmark = pytest.mark.gpu
ERR_WRITERS_BIT = 4


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.node.name}", flush=True)


def test_writer_check_detects_a_second_writer():
    """The detection itself, on a private shadow: one writer noting a node
    twice passes, two writers of one node in one phase are caught."""
    with Index(check_writers=1) as ix:
        same, two = ix.writer_selftest()
        assert same == 0
        assert two & ERR_WRITERS_BIT


def _stress_batches(rng, lk, n):
    """Three batches: a hot key, chains of new keys, delete-then-revive."""
    hot = lk[7]
    ops = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=n, p=[0.4, 0.3, 0.3])
    keys = np.where(rng.random(n) < 0.6, hot, lk[rng.integers(0, lk.size, n)]).astype(np.uint64)
    vals = np.arange(n, dtype=np.uint64)
    b1 = (ops, keys, vals)
    # new keys packed between two loaded keys: long chains behind one predecessor
    gaps = lk[:64]
    chain = (gaps[rng.integers(0, gaps.size, n)] + rng.integers(1, 200, n).astype(np.uint64)).astype(np.uint64)
    b2 = (np.ones(n, dtype=np.uint8), chain, rng.integers(0, 1 << 63, size=n, dtype=np.uint64))
    # delete loaded keys, then insert them again in the same batch (revive) and
    # in the next one
    victims = lk[rng.integers(0, min(5000, lk.size), n // 2)]
    ops3 = np.concatenate([np.full(n // 2, 2, dtype=np.uint8), np.ones(n - n // 2, dtype=np.uint8)])
    keys3 = np.concatenate([victims, victims[: n - n // 2]])
    b3 = (ops3, keys3, rng.integers(0, 1 << 63, size=n, dtype=np.uint64))
    b4 = (np.ones(n // 2, dtype=np.uint8), victims, rng.integers(0, 1 << 63, size=n // 2, dtype=np.uint64))
    return [b1, b2, b3, b4]


@pytest.mark.parametrize("path", ["multi-kernel one launch", "multi-kernel separate", "one-workgroup"])
def test_single_writer_holds_on_stress_batches(path):
    """The multi-kernel path in both forms of its post-descent steps (one
    launch with grid barriers; separate kernels), and the one-workgroup
    path."""
    rng = np.random.default_rng({"multi-kernel one launch": 1, "multi-kernel separate": 4, "one-workgroup": 2}[path])
    lk = (np.unique(rng.integers(0, 1 << 40, size=40_000, dtype=np.uint64)) << np.uint64(10)).astype(np.uint64)
    n = 120_000 if path.startswith("multi") else 4096
    kw = {"small_batch_log2": 255} if path.startswith("multi") else {"small_batch_log2": 12}
    if path.startswith("multi"):
        kw["post_form"] = 1 if path.endswith("one launch") else 2
    orc = SkipList()
    orc.bulk_load(lk, lk)
    with Index(check_writers=1, rebuild_policy="never", **kw) as ix:
        ix.bulk_load(lk, lk)
        for i, b in enumerate(_stress_batches(rng, lk, n)):
            gv, gs = ix.execute(*b)
            torch.cuda.synchronize()
            wv, ws = orc.execute_batch(*b)
            assert np.array_equal(gs.cpu().numpy(), ws) and np.array_equal(to_numpy_u64(gv), wv), (path, i)
            st = ix.stats()  # raises PI_ERR_DEVICE if the check fired
            print(f"  batch {i}: new {st['new_nodes']}, deletes {st['deletes']}, revives {st['revives']}",
                  flush=True)
        assert st["revives"] > 0 and st["new_nodes"] > 0 and st["deletes"] > 0
        k, v = ix.export()
        ok, ov = orc.export()
        assert np.array_equal(to_numpy_u64(k), ok) and np.array_equal(to_numpy_u64(v), ov)


def test_single_writer_holds_in_the_many_index_launch():
    """The fused many-index launch, with batches larger than one workgroup
    chunk (each chunk checked as a batch of its own)."""
    rng = np.random.default_rng(3)
    dev = torch.device("cuda", 0)
    loads = [(np.unique(rng.integers(0, 1 << 40, size=s, dtype=np.uint64)) << np.uint64(10)).astype(np.uint64)
             for s in (3000, 9000, 20_000)]
    orcs, ixs = [], []
    try:
        for lk in loads:
            o = SkipList()
            o.bulk_load(lk, lk)
            orcs.append(o)
            ix = Index(check_writers=1, rebuild_policy="never")
            ix.bulk_load(lk, lk)
            ixs.append(ix)
        with Group(fused_max=16384) as g:
            for r in range(4):
                batches = [_stress_batches(rng, lk, m)[r] for lk, m in zip(loads, (900, 5000, 12_000))]
                dev_b = [(to_device_u8(o, dev), to_device_u64(k, dev), to_device_u64(v, dev),
                          torch.empty(o.size, dtype=torch.int64, device=dev),
                          torch.empty(o.size, dtype=torch.uint8, device=dev)) for o, k, v in batches]
                g.execute(ixs, dev_b)
                torch.cuda.synchronize()
                for j, (b, d) in enumerate(zip(batches, dev_b)):
                    wv, ws = orcs[j].execute_batch(*b)
                    assert np.array_equal(d[4].cpu().numpy(), ws) and np.array_equal(to_numpy_u64(d[3]), wv), (r, j)
        for ix in ixs:
            ix.stats()  # raises if the check fired
    finally:
        for ix in ixs:
            ix.close()
