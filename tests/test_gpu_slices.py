"""Slice repair (rebuild policy SLICES, the finer-grained rebuild of the
paper's future work next to the threshold rebuild of Section 4.3.5): the
lower index levels live in per-key-range segments with gaps, and a repair
round rewrites only the slices that received new nodes.  Repair boundaries
change no answer: the same batches under forced rounds after every batch, no
rebuild at all, the default threshold and the plain threshold policy give
the oracle's answers and final set; the levels stay well formed; clustered
inserts repair few slices; an overflowing segment falls back to a full
rebuild; range search, the one-workgroup path and the many-index launch read
the gapped levels correctly."""
import numpy as np
import pytest
import torch

from oracle.skiplist import SkipList
from paper_1601_00159_amd import bytemodel
from paper_1601_00159_amd.index import Group, Index, to_device_u64, to_device_u8, to_numpy_u64

pytestmark = pytest.mark.gpu
KMAX = (1 << 64) - 1


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.node.name}", flush=True)


def check_levels(ix):
    """Levels strictly increasing; each level-l key sits on level l-1 (down
    pointer) and has height >= l; every level-(l-1) key of height >= l is on
    level l."""
    st = ix.stats()
    prev = None
    for lvl in range(2, st["n_levels"] + 1):
        k, d = ix.level(lvl)
        k, d = to_numpy_u64(k), d.cpu().numpy().astype(np.int64)
        assert np.all(k[1:] > k[:-1]), lvl
        if k.size:
            assert np.all(bytemodel.heights(k) >= lvl), lvl
        if prev is not None:
            if k.size:
                assert np.array_equal(prev[d - 1], k), lvl
            want = prev[bytemodel.heights(prev) >= lvl] if prev.size else prev
            assert np.array_equal(want, k), lvl
        prev = k
    return st


def _batch(rng, pool, n, fresh_hi=1 << 63):
    ops = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=n, p=[0.4, 0.4, 0.2])
    keys = pool[rng.integers(0, pool.size, n)]
    ins = ops == 1
    keys[ins] = rng.integers(0, fresh_hi, size=int(ins.sum()), dtype=np.uint64)
    vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
    return ops, keys, vals


def test_repair_boundaries_do_not_change_answers():
    rng = np.random.default_rng(200)
    lk = np.unique(rng.integers(0, 1 << 63, size=70_000, dtype=np.uint64))
    lv = rng.integers(0, 1 << 64, size=lk.size, dtype=np.uint64, endpoint=False)
    batches = [_batch(rng, lk, n) for n in (30_000, 700, 30_000, 5000, 20_000, 3000, 30_000, 10_000)]
    orc = SkipList()
    orc.bulk_load(lk, lv)
    want = [orc.execute_batch(*b) for b in batches]
    ok, ov = orc.export()
    runs = {"forced": dict(rebuild_policy="slices", rebuild_fraction=0.0, rebuild_min=1),
            "default": dict(rebuild_policy="slices"),
            "small-threshold": dict(rebuild_policy="slices", rebuild_fraction=0.02, rebuild_min=1),
            "none": dict(rebuild_policy="never"),
            "threshold": dict(rebuild_policy="threshold", rebuild_fraction=0.02, rebuild_min=1)}
    for name, kw in runs.items():
        with Index(**kw) as ix:
            ix.bulk_load(lk, lv)
            for i, b in enumerate(batches):
                gv, gs = ix.execute(*b)
                torch.cuda.synchronize()
                assert np.array_equal(gs.cpu().numpy(), want[i][1]), (name, i)
                assert np.array_equal(to_numpy_u64(gv), want[i][0]), (name, i)
            ek, ev = ix.export()
            assert np.array_equal(to_numpy_u64(ek), ok) and np.array_equal(to_numpy_u64(ev), ov), name
            st = check_levels(ix) if kw["rebuild_policy"] == "slices" else ix.stats()
            print(f"  {name}: rounds {st['slice_rounds']}, slices repaired {st['slices_repaired']} of "
                  f"{st['slices']}, full rebuilds {st['repairs']}", flush=True)
            if name == "forced":
                assert st["slice_rounds"] >= 6 and st["slices"] >= 16


def test_clustered_inserts_repair_few_slices():
    """Inserts confined to a narrow key range touch a few slices per round;
    searches over the whole key space stay right."""
    rng = np.random.default_rng(201)
    lk = np.unique(rng.integers(0, 1 << 63, size=1 << 20, dtype=np.uint64))
    lv = rng.integers(0, 1 << 64, size=lk.size, dtype=np.uint64, endpoint=False)
    lo, hi = lk[100_000], lk[112_000]  # about three slices of 4096 keys
    orc = SkipList()
    orc.bulk_load(lk, lv)
    with Index(rebuild_policy="slices", rebuild_fraction=0.0, rebuild_min=1) as ix:
        ix.bulk_load(lk, lv)
        for b in range(6):
            n = 600  # about 200 new keys per slice and round: the segments' room absorbs them
            ops = np.ones(n, dtype=np.uint8)
            keys = rng.integers(lo, hi, size=n, dtype=np.uint64)
            vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
            gv, gs = ix.execute(ops, keys, vals)
            torch.cuda.synchronize()
            wv, ws = orc.execute_batch(ops, keys, vals)
            assert np.array_equal(gs.cpu().numpy(), ws) and np.array_equal(to_numpy_u64(gv), wv), b
        q = np.concatenate([lk[rng.integers(0, lk.size, 50_000)], keys[:20_000],
                            rng.integers(0, 1 << 63, size=10_000, dtype=np.uint64)])
        sops = np.zeros(q.size, dtype=np.uint8)
        gv, gs = ix.execute(sops, q, q)
        torch.cuda.synchronize()
        wv, ws = orc.execute_batch(sops, q, q)
        assert np.array_equal(gs.cpu().numpy(), ws) and np.array_equal(to_numpy_u64(gv), wv)
        st = check_levels(ix)
        print(f"  rounds {st['slice_rounds']}, slices repaired {st['slices_repaired']} of {st['slices']}, "
              f"full rebuilds {st['repairs']}", flush=True)
        assert st["slice_rounds"] >= 3 and st["repairs"] == 0
        assert st["slices_repaired"] <= 4 * st["slice_rounds"]  # a few of the 256 slices per round
        ek, ev = ix.export()
        ok, ov = orc.export()
        assert np.array_equal(to_numpy_u64(ek), ok) and np.array_equal(to_numpy_u64(ev), ov)


def test_overflowing_segment_falls_back_to_a_full_rebuild():
    rng = np.random.default_rng(202)
    lk = (np.unique(rng.integers(0, 1 << 40, size=200_000, dtype=np.uint64)) << np.uint64(20)).astype(np.uint64)
    orc = SkipList()
    orc.bulk_load(lk, lk)
    with Index(rebuild_policy="slices", rebuild_fraction=0.0, rebuild_min=1) as ix:
        ix.bulk_load(lk, lk)
        base = lk[50_000]
        for b in range(3):
            n = 30_000  # far more keys than one segment holds, all in one slice
            ops = np.ones(n, dtype=np.uint8)
            keys = base + rng.integers(1, 1 << 19, size=n, dtype=np.uint64)
            gv, gs = ix.execute(ops, keys, keys)
            torch.cuda.synchronize()
            wv, ws = orc.execute_batch(ops, keys, keys)
            assert np.array_equal(gs.cpu().numpy(), ws) and np.array_equal(to_numpy_u64(gv), wv), b
        st = check_levels(ix)
        print(f"  rounds {st['slice_rounds']}, full rebuilds {st['repairs']}", flush=True)
        assert st["repairs"] >= 1
        ek, ev = ix.export()
        ok, ov = orc.export()
        assert np.array_equal(to_numpy_u64(ek), ok) and np.array_equal(to_numpy_u64(ev), ov)


def test_range_search_and_small_batches_on_repaired_slices():
    rng = np.random.default_rng(203)
    lk = np.unique(rng.integers(0, 1 << 63, size=100_000, dtype=np.uint64))
    orc = SkipList()
    orc.bulk_load(lk, lk)
    with Index(rebuild_policy="slices", rebuild_fraction=0.0, rebuild_min=1, small_batch_log2=12) as ix:
        ix.bulk_load(lk, lk)
        for n in (40_000, 4096, 900, 40_000):  # one-workgroup batches between multi-kernel ones
            b = _batch(rng, lk, n)
            gv, gs = ix.execute(*b)
            torch.cuda.synchronize()
            wv, ws = orc.execute_batch(*b)
            assert np.array_equal(gs.cpu().numpy(), ws) and np.array_equal(to_numpy_u64(gv), wv), n
        assert ix.stats()["slice_rounds"] >= 2
        ok, _ = orc.export()
        lo = ok[rng.integers(0, ok.size, 5000)]
        hi = lo + (rng.random(5000) * 200 * ((1 << 63) / ok.size)).astype(np.uint64)
        lo = np.concatenate([lo, np.array([0, KMAX], dtype=np.uint64)])
        hi = np.concatenate([hi, np.array([KMAX, KMAX], dtype=np.uint64)])
        wc, wk, wv = orc.range_batch(lo, hi)
        gc, gk, gv = ix.range_search(lo, hi)
        torch.cuda.synchronize()
        assert np.array_equal(gc.cpu().numpy().astype(np.uint64), wc)
        assert np.array_equal(to_numpy_u64(gk), wk) and np.array_equal(to_numpy_u64(gv), wv)


def test_many_index_launch_with_slice_repair():
    rng = np.random.default_rng(204)
    dev = torch.device("cuda", 0)
    loads = [np.unique(rng.integers(0, 1 << 63, size=s, dtype=np.uint64)) for s in (5000, 30_000, 90_000)]
    orcs, ixs = [], []
    try:
        for lk in loads:
            o = SkipList()
            o.bulk_load(lk, lk)
            orcs.append(o)
            ix = Index(rebuild_policy="slices", rebuild_fraction=0.0, rebuild_min=1)
            ix.bulk_load(lk, lk)
            ixs.append(ix)
        with Group(fused_max=4096) as g:
            for r in range(5):
                batches = [_batch(rng, lk, m) for lk, m in zip(loads, (800, 3000, 20_000))]
                dev_b = [(to_device_u8(o, dev), to_device_u64(k, dev), to_device_u64(v, dev),
                          torch.empty(o.size, dtype=torch.int64, device=dev),
                          torch.empty(o.size, dtype=torch.uint8, device=dev)) for o, k, v in batches]
                g.execute(ixs, dev_b)
                torch.cuda.synchronize()
                for j, (b, d) in enumerate(zip(batches, dev_b)):
                    wv, ws = orcs[j].execute_batch(*b)
                    assert np.array_equal(d[4].cpu().numpy(), ws) and np.array_equal(to_numpy_u64(d[3]), wv), (r, j)
        for ix, o in zip(ixs, orcs):
            st = check_levels(ix)
            assert st["slice_rounds"] >= 2
            ek, ev = ix.export()
            ok, ov = o.export()
            assert np.array_equal(to_numpy_u64(ek), ok) and np.array_equal(to_numpy_u64(ev), ov)
    finally:
        for ix in ixs:
            ix.close()
