"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every answer is an exact integer, so every comparison is bit-exact: per-query
(status, value) in arrival order, the final live key/value set, the index
levels and the interceptions.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import mapref
from oracle.skiplist import SkipList
from paper_1601_00159_amd import workloads as W
from paper_1601_00159_amd._lib import PI_ERR_CAPACITY, PI_ERR_STATE, PiError
from paper_1601_00159_amd.index import Index, to_device_u64, to_numpy_u64

pytestmark = pytest.mark.gpu
KMAX = (1 << 64) - 1
OPS = {"SEARCH": 0, "INSERT": 1, "DELETE": 2}


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.node.name}", flush=True)


def say(*a):
    print("  ", *a, flush=True)


def run_gpu(ix, ops, keys, vals):
    ov, os_ = ix.execute(ops, keys, vals)
    torch.cuda.synchronize()
    return to_numpy_u64(ov), os_.cpu().numpy()


def export_np(ix):
    k, v = ix.export()
    return to_numpy_u64(k), to_numpy_u64(v)


def assert_same(got_v, got_s, want_v, want_s, what=""):
    got_v, want_v = np.asarray(got_v, dtype=np.uint64), np.asarray(want_v, dtype=np.uint64)
    got_s, want_s = np.asarray(got_s, dtype=np.uint8), np.asarray(want_s, dtype=np.uint8)
    bad = np.nonzero((got_s != want_s) | (got_v != want_v))[0]
    if bad.size:
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} mismatches; first at {i}: got ({got_s[i]},{got_v[i]}) "
                             f"want ({want_s[i]},{want_v[i]})")


# ----------------------------------------------------------------- ordering

def _sort_case(kind, n, rng):
    if kind == "uniform+dups":
        keys = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
        keys[rng.random(n) < 0.3] = rng.integers(0, 50, size=1, dtype=np.uint64)[0]  # a hot key
        keys[rng.random(n) < 0.01] = np.uint64(KMAX)
    elif kind == "clustered":
        # nearly all keys in one 16-bit slice of the span: one huge group of
        # distinct keys (no dominant key)
        keys = rng.integers(0, 1 << 20, size=n, dtype=np.uint64)
        keys[0] = np.uint64(1 << 63)
    elif kind == "hot-in-cluster":
        # a dominant key with large runs of other keys on both sides of it
        keys = rng.integers(0, 1 << 20, size=n, dtype=np.uint64)
        keys[rng.random(n) < 0.6] = np.uint64(1 << 19)
        keys[0] = np.uint64(1 << 63)
    elif kind == "two-hot":
        keys = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
        r = rng.random(n)
        keys[r < 0.4] = np.uint64(12345)
        keys[(r >= 0.4) & (r < 0.75)] = np.uint64(12346)
    else:
        raise ValueError(kind)
    return keys


@pytest.mark.parametrize("kind,n", [("uniform+dups", m) for m in (1, 2, 63, 64, 4095, 4096, 4097, 100_003, 1 << 20,
                                                                   4096 * 67 + 5, (1 << 22) + 3)]
                         + [("clustered", 70_001), ("hot-in-cluster", 150_001), ("two-hot", 200_003)])
def test_sort_is_stable_key_order(kind, n):
    rng = np.random.default_rng(n)
    keys = _sort_case(kind, n, rng)
    with Index() as ix:
        sk, perm = ix.sort(keys)
        torch.cuda.synchronize()
        want = np.argsort(keys, kind="stable")
        assert np.array_equal(perm.cpu().numpy().astype(np.int64), want)
        assert np.array_equal(to_numpy_u64(sk), keys[want])


# ------------------------------------------------------------ construction

def test_bulk_load_export_levels_interceptions():
    rng = np.random.default_rng(4)
    n = 300_001
    keys = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
    keys[:5000] = keys[5000:10000]  # duplicates: the last occurrence wins
    keys[7] = np.uint64(KMAX)       # skipped
    vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
    uk, uv = mapref.dedupe_last(keys, vals)
    orc = SkipList()
    orc.bulk_load_sorted(uk, uv)
    with Index() as ix:
        ix.bulk_load(keys, vals)
        ek, ev = export_np(ix)
        assert np.array_equal(ek, uk) and np.array_equal(ev, uv)
        st = ix.stats()
        assert st["live_nodes"] == uk.size == st["base_nodes"]
        prev_keys = uk
        for lvl in range(2, 25):
            want = orc.level_keys(lvl)
            lk, ld = ix.level(lvl)
            lk, ld = to_numpy_u64(lk), ld.cpu().numpy().astype(np.int64)
            assert np.array_equal(lk, want), lvl
            if lk.size:
                # the down pointer of a key is its 1-based position one level below
                # (level 2: its storage slot, base slot i holds the i-th key)
                assert np.array_equal(prev_keys[ld - 1], lk), lvl
            prev_keys = lk
            assert st["level_size"][lvl] == want.size
        # Definition 4 against the oracle
        q = np.concatenate([uk[rng.integers(0, uk.size, 20000)],
                            rng.integers(0, 1 << 63, size=20000, dtype=np.uint64),
                            np.array([0, uk[0], uk[-1], (1 << 63) + 5, KMAX - 1], dtype=np.uint64)])
        ik, hd = ix.interceptions(q)
        ik, hd = to_numpy_u64(ik), hd.cpu().numpy()
        for i in range(q.size):
            w = orc.interception(int(q[i]))
            if w is None:
                assert hd[i] == 1, i
            else:
                assert hd[i] == 0 and int(ik[i]) == w, i
        with pytest.raises(PiError) as e:
            ix.bulk_load(keys[:10], vals[:10])
        assert e.value.status == PI_ERR_STATE


# --------------------------------------------------------------- golden

def _golden(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        g = json.load(f)
    ops = np.array([OPS[o] if isinstance(o, str) else o for o, _, _ in g["batch"]], dtype=np.uint8)
    keys = np.array([k for _, k, _ in g["batch"]], dtype=np.uint64)
    vals = np.array([v for _, _, v in g["batch"]], dtype=np.uint64)
    return g, ops, keys, vals


@pytest.mark.parametrize("policy", ["never", "always"])
@pytest.mark.parametrize("name", ["e1_duplicates_revive.json", "e2_empty_and_edges.json"])
def test_golden(golden_dir, name, policy):
    g, ops, keys, vals = _golden(golden_dir, name)
    with Index(rebuild_policy=policy) as ix:
        if g["initial"]:
            ix.bulk_load(np.array([k for k, _ in g["initial"]], dtype=np.uint64),
                         np.array([v for _, v in g["initial"]], dtype=np.uint64))
        gv, gs = run_gpu(ix, ops, keys, vals)
        assert [[int(s), int(v)] for s, v in zip(gs, gv)] == g["expected"]
        ek, ev = export_np(ix)
        assert [[int(k), int(v)] for k, v in zip(ek, ev)] == g["final"]


# ------------------------------------------------------- mixed batches

def _random_batch(rng, pool, n, p_invalid=0.01):
    ops = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=n, p=[0.5, 0.3, 0.2])
    ops[rng.random(n) < p_invalid] = 7
    keys = pool[rng.integers(0, pool.size, size=n)]
    keys[rng.random(n) < p_invalid] = np.uint64(KMAX)
    vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
    return ops, keys, vals


@pytest.mark.parametrize("policy,form,bits", [("never", 0, 0), ("always", 0, 0), ("threshold", 0, 0),
                                              ("never", 1, 16), ("threshold", 2, 24), ("never", 2, 16),
                                              ("always", 2, 32), ("never", 1, 32)])
def test_mixed_batches_vs_oracle(policy, form, bits):
    """Mixed and SEARCH-only batches in turn (so that the default form of the
    post-descent steps, and the width of the ordering's range position,
    switch with them), and each form and width forced: batches with updates
    ordered by a 16-bit position leave larger groups to the in-group fix-up,
    and SEARCH-only ones leave each wave's queries to the descent's sort;
    a 32-bit position leaves few."""
    rng = np.random.default_rng({"never": 1, "always": 2, "threshold": 3}[policy] + 10 * form + bits)
    lk = rng.integers(0, 1 << 63, size=50_000, dtype=np.uint64)
    lv = rng.integers(0, 1 << 64, size=50_000, dtype=np.uint64, endpoint=False)
    pool = np.concatenate([lk[:20_000], rng.integers(0, 1 << 63, size=20_000, dtype=np.uint64),
                           np.array([0, (1 << 64) - 2], dtype=np.uint64)])
    orc = SkipList()
    orc.bulk_load(lk, lv)
    with Index(rebuild_policy=policy, rebuild_fraction=0.05, rebuild_min=1, post_form=form, order_bits=bits) as ix:
        ix.bulk_load(lk, lv)
        tot = {"queries": 0, "hits": 0, "invalid": 0}
        for b in range(9):
            n = [40_000, 1, 4097, 65_536, 12_345, 40_000, 30_000, 30_000, 20_000][b]
            ops, keys, vals = _random_batch(rng, pool, n)
            if b in (3, 6, 7):
                ops = np.where(ops <= 2, 0, ops).astype(np.uint8)  # SEARCH-only (invalid ops stay)
            say(f"batch {b} n={n}")
            wv, ws = orc.execute_batch(ops, keys, vals)
            gv, gs = run_gpu(ix, ops, keys, vals)
            assert_same(gv, gs, wv, ws, f"batch {b}")
            ws = np.asarray(ws, dtype=np.uint8)
            tot["queries"] += n
            tot["hits"] += int((ws == 1).sum())
            tot["invalid"] += int((ws == 255).sum())
        ek, ev = export_np(ix)
        ok, ov = orc.export()
        assert np.array_equal(ek, ok) and np.array_equal(ev, ov)
        st = ix.stats()
        assert st["live_nodes"] == len(orc)
        # the library's counters agree with the oracle's answers
        for k, v in tot.items():
            assert st[k] == v, (k, st[k], v)
        if policy == "always":
            assert st["repairs"] >= 1 and st["overflow_nodes"] == 0
        # after a rebuild the levels are the canonical ones again
        ix.repair()
        for lvl in range(2, 25):
            lk2, _ = ix.level(lvl)
            assert np.array_equal(to_numpy_u64(lk2), orc.level_keys(lvl)), lvl


def test_hot_keys_and_revives():
    # one key hit by many queries of every type in one batch, plus
    # delete/insert chains spanning the whole batch
    rng = np.random.default_rng(9)
    lk = np.arange(1, 2001, dtype=np.uint64) * np.uint64(1000)
    lv = lk + np.uint64(7)
    n = 200_000
    ops = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=n, p=[0.4, 0.3, 0.3])
    keys = np.where(rng.random(n) < 0.7, np.uint64(5000),
                    rng.integers(0, 2_100_000, size=n).astype(np.uint64)).astype(np.uint64)
    vals = np.arange(n, dtype=np.uint64)
    orc = SkipList()
    orc.bulk_load(lk, lv)
    wv, ws = orc.execute_batch(ops, keys, vals)
    with Index(rebuild_policy="never") as ix:
        ix.bulk_load(lk, lv)
        gv, gs = run_gpu(ix, ops, keys, vals)
        assert_same(gv, gs, wv, ws, "hot keys")
        ek, ev = export_np(ix)
        ok, ov = orc.export()
        assert np.array_equal(ek, ok) and np.array_equal(ev, ov)
        # a second batch walks the linked nodes of the first
        ops2, keys2, vals2 = _random_batch(rng, np.concatenate([ok, keys[:1000]]), 50_000, 0.0)
        wv, ws = orc.execute_batch(ops2, keys2, vals2)
        gv, gs = run_gpu(ix, ops2, keys2, vals2)
        assert_same(gv, gs, wv, ws, "after links")


def test_edge_cases():
    with Index(rebuild_policy="never") as ix:
        e8 = np.zeros(0, dtype=np.uint8)
        e64 = np.zeros(0, dtype=np.uint64)
        gv, gs = run_gpu(ix, e8, e64, e64)                    # empty batch
        assert gv.size == 0
        gv, gs = run_gpu(ix, np.array([0, 2], dtype=np.uint8), np.array([5, 5], dtype=np.uint64),
                         np.zeros(2, dtype=np.uint64))        # empty index
        assert gs.tolist() == [0, 0] and gv.tolist() == [0, 0]
        gv, gs = run_gpu(ix, np.array([3, 9, 1], dtype=np.uint8),
                         np.array([1, KMAX, KMAX], dtype=np.uint64), np.array([1, 2, 3], dtype=np.uint64))
        assert gs.tolist() == [255, 255, 255]                 # all invalid
        ks = np.array([0, (1 << 64) - 2, 1 << 63, 0], dtype=np.uint64)
        gv, gs = run_gpu(ix, np.array([1, 1, 1, 0], dtype=np.uint8), ks, np.array([10, 11, 12, 0], dtype=np.uint64))
        assert gs.tolist() == [0, 0, 0, 1] and gv.tolist() == [0, 0, 0, 10]
        ek, ev = export_np(ix)
        assert ek.tolist() == [0, 1 << 63, (1 << 64) - 2] and ev.tolist() == [10, 12, 11]
        assert ix.stats()["live_nodes"] == 3


def test_capacity_error_leaves_index_unchanged():
    rng = np.random.default_rng(12)
    lk = rng.integers(0, 1 << 63, size=1000, dtype=np.uint64)
    with Index(capacity_hint=1500, rebuild_policy="never") as ix:
        ix.bulk_load(lk, lk)
        before = export_np(ix)
        ops = np.ones(2000, dtype=np.uint8)
        keys = rng.integers(0, 1 << 63, size=2000, dtype=np.uint64)
        with pytest.raises(PiError) as e:
            ix.execute(ops, keys, keys)
        assert e.value.status == PI_ERR_CAPACITY
        after = export_np(ix)
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        # a batch that fits is still accepted
        gv, gs = run_gpu(ix, ops[:100], keys[:100], keys[:100])
        assert (gs == 0).all()


@pytest.mark.parametrize("lds_levels", [1, 3, 64])
def test_results_independent_of_lds_staging(lds_levels):
    w = W.plain_pi(scale=16)
    b = w.batches[0]
    orc = SkipList()
    orc.bulk_load(w.load_keys, w.load_vals)
    wv, ws = orc.execute_batch(b.ops, b.keys, b.vals)
    with Index(lds_levels=lds_levels, rebuild_policy="never") as ix:
        ix.bulk_load(w.load_keys, w.load_vals)
        gv, gs = run_gpu(ix, b.ops, b.keys, b.vals)
        assert_same(gv, gs, wv, ws, f"lds_levels={lds_levels}")


@pytest.mark.parametrize("qpl,block", [(1, 1024), (2, 256), (4, 512), (1, 512), (2, 1024)])
def test_descent_variants_agree(qpl, block):
    """Every descent launch shape (queries per lane, block size) gives the
    oracle's answers, on base nodes and on linked ones, and the oracle's
    interceptions."""
    rng = np.random.default_rng(100 + 10 * qpl + block)
    lk = rng.integers(0, 1 << 63, size=60_000, dtype=np.uint64)
    lv = rng.integers(0, 1 << 64, size=60_000, dtype=np.uint64, endpoint=False)
    pool = np.concatenate([lk[:30_000], rng.integers(0, 1 << 63, size=30_000, dtype=np.uint64),
                           np.array([0, (1 << 64) - 2], dtype=np.uint64)])
    orc = SkipList()
    orc.bulk_load(lk, lv)
    with Index(rebuild_policy="never", queries_per_lane=qpl, descent_block=block, lds_budget=2000) as ix:
        ix.bulk_load(lk, lv)
        for b, n in enumerate([30_001, 1, 70_000]):
            ops, keys, vals = _random_batch(rng, pool, n)
            if b == 2:
                ops[:] = 0  # read-only batch over base and linked nodes
            wv, ws = orc.execute_batch(ops, keys, vals)
            gv, gs = run_gpu(ix, ops, keys, vals)
            assert_same(gv, gs, wv, ws, f"batch {b}")
        q = np.concatenate([pool[rng.integers(0, pool.size, 5000)],
                            np.array([0, lk.min(), lk.max(), KMAX - 1], dtype=np.uint64)])
        ik, hd = ix.interceptions(q)
        ik, hd = to_numpy_u64(ik), hd.cpu().numpy()
        # with rebuilds off the index levels are those of the bulk load, so the
        # interceptions are those of an oracle holding the loaded set
        ref = SkipList()
        uk, uv = mapref.dedupe_last(lk, lv)
        ref.bulk_load_sorted(uk, uv)
        for i in range(q.size):
            w = ref.interception(int(q[i]))
            assert (hd[i] == 1) if w is None else (hd[i] == 0 and int(ik[i]) == w), i
        ref.close()


# ------------------------------------------------ the named workloads

def test_plain_pi_full_size():
    """2^20 loaded keys, one 2^20-query batch, 80/10/10, every answer and the
    final set against the Pugh oracle."""
    w = W.plain_pi(scale=20)
    b = w.batches[0]
    orc = SkipList()
    orc.bulk_load(w.load_keys, w.load_vals)
    wv, ws = orc.execute_batch(b.ops, b.keys, b.vals)
    with Index() as ix:
        ix.bulk_load(w.load_keys, w.load_vals)
        gv, gs = run_gpu(ix, b.ops, b.keys, b.vals)
        assert_same(gv, gs, wv, ws, "plain 2^20")
        ek, ev = export_np(ix)
        ok, ov = orc.export()
        assert np.array_equal(ek, ok) and np.array_equal(ev, ov)


@pytest.mark.parametrize("theta", [None, 0.99])
def test_read_scaling_reduced(theta):
    w = W.read_scaling(theta, load_log2=22, query_log2=20, n_batches=2)
    ms = mapref.MapState(w.load_keys, w.load_vals)
    with Index() as ix:
        ix.bulk_load(w.load_keys, w.load_vals)
        for b in w.batches:
            wv, ws = ms.search_batch(b.keys)
            gv, gs = run_gpu(ix, b.ops, b.keys, b.vals)
            assert_same(gv, gs, wv, ws, w.name)


def test_write_skew_reduced():
    w = W.write_skew(load_log2=20, query_log2=18, n_batches=6)
    ms = mapref.MapState(w.load_keys, w.load_vals)
    with Index(rebuild_fraction=0.15) as ix:
        ix.bulk_load(w.load_keys, w.load_vals)
        for i, b in enumerate(w.batches):
            wv, ws = ms.apply_batch(b.ops, b.keys, b.vals)
            gv, gs = run_gpu(ix, b.ops, b.keys, b.vals)
            assert_same(gv, gs, wv, ws, f"{w.name} batch {i}")
        ek, ev = export_np(ix)
        assert np.array_equal(ek, ms.keys) and np.array_equal(ev, ms.vals)
        assert ix.stats()["repairs"] >= 1


def test_headline_full_size_search():
    """2^26 loaded keys, one batch of 2^22 uniform SEARCH queries, in the
    launch configuration the benchmark times; every answer checked."""
    w = W.headline(None, n_batches=1)
    ms = mapref.MapState(w.load_keys, w.load_vals)
    b = w.batches[0]
    wv, ws = ms.search_batch(b.keys)
    with Index() as ix:
        ix.bulk_load(w.load_keys, w.load_vals)
        gv, gs = run_gpu(ix, b.ops, b.keys, b.vals)
        assert_same(gv, gs, wv, ws, w.name)
        assert (gs == 1).all()


# ------------------------------------------------------------ range search

def _ranges(rng, keys, n):
    gap = (1 << 63) // max(keys.size, 1)
    lo = np.where(rng.random(n) < 0.5, keys[rng.integers(0, keys.size, n)],
                  rng.integers(0, 1 << 63, size=n, dtype=np.uint64)).astype(np.uint64)
    gran = rng.choice(np.array([0, 1, 10, 100, 1000]), size=n)
    width = (rng.random(n) * gran * gap).astype(np.uint64)
    hi = lo + width
    edge_lo = np.array([0, 0, KMAX, 10, keys[0], keys[-1], KMAX - 1, 0, keys[5]], dtype=np.uint64)
    edge_hi = np.array([KMAX, 0, KMAX, 9, keys[0], KMAX, KMAX, KMAX - 1, keys[5] - 1], dtype=np.uint64)
    return np.concatenate([lo, edge_lo]), np.concatenate([hi, edge_hi])


@pytest.mark.parametrize("state", ["base", "dead", "linked", "rebuilt"])
def test_range_search_vs_oracle(state):
    """Range search (Section 3.2.5) against the oracle on every storage state:
    base nodes only, base nodes with delete flags, linked new nodes, and after
    a rebuild; granularity 0 to ~1000 keys per range plus edge ranges."""
    rng = np.random.default_rng({"base": 1, "dead": 2, "linked": 3, "rebuilt": 4}[state])
    lk = rng.integers(0, 1 << 63, size=200_000, dtype=np.uint64)
    lv = rng.integers(0, 1 << 64, size=200_000, dtype=np.uint64, endpoint=False)
    orc = SkipList()
    orc.bulk_load(lk, lv)
    with Index(rebuild_policy="never") as ix:
        ix.bulk_load(lk, lv)
        if state != "base":
            n = 40_000
            ops = np.full(n, 2, dtype=np.uint8)
            keys = lk[rng.integers(0, lk.size, n)]
            if state in ("linked", "rebuilt"):
                ops[: n // 2] = 1
                keys[: n // 2] = rng.integers(0, 1 << 63, size=n // 2, dtype=np.uint64)
            vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
            orc.execute_batch(ops, keys, vals)
            run_gpu(ix, ops, keys, vals)
            st = ix.stats()
            assert (st["overflow_nodes"] > 0) == (state == "linked" or state == "rebuilt")
            if state == "rebuilt":
                ix.repair()
        ok, _ = orc.export()
        lo, hi = _ranges(rng, ok, 20_000)
        wc, wk, wv = orc.range_batch(lo, hi)
        say(f"{lo.size} ranges, {int(wc.sum())} results, max {int(wc.max())}")
        gc, gk, gv = ix.range_search(lo, hi)
        torch.cuda.synchronize()
        assert np.array_equal(gc.cpu().numpy().astype(np.uint64), wc)
        assert np.array_equal(to_numpy_u64(gk), wk) and np.array_equal(to_numpy_u64(gv), wv)


def test_range_collect_after_other_counts():
    """A collect reuses the ordering of the count just before it only when
    that count was of the same ranges: two counts, then the two collects in
    the other order, give the oracle's pairs for both."""
    rng = np.random.default_rng(12)
    lk = rng.integers(0, 1 << 63, size=50_000, dtype=np.uint64)
    lv = rng.integers(0, 1 << 64, size=50_000, dtype=np.uint64, endpoint=False)
    orc = SkipList()
    orc.bulk_load(lk, lv)
    ok, _ = orc.export()
    sets = [_ranges(rng, ok, 3_000), _ranges(rng, ok, 5_000)]
    with Index() as ix:
        ix.bulk_load(lk, lv)
        dev = [(to_device_u64(lo, ix.device), to_device_u64(hi, ix.device)) for lo, hi in sets]
        offs = [ix.range_count(lo, hi) for lo, hi in dev]
        for j in (0, 1, 1):  # the other set's count came last; then the same set twice
            lo, hi = dev[j]
            total = int(offs[j][-1].item())
            gk, gv = ix.range_collect(lo, hi, offs[j], total)
            torch.cuda.synchronize()
            wc, wk, wv = orc.range_batch(*sets[j])
            assert np.array_equal((offs[j][1:] - offs[j][:-1]).cpu().numpy().astype(np.uint64), wc)
            assert np.array_equal(to_numpy_u64(gk), wk) and np.array_equal(to_numpy_u64(gv), wv), j


def test_range_collect_after_a_group_rebuild():
    """A range count, then a group call in which the index sits out but its
    rebuild policy acts on the counters of the call before (the storage is
    merged, so slots move), then the collect of the same ranges: the collect
    must not reuse the count's interceptions, and gives the oracle's pairs."""
    from paper_1601_00159_amd.index import Group
    from paper_1601_00159_amd.index import to_device_u8 as d8
    rng = np.random.default_rng(21)
    lk = np.unique(rng.integers(0, 1 << 63, size=40_000, dtype=np.uint64))
    lv = rng.integers(0, 1 << 64, size=lk.size, dtype=np.uint64, endpoint=False)
    orc = SkipList()
    orc.bulk_load(lk, lv)
    dev = torch.device("cuda", 0)

    def batch(n):
        ops = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=n, p=[0.4, 0.4, 0.2])
        keys = np.where(ops == 1, rng.integers(0, 1 << 63, size=n, dtype=np.uint64), lk[rng.integers(0, lk.size, n)])
        vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
        return ops, keys.astype(np.uint64), vals

    def dev_batch(ops, keys, vals):
        return (d8(ops, dev), to_device_u64(keys, dev), to_device_u64(vals, dev),
                torch.empty(len(keys), dtype=torch.int64, device=dev),
                torch.empty(len(keys), dtype=torch.uint8, device=dev))

    with Index(rebuild_policy="threshold", rebuild_fraction=0.01, rebuild_min=1) as a, Index() as b, Group() as g:
        a.bulk_load(lk, lv)
        b.bulk_load(lk, lv)
        ops, keys, vals = batch(30_000)  # ~12K new nodes: the next call rebuilds a
        wv, ws = orc.execute_batch(ops, keys, vals)
        ba = dev_batch(ops, keys, vals)
        g.execute([a, b], [ba, dev_batch(*batch(1_000))])
        torch.cuda.synchronize()
        assert_same(to_numpy_u64(ba[3]), ba[4].cpu().numpy(), wv, ws, "group call")
        rep0 = a.stats()["repairs"]
        ok, _ = orc.export()
        lo, hi = _ranges(rng, ok, 4_000)
        dlo, dhi = to_device_u64(lo, a.device), to_device_u64(hi, a.device)
        off = a.range_count(dlo, dhi)
        torch.cuda.synchronize()
        g.execute([b], [dev_batch(*batch(1_000))])  # a sits out; its policy rebuilds it
        torch.cuda.synchronize()
        assert a.stats()["repairs"] > rep0, "the call did not rebuild the index that sat out"
        total = int(off[-1].item())
        gk, gv = a.range_collect(dlo, dhi, off, total)
        torch.cuda.synchronize()
        wc, wk, wv2 = orc.range_batch(lo, hi)
        assert np.array_equal((off[1:] - off[:-1]).cpu().numpy().astype(np.uint64), wc)
        assert np.array_equal(to_numpy_u64(gk), wk) and np.array_equal(to_numpy_u64(gv), wv2)


def test_range_search_edges():
    with Index() as ix:
        off = ix.range_count(np.zeros(0, dtype=np.uint64), np.zeros(0, dtype=np.uint64))
        assert off.cpu().tolist() == [0]
        c, k, v = ix.range_search(np.array([0, 5], dtype=np.uint64), np.array([KMAX, 1], dtype=np.uint64))
        assert c.cpu().tolist() == [0, 0] and k.numel() == 0          # empty index
        ix.bulk_load(np.array([3, 7, 11], dtype=np.uint64), np.array([30, 70, 110], dtype=np.uint64))
        c, k, v = ix.range_search(np.array([0, 7, 8, 12, 0], dtype=np.uint64),
                                  np.array([KMAX, 11, 10, KMAX, 3], dtype=np.uint64))
        assert c.cpu().tolist() == [3, 2, 0, 0, 1]
        assert to_numpy_u64(k).tolist() == [3, 7, 11, 7, 11, 3]
        assert to_numpy_u64(v).tolist() == [30, 70, 110, 70, 110, 30]


# ------------------------------------------------------------ serving loop

def test_serving_loop_matches_serial_replay():
    """Continuous batching (pi_serve): every answer and the final set equal
    the serial replay of the whole arrival stream, whatever the batching --
    the same stream served with different deadlines, batch caps and slot
    counts gives identical answers."""
    w = W.serving(load_log2=16, rate_qps=100e6, n_queries=300_000)
    ms = mapref.MapState(w.load_keys, w.load_vals)
    wv, ws = ms.apply_batch(w.ops, w.keys, w.vals)
    runs = []
    for deadline, cap, inflight in [(100.0, 0, 4), (0.0, 0, 1), (20.0, 1000, 2)]:
        with Index() as ix:
            ix.bulk_load(w.load_keys, w.load_vals)
            torch.cuda.synchronize()
            gv, gs, done, ends = ix.serve(w.arrival_us, w.ops, w.keys, w.vals, deadline_us=deadline,
                                          max_batch=cap, max_inflight=inflight)
            torch.cuda.synchronize()
            gv, gs = to_numpy_u64(gv), gs.cpu().numpy()
            say(f"deadline {deadline} cap {cap} inflight {inflight}: {ends.size} micro-batches, "
                f"p99 latency {np.percentile(done - w.arrival_us, 99):.1f} us")
            assert_same(gv, gs, wv, ws, f"serve deadline={deadline}")
            assert ends[-1] == w.ops.size and np.all(np.diff(ends) > 0) and ends[0] > 0
            if cap:
                assert np.max(np.diff(np.concatenate([[0], ends]))) <= cap
            # a micro-batch is launched only once its queries have arrived
            assert np.all(done >= w.arrival_us - 50.0)
            ek, ev = export_np(ix)
            assert np.array_equal(ek, ms.keys) and np.array_equal(ev, ms.vals)
            runs.append(ends.size)
    assert len(set(runs)) > 1  # the batchings differed


def test_graph_replays_match_eager_batches():
    """Small batches replay a captured graph (padded to a power of two with
    invalid queries).  The same sequence of batches -- sizes across several
    classes, repeats of one class, a rebuild in between that forces a new
    capture -- gives the oracle's answers and final set through both the
    graph path and the eager path, replay after replay, with host
    synchronisation between them, and the two paths keep equal counters."""
    rng = np.random.default_rng(77)
    lk = rng.integers(0, 1 << 63, size=100_000, dtype=np.uint64)
    lv = rng.integers(0, 1 << 64, size=100_000, dtype=np.uint64, endpoint=False)
    pool = np.concatenate([lk[:50_000], rng.integers(0, 1 << 63, size=50_000, dtype=np.uint64)])
    sizes = [1, 100, 4096, 4097, 5000, 5000, 5000, 70_000, 3000, 262_144, 9]
    batches = [_random_batch(rng, pool, n) for n in sizes]
    orc = SkipList()
    orc.bulk_load(lk, lv)
    want = [orc.execute_batch(*b) for b in batches]
    want_k, want_v = orc.export()
    res = {}
    for mode, glog in (("eager", 0), ("graph", 18)):
        with Index(rebuild_policy="never", graph_max_log2=glog) as ix:
            ix.bulk_load(lk, lv)
            out = []
            for b, (ops, keys, vals) in enumerate(batches):
                if b == 8:
                    ix.repair()  # new levels and storage: the graphs must be captured again
                out.append(run_gpu(ix, ops, keys, vals))
            res[mode] = (out, export_np(ix), ix.stats())
    for mode in ("eager", "graph"):
        for b in range(len(sizes)):
            assert_same(*res[mode][0][b], *want[b], f"{mode} batch {b} (n={sizes[b]}) against the oracle")
        assert np.array_equal(res[mode][1][0], want_k) and np.array_equal(res[mode][1][1], want_v), mode
    for k in ("queries", "hits", "invalid", "new_nodes", "deletes", "revives", "live_nodes"):
        assert res["graph"][2][k] == res["eager"][2][k], k


@pytest.mark.parametrize("policy", ["never", "always"])
def test_small_batches_in_one_workgroup(policy):
    """Batches of at most 4096 queries run as one workgroup (sort, descent,
    ownership, apply and linking in one launch).  Against the oracle: hot
    keys, chains of new nodes behind one predecessor, deletes, revives,
    invalid queries, batch sizes across the power-of-two edges, over linked
    and rebuilt storage."""
    rng = np.random.default_rng({"never": 5, "always": 6}[policy])
    lk = (rng.integers(0, 1 << 40, size=20_000, dtype=np.uint64) << np.uint64(8))  # room for keys in between
    lv = rng.integers(0, 1 << 64, size=20_000, dtype=np.uint64, endpoint=False)
    pool = np.concatenate([lk[:5000], lk[:200] + np.uint64(1), lk[:200] + np.uint64(2), lk[:200] + np.uint64(3),
                           rng.integers(0, 1 << 48, size=3000, dtype=np.uint64), np.array([0], dtype=np.uint64)])
    orc = SkipList()
    orc.bulk_load(lk, lv)
    with Index(rebuild_policy=policy, small_batch_log2=12) as ix:
        ix.bulk_load(lk, lv)
        for b, n in enumerate([1, 2, 63, 64, 65, 1000, 4095, 4096, 4096, 3000, 4096, 17, 4096]):
            ops, keys, vals = _random_batch(rng, pool, n, p_invalid=0.02)
            if b % 4 == 1:
                keys[: n // 2] = pool[3]  # a hot key
            wv, ws = orc.execute_batch(ops, keys, vals)
            gv, gs = run_gpu(ix, ops, keys, vals)
            assert_same(gv, gs, wv, ws, f"batch {b} (n={n})")
        ek, ev = export_np(ix)
        ok, ov = orc.export()
        assert np.array_equal(ek, ok) and np.array_equal(ev, ov)
        st = ix.stats()
        assert st["live_nodes"] == len(orc)
        if policy == "never":
            assert st["overflow_nodes"] > 0
        # small and large paths agree on one state: a large batch after small ones
        ops, keys, vals = _random_batch(rng, pool, 50_000)
        wv, ws = orc.execute_batch(ops, keys, vals)
        gv, gs = run_gpu(ix, ops, keys, vals)
        assert_same(gv, gs, wv, ws, "large batch after small ones")


# ------------------------------------------------------- many indices

@pytest.mark.parametrize("fused_max,threads,policy", [(4096, 0, "threshold"), (0, 0, "threshold"),
                                                       (16384, 0, "threshold"), (0, 1, "threshold"),
                                                       (0, 2, "always"), (0, 0, "background"), (0, 0, "slices")])
def test_group_matches_each_index_alone(fused_max, threads, policy):
    """One batch on each of many indices per call (pi_group_execute): each
    index's answers and final set equal the serial replay of its own
    batches, whichever batches take the fused launch (fused_max 0: none;
    16384: chunks of 4096 in one workgroup), with the large batches and the
    rebuilds the policies start issued by one to four host threads."""
    from paper_1601_00159_amd.index import Group
    from paper_1601_00159_amd.index import to_device_u64 as d64, to_device_u8 as d8
    w = W.many_indices(n_indices=24, size_log2=(8, 15), batch_log2=(5, 14), n_rounds=4,
                       seed_id=10 + fused_max % 7 + threads + len(policy))
    dev = torch.device("cuda", 0)
    refs = [mapref.MapState(k, v) for k, v in w.loads]
    ixs = [Index(rebuild_policy=policy, rebuild_fraction=0.05, rebuild_min=1) for _ in w.loads]
    try:
        for ix, (k, v) in zip(ixs, w.loads):
            ix.bulk_load(k, v)
        with Group(fused_max=fused_max if fused_max else 1, host_threads=threads) as g:
            for r, batches in enumerate(w.rounds):
                dev_b = [(d8(b.ops, dev), d64(b.keys, dev), d64(b.vals, dev),
                          torch.empty(len(b), dtype=torch.int64, device=dev),
                          torch.empty(len(b), dtype=torch.uint8, device=dev)) for b in batches]
                # an index may sit out a call: in the first one, and in a
                # later one after a batch of its own (its rebuild policy
                # then acts on its own, beside the others' batches)
                out = {0: 3, 2: 5}.get(r)
                if out is not None:
                    dev_b[out] = None
                g.execute(ixs, dev_b)
                torch.cuda.synchronize()
                for i, b in enumerate(batches):
                    if dev_b[i] is None:
                        continue
                    wv, ws = refs[i].apply_batch(b.ops, b.keys, b.vals)
                    assert_same(to_numpy_u64(dev_b[i][3]), dev_b[i][4].cpu().numpy(), wv, ws,
                                f"round {r} index {i} (n={len(b)})")
        for i, ix in enumerate(ixs):
            ek, ev = export_np(ix)
            assert np.array_equal(ek, refs[i].keys) and np.array_equal(ev, refs[i].vals), i
        st = [ix.stats() for ix in ixs]
        print(f"  rebuilds {sum(x['repairs'] for x in st)}, slice rounds {sum(x['slice_rounds'] for x in st)}",
              flush=True)
        if policy in ("threshold", "always"):
            assert sum(x["repairs"] for x in st) > 0
    finally:
        for ix in ixs:
            ix.close()


def test_group_autotune_and_errors():
    from paper_1601_00159_amd._lib import PI_ERR_INVALID_ARG
    from paper_1601_00159_amd.index import Group
    from paper_1601_00159_amd.index import to_device_u64 as d64, to_device_u8 as d8
    w = W.many_indices(n_indices=8, size_log2=(10, 14), batch_log2=(6, 13), n_rounds=1, seed_id=20)
    dev = torch.device("cuda", 0)
    ixs = [Index() for _ in w.loads]
    try:
        for ix, (k, v) in zip(ixs, w.loads):
            ix.bulk_load(k, v)
        before = [export_np(ix) for ix in ixs]
        b = w.rounds[0]
        dev_b = [(d8(x.ops, dev), d64(x.keys, dev), d64(x.vals, dev), torch.empty(len(x), dtype=torch.int64, device=dev),
                  torch.empty(len(x), dtype=torch.uint8, device=dev)) for x in b]
        with Group() as g:
            t = g.autotune(ixs, dev_b)
            assert t in (0, 1024, 4096, 16384, 32768, 65536, 131072, 262144, 524288, 1048576)
            ft, blk, lds = g.tuning()
            assert ft == t
            if any(len(x) > t for x in b):  # the descent shape was tuned and applied
                assert blk in (256, 512, 1024) and 3000 <= lds <= 12000
                assert all(ix.stats()["lds_from"] >= 2 for ix in ixs)
            else:
                assert (blk, lds) == (0, 0)
            # the SEARCH-only replays left every index as it was
            for ix, (k0, v0) in zip(ixs, before):
                k1, v1 = export_np(ix)
                assert np.array_equal(k0, k1) and np.array_equal(v0, v1)
            # and the tuned group still gives every index its serial answers
            orcs = []
            for (k, v) in w.loads:
                o = SkipList()
                o.bulk_load(k, v)
                orcs.append(o)
            g.execute(ixs, dev_b)
            torch.cuda.synchronize()
            for j, (o, x) in enumerate(zip(orcs, b)):
                wv, ws = o.execute_batch(x.ops, x.keys, x.vals)
                assert_same(to_numpy_u64(dev_b[j][3]), dev_b[j][4].cpu().numpy(), wv, ws, f"index {j}")
            with pytest.raises(PiError) as e:
                g.execute([ixs[0], ixs[0]], [dev_b[0], dev_b[0]])  # one index twice
            assert e.value.status == PI_ERR_INVALID_ARG
    finally:
        for ix in ixs:
            ix.close()
    # batches too large to fuse: the descent shape is tuned, and applied
    w = W.many_indices(n_indices=2, size_log2=(14, 15), batch_log2=(18.3, 18.4), n_rounds=1, seed_id=21)
    ixs = [Index() for _ in w.loads]
    try:
        orcs = []
        for ix, (k, v) in zip(ixs, w.loads):
            ix.bulk_load(k, v)
            o = SkipList()
            o.bulk_load(k, v)
            orcs.append(o)
        b = w.rounds[0]
        dev_b = [(d8(x.ops, dev), d64(x.keys, dev), d64(x.vals, dev), torch.empty(len(x), dtype=torch.int64, device=dev),
                  torch.empty(len(x), dtype=torch.uint8, device=dev)) for x in b]
        with Group() as g:
            t = g.autotune(ixs, dev_b)
            ft, blk, lds = g.tuning()
            say(f"fused_max {t}, descent block {blk}, lds budget {lds}")
            assert ft == t and t < min(len(x) for x in b)
            assert blk in (256, 512, 1024) and 3000 <= lds <= 12000
            g.execute(ixs, dev_b)
            torch.cuda.synchronize()
            for j, (o, x) in enumerate(zip(orcs, b)):
                wv, ws = o.execute_batch(x.ops, x.keys, x.vals)
                assert_same(to_numpy_u64(dev_b[j][3]), dev_b[j][4].cpu().numpy(), wv, ws, f"index {j}")
    finally:
        for ix in ixs:
            ix.close()


# ---------------------------------------------------- background rebuild

@pytest.mark.parametrize("compact", [0, 30])
def test_background_index_rebuild(compact):
    """Rebuild policy BACKGROUND: the index layer is rebuilt over the base
    region and the new nodes on a second stream while batches go on, and
    switched in at a batch boundary; with a small compact_percent the
    storage is merged by full rebuilds too.  Every batch's answers and the
    final set against the oracle; the levels stay well formed."""
    rng = np.random.default_rng(40 + compact)
    lk = rng.integers(0, 1 << 63, size=100_000, dtype=np.uint64)
    lv = rng.integers(0, 1 << 64, size=100_000, dtype=np.uint64, endpoint=False)
    pool = np.concatenate([lk[:40_000], rng.integers(0, 1 << 63, size=60_000, dtype=np.uint64)])
    orc = SkipList()
    orc.bulk_load(lk, lv)
    with Index(rebuild_policy="background", rebuild_fraction=0.02, rebuild_min=1, compact_percent=compact) as ix:
        ix.bulk_load(lk, lv)
        for b in range(14):
            n = [30_000, 700, 30_000, 5000][b % 4]
            ops, keys, vals = _random_batch(rng, pool, n)
            wv, ws = orc.execute_batch(ops, keys, vals)
            gv, gs = run_gpu(ix, ops, keys, vals)
            assert_same(gv, gs, wv, ws, f"batch {b} (n={n})")
        ek, ev = export_np(ix)
        ok, ov = orc.export()
        assert np.array_equal(ek, ok) and np.array_equal(ev, ov)
        st = ix.stats()
        say(f"index rebuilds {st['index_rebuilds']}, full rebuilds {st['repairs']}, overflow {st['overflow_nodes']}")
        if compact:
            assert st["repairs"] >= 1  # the storage was merged (a full rebuild drops any build in flight)
        else:
            assert st["index_rebuilds"] >= 1 and st["repairs"] == 0
        prev = None
        for lvl in range(2, st["n_levels"] + 1):
            k, d = ix.level(lvl)
            k, d = to_numpy_u64(k), d.cpu().numpy().astype(np.int64)
            assert np.all(k[1:] > k[:-1]), lvl
            if prev is not None and k.size:
                assert np.array_equal(prev[d - 1], k), lvl  # each key sits on the level below
            prev = k
