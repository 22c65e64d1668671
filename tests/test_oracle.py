"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* published test vectors of the splitmix64 finalizer (height rule);
* the geometric level occupancy the paper requires of tower heights;
* brute force over a sorted list of pairs, exhaustively on tiny inputs;
* a Python dict replay (the plain definition) on random batches;
* hand-worked examples E1 and E2 (tests/golden);
* structural invariants of a skip list;
* Definition 4 (interception) by brute force;
* Algorithm 3 on the E1 trace and the latch-free invariant.
"""
import bisect
import itertools
import json
import math
import os
import random

import numpy as np
import pytest

from oracle import mapref, redistribute
from oracle.skiplist import (ABSENT, DELETE, INSERT, INVALID, PRESENT, SEARCH, SkipList,
                             height_rule, mix64)

OPS = {"SEARCH": SEARCH, "INSERT": INSERT, "DELETE": DELETE}
KMAX = (1 << 64) - 1


# --------------------------------------------------------------- height rule

def test_mix64_published_vectors():
    # splitmix64 seeded with 0: state advances by the golden gamma, each output
    # is the finalizer of the state.  Published first three outputs.
    gamma = 0x9E3779B97F4A7C15
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    state = 0
    for e in expect:
        state = (state + gamma) & KMAX
        assert mix64(state) == e


def test_height_rule_special_cases():
    seed = 0x1234_5678_9ABC_DEF0
    # the finalizer maps 0 to 0, so key == seed gives ctz(0)=64: the cap
    assert height_rule(seed, seed, 1, 24) == 24
    assert height_rule(seed, seed, 2, 24) == 24
    assert height_rule(seed, seed, 1, 5) == 5
    # height 1 exactly when the mixed word is odd (p = 1/2)
    for k in range(200):
        z = mix64(k ^ seed)
        assert (height_rule(k, seed, 1, 24) == 1) == bool(z & 1)
        assert (height_rule(k, seed, 2, 24) == 1) == bool(z & 3)


@pytest.mark.parametrize("log2_inv_p", [1, 2])
def test_height_rule_geometric_occupancy(log2_inv_p):
    # Section 3.2: heights are geometric; #keys with height >= h is
    # Binomial(N, p^(h-1)).  Check every level within 6 sigma.
    rng = np.random.default_rng(7)
    keys = np.unique(rng.integers(0, 1 << 63, size=200_000, dtype=np.uint64))
    n = keys.size
    seed = 0x9E3779B97F4A7C15
    hs = np.array([height_rule(int(k), seed, log2_inv_p, 24) for k in keys])
    p = 2.0 ** -log2_inv_p
    for h in range(1, 12):
        q = p ** (h - 1)
        cnt = int((hs >= h).sum())
        mu = n * q
        sd = math.sqrt(n * q * (1 - q)) + 1e-9
        assert abs(cnt - mu) <= 6 * sd + 1, (h, cnt, mu)


# ------------------------------------------------------------- brute force

class SortedPairs:
    """Brute force: a sorted Python list of [key, value] pairs."""

    def __init__(self, pairs=()):
        self.keys, self.vals = [], []
        for k, v in pairs:
            self.insert(k, v)

    def find(self, k):
        for kk, vv in zip(self.keys, self.vals):
            if kk == k:
                return PRESENT, vv
        return ABSENT, 0

    def insert(self, k, v):
        r = self.find(k)
        i = bisect.bisect_left(self.keys, k)
        if i < len(self.keys) and self.keys[i] == k:
            self.vals[i] = v
        else:
            self.keys.insert(i, k)
            self.vals.insert(i, v)
        return r

    def erase(self, k):
        r = self.find(k)
        if r[0] == PRESENT:
            i = self.keys.index(k)
            del self.keys[i]
            del self.vals[i]
        return r

    def run(self, ops, keys, vals):
        out = []
        for op, k, v in zip(ops, keys, vals):
            if op > DELETE or k == KMAX:
                out.append((INVALID, 0))
            elif op == SEARCH:
                out.append(self.find(k))
            elif op == INSERT:
                out.append(self.insert(k, v))
            else:
                out.append(self.erase(k))
        return out


def _oracle_run(initial, ops, keys, vals, **kw):
    s = SkipList(**kw)
    if initial:
        s.bulk_load(np.array([k for k, _ in initial], dtype=np.uint64),
                    np.array([v for _, v in initial], dtype=np.uint64))
    ov, os_ = s.execute_batch(np.array(ops, dtype=np.uint8), np.array(keys, dtype=np.uint64),
                              np.array(vals, dtype=np.uint64))
    res = list(zip(os_.tolist(), ov.tolist()))
    ek, ev = s.export()
    assert s.check() == 0
    return res, list(zip(ek.tolist(), ev.tolist()))


def test_exhaustive_tiny_vs_brute_force():
    universe = [3, 10, 17]
    initials = [[], [(10, 1)], [(3, 7), (17, 9)]]
    choices = [(op, k) for op in (SEARCH, INSERT, DELETE) for k in universe]
    n_cases = 0
    for init in initials:
        for length in range(1, 5):
            for seq in itertools.product(choices, repeat=length):
                ops = [c[0] for c in seq]
                keys = [c[1] for c in seq]
                vals = [100 + i for i in range(length)]
                bf = SortedPairs(init)
                want = bf.run(ops, keys, vals)
                got, final = _oracle_run(init, ops, keys, vals, max_height=4)
                assert got == want, (init, seq)
                assert final == list(zip(bf.keys, bf.vals))
                n_cases += 1
    assert n_cases == 3 * (9 + 81 + 729 + 6561)


def test_random_longer_vs_brute_force():
    rng = random.Random(11)
    for trial in range(300):
        universe = rng.sample(range(0, 60), 8) + [0]
        n = rng.randint(1, 40)
        ops = [rng.choice([0, 0, 1, 1, 2, 3]) for _ in range(n)]
        keys = [rng.choice(universe + [KMAX]) for _ in range(n)]
        vals = [rng.randrange(0, 1 << 64) for _ in range(n)]
        init = [(k, rng.randrange(1 << 64)) for k in rng.sample(universe, rng.randint(0, 6))]
        bf = SortedPairs(init)
        want = bf.run(ops, keys, vals)
        got, final = _oracle_run(init, ops, keys, vals, max_height=6)
        assert got == want
        assert final == list(zip(bf.keys, bf.vals))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_vs_dict_replay(seed):
    rng = np.random.default_rng(seed)
    n_load, n_q = 20_000, 60_000
    lk = rng.integers(0, 1 << 63, size=n_load, dtype=np.uint64)
    lk[:100] = lk[100:200]  # duplicated loaded keys: last occurrence wins
    lv = rng.integers(0, 1 << 63, size=n_load, dtype=np.uint64)
    ops = rng.choice(np.array([0, 1, 2, 5], dtype=np.uint8), size=n_q, p=[0.5, 0.3, 0.19, 0.01])
    pool = np.concatenate([lk[:2000], rng.integers(0, 1 << 63, size=2000, dtype=np.uint64),
                           np.array([KMAX], dtype=np.uint64)])
    keys = pool[rng.integers(0, pool.size, size=n_q)]
    vals = rng.integers(0, 1 << 63, size=n_q, dtype=np.uint64)
    m = {}
    for k, v in zip(lk.tolist(), lv.tolist()):
        m[k] = v
    want_v, want_s = mapref.replay_dict(m, ops.tolist(), keys.tolist(), vals.tolist())
    s = SkipList()
    s.bulk_load(lk, lv)
    got_v, got_s = s.execute_batch(ops, keys, vals)
    assert got_s.tolist() == want_s
    assert got_v.tolist() == want_v
    ek, ev = s.export()
    assert ek.tolist() == sorted(m)
    assert ev.tolist() == [m[k] for k in sorted(m)]
    assert s.check() == 0
    # the sorted-array replay used at large sizes gives the same thing
    ms = mapref.MapState(lk, lv)
    mv, mst = ms.apply_batch(ops, keys, vals)
    assert mst.tolist() == want_s and mv.tolist() == want_v
    assert ms.keys.tolist() == sorted(m)


def test_bulk_load_sorted_equals_sequential():
    rng = np.random.default_rng(5)
    k = rng.integers(0, 1 << 63, size=30_000, dtype=np.uint64)
    v = rng.integers(0, 1 << 63, size=30_000, dtype=np.uint64)
    a = SkipList()
    a.bulk_load(k, v)
    uk, uv = mapref.dedupe_last(k, v)
    b = SkipList()
    b.bulk_load_sorted(uk, uv)
    assert a.check() == 0 and b.check() == 0
    for lvl in range(1, 25):
        assert a.level_keys(lvl).tolist() == b.level_keys(lvl).tolist()


# ------------------------------------------------------------------ golden

def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _batch(g):
    ops = [OPS[o] if isinstance(o, str) else o for o, _, _ in g["batch"]]
    keys = [k for _, k, _ in g["batch"]]
    vals = [v for _, _, v in g["batch"]]
    return ops, keys, vals


def test_golden_e1(golden_dir):
    g = _load(golden_dir, "e1_duplicates_revive.json")
    s = SkipList(max_height=4)
    for (k, v), h in zip(g["initial"], g["forced_heights"]):
        s.force_height(h)
        s.insert(k, v)
    s.force_height(0)
    assert s.level_keys(2).tolist() == [10, 30, 50]
    assert s.level_keys(3).tolist() == [30]
    ops, keys, vals = _batch(g)
    # Definition 4 on the initial structure, in stable key order
    order = sorted(range(len(keys)), key=lambda i: (keys[i], i))
    assert order == g["sorted_order"]
    icpt = [s.interception(keys[i]) for i in order]
    assert icpt == g["interceptions_by_sorted_query"]
    seg = [0]
    for a, b in zip(icpt, icpt[1:]):
        seg.append(seg[-1] + (a != b))
    assert seg == g["segment_ids_by_sorted_query"]
    owner = redistribute.redistribute(icpt, 3)
    assert owner == g["three_worker_owner_by_sorted_query"]
    assert redistribute.check_latch_free(icpt, owner)
    s.force_height(1)  # new keys of the batch stay at height 1 as in the example
    ov, os_ = s.execute_batch(np.array(ops, dtype=np.uint8), np.array(keys, dtype=np.uint64),
                              np.array(vals, dtype=np.uint64))
    assert [list(x) for x in zip(os_.tolist(), ov.tolist())] == g["expected"]
    ek, ev = s.export()
    assert [list(x) for x in zip(ek.tolist(), ev.tolist())] == g["final"]


def test_golden_e2(golden_dir):
    g = _load(golden_dir, "e2_empty_and_edges.json")
    ops, keys, vals = _batch(g)
    s = SkipList()
    ov, os_ = s.execute_batch(np.array(ops, dtype=np.uint8), np.array(keys, dtype=np.uint64),
                              np.array(vals, dtype=np.uint64))
    assert [list(x) for x in zip(os_.tolist(), ov.tolist())] == g["expected"]
    ek, ev = s.export()
    assert [list(x) for x in zip(ek.tolist(), ev.tolist())] == g["final"]
    # an empty batch changes nothing
    e = np.zeros(0, dtype=np.uint64)
    ov, os_ = s.execute_batch(np.zeros(0, dtype=np.uint8), e, e)
    assert ov.size == 0 and len(s) == 3


def test_golden_via_dict_replay(golden_dir):
    for name in ("e1_duplicates_revive.json", "e2_empty_and_edges.json"):
        g = _load(golden_dir, name)
        ops, keys, vals = _batch(g)
        m = {k: v for k, v in g["initial"]}
        ov, os_ = mapref.replay_dict(m, ops, keys, vals)
        assert [list(x) for x in zip(os_, ov)] == g["expected"]
        assert sorted(m.items()) == [tuple(x) for x in g["final"]]


# --------------------------------------------------------------- structure

def test_invariants_and_interception_brute_force():
    rng = np.random.default_rng(21)
    seed = 0x9E3779B97F4A7C15
    k = rng.integers(0, 1 << 40, size=20_000, dtype=np.uint64)
    v = rng.integers(0, 1 << 63, size=20_000, dtype=np.uint64)
    s = SkipList()
    s.bulk_load(k, v)
    ops = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=20_000)
    qk = np.concatenate([k[:10_000], rng.integers(0, 1 << 40, size=10_000, dtype=np.uint64)])
    s.execute_batch(ops, qk, v)
    assert s.check() == 0
    keys = s.export()[0].tolist()
    # level l holds exactly the keys whose height is >= l, in order
    hs = {kk: height_rule(kk, seed, 1, 24) for kk in keys}
    for lvl in range(1, 25):
        assert s.level_keys(lvl).tolist() == [kk for kk in keys if hs[kk] >= lvl]
    # Definition 4: the largest key of height > 1 that is <= q
    idx = [kk for kk in keys if hs[kk] > 1]
    for q in rng.integers(0, 1 << 40, size=3000, dtype=np.uint64).tolist() + [0, keys[0], idx[0],
                                                                             idx[-1], (1 << 40)]:
        j = bisect.bisect_right(idx, q)
        want = idx[j - 1] if j else None
        assert s.interception(q) == want


def test_alg3_random_latch_free():
    rng = random.Random(3)
    for trial in range(300):
        n = rng.randint(0, 80)
        vals = sorted(rng.randint(0, 30) for _ in range(n))
        icpt = [None if x < 3 else (x // 4) * 4 for x in vals]
        w = rng.randint(1, 9)
        owner = redistribute.redistribute(icpt, w)
        assert all(o is not None for o in owner)
        assert redistribute.check_latch_free(icpt, owner)


def test_alg3_checker_catches_a_planted_split():
    # a split segment (two owners for one interception) must be rejected
    icpt = [None, 10, 10, 10, 30]
    assert not redistribute.check_latch_free(icpt, [0, 0, 1, 1, 1])
    assert redistribute.check_latch_free(icpt, [0, 1, 1, 1, 1])


# --------------------------------------------------------------- range search

def _brute_range(pairs, lo, hi):
    """Every pair with lo <= key <= hi, by a linear scan of the sorted pairs."""
    return [(k, v) for k, v in pairs if lo <= k <= hi]


def test_range_search_brute_force_and_special_cases():
    """The range query of Section 3.2.5 (SEARCH only): the oracle and the numpy
    reference against a linear scan, after inserts and deletes, with empty,
    reversed, single-key, full-span and out-of-span ranges."""
    rng = random.Random(31)
    s = SkipList()
    ref = SortedPairs()
    for _ in range(3000):
        k = rng.randrange(0, 5000)
        if rng.random() < 0.7:
            s.insert(k, k * 3 + 1)
            ref.insert(k, k * 3 + 1)
        else:
            s.erase(k)
            ref.erase(k)
    pairs = list(zip(ref.keys, ref.vals))
    lo = [rng.randrange(0, 5200) for _ in range(400)]
    hi = [x + rng.randrange(0, 300) for x in lo]
    present = ref.keys[len(ref.keys) // 2]
    lo += [0, 0, 10, present, 4000, 7000, 0, 6000]
    hi += [KMAX, 0, 9, present, 3999, 9000, (1 << 64) - 2, KMAX]
    counts, keys, vals = s.range_batch(np.array(lo, dtype=np.uint64), np.array(hi, dtype=np.uint64))
    ms = mapref.MapState(np.array(ref.keys, dtype=np.uint64), np.array(ref.vals, dtype=np.uint64))
    mc, mk, mv = ms.range_batch(np.array(lo, dtype=np.uint64), np.array(hi, dtype=np.uint64))
    off = 0
    for i, (a, b) in enumerate(zip(lo, hi)):
        want = _brute_range(pairs, a, b)
        got = list(zip(keys[off:off + int(counts[i])].tolist(), vals[off:off + int(counts[i])].tolist()))
        assert got == want, (i, a, b)
        off += int(counts[i])
    assert off == keys.size
    assert np.array_equal(counts, mc) and np.array_equal(keys, mk) and np.array_equal(vals, mv)
    # the special cases, spelled out
    n_all = len(pairs)
    assert counts[-8] == n_all and counts[-7] == (1 if ref.keys[0] == 0 else 0)
    assert counts[-6] == 0 and counts[-5] == 1 and counts[-4] == 0 and counts[-3] == 0
    assert counts[-2] == n_all and counts[-1] == 0


# ------------------------------------------------- self-check negative pins

@pytest.mark.parametrize("kind,code", [(1, 1), (2, 2), (3, 3), (4, 4)])
def test_self_check_rejects_planted_faults(kind, code):
    """orc_check is pinned both ways: it accepts every well-formed list built
    above, and it rejects each planted fault with that fault's code -- a level
    out of order (1), a level-2 key missing on level 1 (2), a height that
    differs from the rule (3), a size that differs from the level-1 count
    (4) -- and accepts the list again once the fault is undone."""
    rng = np.random.default_rng(50 + kind)
    keys = np.unique(rng.integers(0, 1 << 63, size=5000, dtype=np.uint64))
    s = SkipList()
    s.bulk_load(keys, keys)
    assert s.check() == 0
    assert s.plant(kind) == 0
    assert s.check() == code
    s.restore()
    assert s.check() == 0
    s.close()


def test_oracle_under_sanitizers(tmp_path):
    """The oracle's self-test driver (every entry point against a brute-force
    sorted array, planted faults included) built with AddressSanitizer and
    UndefinedBehaviorSanitizer: no memory error, no undefined behaviour, no
    leak, every answer right."""
    import shutil
    import subprocess

    from oracle import build as ob

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = ob.build_selftest(str(tmp_path / "selftest"), sanitize=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "selftest ok" in r.stdout
