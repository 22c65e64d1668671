"""Seeded synthetic workloads for the batched skip-list index.

This module only draws random inputs; it holds none of the index's own
arithmetic (no height rule, no search, no ordering of queries), so both the GPU
path and the CPU checker can consume the same arrays.

The paper measures on YCSB-generated query streams with uniform or Zipfian key
choice and update ratios of 0 / 5% / 50% (Section 6, parameter table and
Section 6.6).  YCSB itself is not used here: these generators reproduce its
shapes -- uniform or Zipf(theta) choice over the loaded keys, fresh uniform keys
for inserts, fixed op mixes -- at the sizes of the workloads below.

Every array comes from ``numpy.random.Generator(PCG64(SeedSequence([base,
stream, batch])))`` with ``base = 0x50490000 + 16 * workload_id``; streams:
0 loaded keys, 1 ops, 2 query keys, 3 values, 4 arrivals, 5 choice of source.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEARCH, INSERT, DELETE = 0, 1, 2
KEY_SPACE = 1 << 63  # loaded and fresh keys are uniform in [0, 2^63)

ST_LOAD, ST_OPS, ST_QKEYS, ST_VALS, ST_ARRIVAL, ST_SOURCE = range(6)


def rng_for(base: int, stream: int, batch: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([base, stream, batch])))


def workload_base(workload_id: int) -> int:
    return 0x50490000 + 16 * workload_id


def unique_uniform_keys(n: int, rng: np.random.Generator, hi: int = KEY_SPACE) -> np.ndarray:
    """n distinct uint64 keys uniform in [0, hi), in random order."""
    keys = np.zeros(0, dtype=np.uint64)
    while keys.size < n:
        need = n - keys.size
        draw = rng.integers(0, hi, size=need + need // 64 + 16, dtype=np.uint64)
        keys = np.unique(np.concatenate([keys, draw]))
    if keys.size > n:
        keys = rng.choice(keys, size=n, replace=False)
    return rng.permutation(keys)


def uniform_values(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)


class Zipf:
    """Zipf(theta) over ranks 0..n-1, P(r) proportional to (r+1)^-theta,
    sampled exactly by inverse CDF on a float64 cumulative table."""

    def __init__(self, n: int, theta: float):
        self.n = int(n)
        self.theta = float(theta)
        w = np.arange(1, self.n + 1, dtype=np.float64) ** (-self.theta)
        self.cdf = np.cumsum(w)
        self.cdf /= self.cdf[-1]

    def pmf(self, r):
        r = np.asarray(r)
        prev = np.where(r > 0, self.cdf[np.maximum(r - 1, 0)], 0.0)
        return self.cdf[r] - prev

    def sample(self, size: int, rng: np.random.Generator) -> np.ndarray:
        u = rng.random(size)
        r = np.searchsorted(self.cdf, u, side="right")
        return np.minimum(r, self.n - 1).astype(np.int64)


def draw_ops(n: int, mix, rng: np.random.Generator) -> np.ndarray:
    """iid ops with probabilities mix = (p_search, p_insert, p_delete)."""
    p = np.asarray(mix, dtype=np.float64)
    p = p / p.sum()
    return rng.choice(np.array([SEARCH, INSERT, DELETE], dtype=np.uint8), size=n, p=p)


@dataclass
class Batch:
    ops: np.ndarray
    keys: np.ndarray
    vals: np.ndarray

    def __len__(self):
        return int(self.ops.size)


@dataclass
class Workload:
    name: str
    load_keys: np.ndarray
    load_vals: np.ndarray
    batches: List[Batch] = field(default_factory=list)
    note: str = ""


def mixed_uniform(workload_id: int, n_load: int, n_query: int, n_batches: int = 1,
                  mix=(0.8, 0.1, 0.1), p_loaded: float = 0.5, name: str = "mixed-uniform") -> Workload:
    """Load n_load distinct uniform keys; batches of iid ops with the given
    mix; each query key is, with probability p_loaded, a uniformly chosen
    loaded key and otherwise a fresh uniform key in [0, 2^63)."""
    base = workload_base(workload_id)
    lk = unique_uniform_keys(n_load, rng_for(base, ST_LOAD))
    lv = uniform_values(n_load, rng_for(base, ST_VALS, 1 << 20))
    batches = []
    for b in range(n_batches):
        ops = draw_ops(n_query, mix, rng_for(base, ST_OPS, b))
        src = rng_for(base, ST_SOURCE, b).random(n_query) < p_loaded
        rq = rng_for(base, ST_QKEYS, b)
        fresh = rq.integers(0, KEY_SPACE, size=n_query, dtype=np.uint64)
        pick = lk[rq.integers(0, max(n_load, 1), size=n_query)] if n_load else fresh
        keys = np.where(src, pick, fresh).astype(np.uint64)
        vals = uniform_values(n_query, rng_for(base, ST_VALS, b))
        batches.append(Batch(ops, keys, vals))
    return Workload(name, lk, lv, batches,
                    note=f"load {n_load} uniform keys; {n_batches} x {n_query} queries, mix {mix}, "
                         f"{p_loaded:.0%} of keys drawn from the loaded set")


def search_only(workload_id: int, n_load: int, n_query: int, n_batches: int,
                theta: Optional[float] = None, name: str = "search") -> Workload:
    """All-SEARCH batches; keys uniform over the loaded keys (theta None) or
    Zipf(theta) over them (rank r -> the r-th loaded key, which is a seeded
    random permutation of the key space)."""
    base = workload_base(workload_id)
    lk = unique_uniform_keys(n_load, rng_for(base, ST_LOAD))
    lv = uniform_values(n_load, rng_for(base, ST_VALS, 1 << 20))
    z = Zipf(n_load, theta) if theta else None
    batches = []
    for b in range(n_batches):
        rq = rng_for(base, ST_QKEYS, b)
        idx = z.sample(n_query, rq) if z is not None else rq.integers(0, n_load, size=n_query)
        keys = lk[idx]
        batches.append(Batch(np.zeros(n_query, dtype=np.uint8), keys, np.zeros(n_query, dtype=np.uint64)))
    dist = f"Zipf theta={theta}" if theta else "uniform"
    return Workload(name, lk, lv, batches,
                    note=f"load {n_load} uniform keys; {n_batches} x {n_query} SEARCH, keys {dist} over loaded keys")


def write_heavy(workload_id: int, n_load: int, n_query: int, n_batches: int,
                theta: float = 0.99, mix=(0.4, 0.5, 0.1), name: str = "write-heavy") -> Workload:
    """INSERT keys are fresh uniform keys; SEARCH and DELETE keys are
    Zipf(theta) over the originally loaded keys."""
    base = workload_base(workload_id)
    lk = unique_uniform_keys(n_load, rng_for(base, ST_LOAD))
    lv = uniform_values(n_load, rng_for(base, ST_VALS, 1 << 20))
    z = Zipf(n_load, theta)
    batches = []
    for b in range(n_batches):
        ops = draw_ops(n_query, mix, rng_for(base, ST_OPS, b))
        rq = rng_for(base, ST_QKEYS, b)
        fresh = rq.integers(0, KEY_SPACE, size=n_query, dtype=np.uint64)
        hot = lk[z.sample(n_query, rq)]
        keys = np.where(ops == INSERT, fresh, hot).astype(np.uint64)
        vals = uniform_values(n_query, rng_for(base, ST_VALS, b))
        batches.append(Batch(ops, keys, vals))
    return Workload(name, lk, lv, batches,
                    note=f"load {n_load} uniform keys; {n_batches} x {n_query} queries mix {mix} "
                         f"(S/I/D), inserts fresh uniform, others Zipf theta={theta}")


# --- the named workloads -----------------------------------------------------

def plain_pi(scale: int = 20) -> Workload:
    """2^scale loaded keys, one batch of 2^scale queries, 80/10/10, half of the
    query keys drawn from the loaded set (full size: scale 20)."""
    return mixed_uniform(1, 1 << scale, 1 << scale, 1, (0.8, 0.1, 0.1), 0.5, name=f"plain-pi-2^{scale}")


def read_scaling(theta: Optional[float] = None, load_log2: int = 24, query_log2: int = 22,
                 n_batches: int = 32) -> Workload:
    return search_only(2, 1 << load_log2, 1 << query_log2, n_batches, theta,
                       name=f"search-2^{load_log2}-{'zipf' + str(theta) if theta else 'uniform'}")


def write_skew(load_log2: int = 26, query_log2: int = 22, n_batches: int = 16) -> Workload:
    return write_heavy(3, 1 << load_log2, 1 << query_log2, n_batches, 0.99, (0.4, 0.5, 0.1),
                       name=f"write-skew-2^{load_log2}")


def headline(theta: Optional[float] = None, load_log2: int = 26, query_log2: int = 22,
             n_batches: int = 32) -> Workload:
    """64M-key search workload: 2^26 loaded keys, batches of 2^22 SEARCH."""
    return search_only(6, 1 << load_log2, 1 << query_log2, n_batches, theta,
                       name=f"search-2^{load_log2}-{'zipf' + str(theta) if theta else 'uniform'}")


@dataclass
class RangeWorkload:
    name: str
    load_keys: np.ndarray
    load_vals: np.ndarray
    batches: List[tuple] = field(default_factory=list)  # (lo, hi) arrays
    note: str = ""


def range_scan(load_log2: int = 26, n_ranges: int = 8192, granularity: int = 100,
               n_batches: int = 8) -> RangeWorkload:
    """Range searches over 2^load_log2 uniform keys (the paper's range-query
    experiment, Section 6: batches of 8192 range queries, granularity = mean
    number of keys per range).  lo is a uniformly chosen loaded key and
    hi = lo + U(0, 2) * granularity * (mean gap between loaded keys)."""
    base = workload_base(7)
    n_load = 1 << load_log2
    lk = unique_uniform_keys(n_load, rng_for(base, ST_LOAD))
    lv = uniform_values(n_load, rng_for(base, ST_VALS, 1 << 20))
    gap = KEY_SPACE / n_load
    batches = []
    for b in range(n_batches):
        rq = rng_for(base, ST_QKEYS, (granularity << 8) + b)
        lo = lk[rq.integers(0, n_load, size=n_ranges)]
        width = (rq.random(n_ranges) * 2.0 * granularity * gap).astype(np.uint64)
        batches.append((lo, lo + width))
    return RangeWorkload(f"range-2^{load_log2}-g{granularity}", lk, lv, batches,
                         note=f"load {n_load} uniform keys; {n_batches} x {n_ranges} ranges, "
                              f"about {granularity} keys per range")


@dataclass
class ServingWorkload:
    name: str
    load_keys: np.ndarray
    load_vals: np.ndarray
    arrival_us: np.ndarray   # float64, non-decreasing
    ops: np.ndarray
    keys: np.ndarray
    vals: np.ndarray
    note: str = ""


def serving(load_log2: int = 25, rate_qps: float = 200e6, n_queries: int = 1 << 22, theta: float = 0.8,
            mix=(0.9, 0.05, 0.05)) -> ServingWorkload:
    """Open-loop Poisson arrivals at rate_qps (seeded exponential gaps) of
    queries with the given S/I/D mix; SEARCH and DELETE keys Zipf(theta) over
    the loaded keys, INSERT keys fresh uniform."""
    base = workload_base(8)
    n_load = 1 << load_log2
    lk = unique_uniform_keys(n_load, rng_for(base, ST_LOAD))
    lv = uniform_values(n_load, rng_for(base, ST_VALS, 1 << 20))
    ra = rng_for(base, ST_ARRIVAL, int(rate_qps // 1000))
    gaps = ra.exponential(1e6 / rate_qps, size=n_queries)
    arrival = np.cumsum(gaps)
    ops = draw_ops(n_queries, mix, rng_for(base, ST_OPS))
    rq = rng_for(base, ST_QKEYS)
    fresh = rq.integers(0, KEY_SPACE, size=n_queries, dtype=np.uint64)
    hot = lk[Zipf(n_load, theta).sample(n_queries, rq)]
    keys = np.where(ops == INSERT, fresh, hot).astype(np.uint64)
    vals = uniform_values(n_queries, rng_for(base, ST_VALS))
    return ServingWorkload(f"serve-2^{load_log2}-{rate_qps / 1e6:g}Mqps", lk, lv, arrival, ops, keys, vals,
                           note=f"load {n_load} keys; {n_queries} Poisson arrivals at {rate_qps / 1e6:g} M/s, "
                                f"mix {mix}, Zipf theta={theta}")


@dataclass
class ManyIndexWorkload:
    name: str
    loads: List[tuple]            # per index (keys, values)
    rounds: List[List[Batch]]     # per round, per index
    note: str = ""


def many_indices(n_indices: int = 512, size_log2=(10, 22), batch_log2=(8, 18), n_rounds: int = 2,
                 mix=(0.9, 0.05, 0.05), seed_id: int = 9) -> ManyIndexWorkload:
    """Independent indices with sizes log-uniform in 2^size_log2 and per-index
    batches log-uniform in 2^batch_log2; SEARCH and DELETE keys uniform over
    that index's loaded keys, INSERT keys fresh uniform."""
    base = workload_base(seed_id)
    rs = rng_for(base, ST_SOURCE)
    sizes = np.round(2.0 ** rs.uniform(size_log2[0], size_log2[1], size=n_indices)).astype(np.int64)
    loads = []
    for i in range(n_indices):
        lk = unique_uniform_keys(int(sizes[i]), rng_for(base, ST_LOAD, i))
        lv = uniform_values(int(sizes[i]), rng_for(base, ST_VALS, (1 << 20) + i))
        loads.append((lk, lv))
    rounds = []
    for r in range(n_rounds):
        rb = rng_for(base, ST_SOURCE, 1 + r)
        nq = np.round(2.0 ** rb.uniform(batch_log2[0], batch_log2[1], size=n_indices)).astype(np.int64)
        batches = []
        for i in range(n_indices):
            n = int(nq[i])
            seq = (r << 16) + i
            ops = draw_ops(n, mix, rng_for(base, ST_OPS, seq))
            rq = rng_for(base, ST_QKEYS, seq)
            fresh = rq.integers(0, KEY_SPACE, size=n, dtype=np.uint64)
            lk = loads[i][0]
            pick = lk[rq.integers(0, lk.size, size=n)]
            keys = np.where(ops == INSERT, fresh, pick).astype(np.uint64)
            vals = uniform_values(n, rng_for(base, ST_VALS, seq))
            batches.append(Batch(ops, keys, vals))
        rounds.append(batches)
    return ManyIndexWorkload(f"many-{n_indices}-indices", loads, rounds,
                             note=f"{n_indices} indices, sizes 2^{size_log2[0]}..2^{size_log2[1]} "
                                  f"(total {int(sizes.sum())} keys), batches 2^{batch_log2[0]}..2^{batch_log2[1]}, "
                                  f"mix {mix}")
