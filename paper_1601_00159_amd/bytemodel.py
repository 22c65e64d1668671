"""Algorithmic memory traffic of the descent, for the roofline.

Two things live here:

* ``paper_cost_lines`` -- the cache-line count of the paper's performance
  model (Section 5.1): an index of height H = ceil(-log_P N) costs
  (H-1) * ceil(Se/Sl) * ceil((1+P)/(2PM)) lines in the index layer and
  ceil(Sn/Sl) * ceil((1+P)/(2P)) lines in the storage layer per search (the
  storage term is read without the /M that the printed formula carries: the
  storage layer has no entries, and only this reading gives the 3 lines of
  the paper's worked example).

* ``descent_bytes`` -- the exact number of bytes one descent launch must move
  for a given index and sorted batch, counted on a reference layout rather
  than on the kernel's own (so that padding cannot inflate it): per level a
  u64 key array and a u32 down array, each starting on a 128-byte line with
  the head entry at index 0; storage as u64 key and u64 value arrays indexed
  by slot (head = slot 0).  A query reads, on every level, the keys from the
  one after its start position up to the first key greater than it and the
  down pointer of the key it stops on; then the storage keys from its
  interception up to the first key greater than it, and the value of the node
  it stops on when that node holds its key.  Bytes = distinct 128-byte lines
  touched, times 128, plus the levels kept in LDS counted once at their full
  size, plus the sorted input read (12 B per query) and the answers written
  (9 B per query).

The height rule used to rebuild the levels is the library's (splitmix64
finalizer of key ^ seed, trailing zeros, capped): the model must see the same
levels as the kernel.
"""
import math

import numpy as np

LINE = 128
KEY_BYTES, DOWN_BYTES, VAL_BYTES = 8, 4, 8
KEYS_PER_LINE = LINE // KEY_BYTES
DOWNS_PER_LINE = LINE // DOWN_BYTES


def paper_cost_lines(N, P, M, entry_bytes, node_bytes, line_bytes):
    """(index lines, storage lines) per search of the Section 5.1 model."""
    H = math.ceil(-math.log(N) / math.log(P) - 1e-12)
    per_level = math.ceil(entry_bytes / line_bytes) * math.ceil((1 + P) / (2 * P * M))
    index_lines = (H - 1) * per_level
    storage_lines = math.ceil(node_bytes / line_bytes) * math.ceil((1 + P) / (2 * P))
    return index_lines, storage_lines


def paper_index_bytes(N, P, entry_bytes, node_bytes):
    """Index size as the worked example of Section 5.1 computes it: N data
    nodes plus N*P/(1-P) index keys, each charged a whole entry (the printed
    arithmetic, 20*512K + 1/3*48*512K = 18M, charges 48 bytes per index key
    although an entry holds 4 keys; this follows the printed figure)."""
    index_keys = N * P / (1 - P)
    return N * node_bytes + index_keys * entry_bytes


def heights(keys, seed=0x9E3779B97F4A7C15, log2_inv_p=1, max_height=24):
    """Tower heights of uint64 keys (vectorised)."""
    z = np.asarray(keys, dtype=np.uint64) ^ np.uint64(seed)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        low = z & (~z + np.uint64(1))
    tz = np.where(z == 0, 64, np.log2(np.where(z == 0, 1, low).astype(np.float64)).astype(np.int64))
    extra = np.minimum(tz // log2_inv_p, max_height - 1)
    return (1 + extra).astype(np.int64)


def build_levels(sorted_keys, h):
    """Level l (2..top) -> its keys in order."""
    levels = {}
    for l in range(2, int(h.max(initial=1)) + 1):
        k = sorted_keys[h >= l]
        if k.size:
            levels[l] = k
    return levels


def _distinct_lines(first, last):
    """Number of distinct line ids covered by the inclusive ranges [first, last]."""
    first = np.asarray(first, dtype=np.int64)
    last = np.asarray(last, dtype=np.int64)
    span = last - first
    parts = [first, last]
    wide = np.nonzero(span > 1)[0]
    if wide.size:
        extra = np.concatenate([np.arange(a + 1, b) for a, b in zip(first[wide], last[wide])])
        parts.append(extra)
    return np.unique(np.concatenate(parts)).size


def descent_bytes(sorted_keys, queries_sorted, lds_from=None, seed=0x9E3779B97F4A7C15, log2_inv_p=1,
                  max_height=24, level_pad=16, h=None, with_values=True):
    """Algorithmic bytes of one descent launch (see module docstring).

    sorted_keys: the index's keys, strictly increasing (slot i+1 holds
    sorted_keys[i]).  queries_sorted: the batch's keys in non-decreasing order.
    lds_from: lowest level staged in LDS (None = none).  Returns a dict."""
    sk = np.asarray(sorted_keys, dtype=np.uint64)
    q = np.asarray(queries_sorted, dtype=np.uint64)
    if h is None:
        h = heights(sk, seed, log2_inv_p, max_height)
    levels = build_levels(sk, h)
    top = max(levels) if levels else 1
    nq = q.size
    index_lines = 0
    lds_bytes = 0
    start = np.zeros(nq, dtype=np.int64)  # position (head = 0) at the level above
    start_key_level = None
    for l in range(top, 1, -1):
        lk = levels[l]
        if start_key_level is not None:
            # position on this level of the key found one level up
            start = np.where(start_found, np.searchsorted(lk, start_key, side="right"), 0)
        pos = np.searchsorted(lk, q, side="right")  # keys <= q, i.e. 1-based position, head = 0
        if lds_from is not None and l >= lds_from:
            lds_bytes += (lk.size + 1 + level_pad) * (KEY_BYTES + DOWN_BYTES)
        else:
            # keys read: entries start+1 .. pos+1 ; down read: entry pos
            kf = (start + 1) // KEYS_PER_LINE
            kl = (pos + 1) // KEYS_PER_LINE
            index_lines += _distinct_lines(kf, kl)
            index_lines += np.unique(pos // DOWNS_PER_LINE).size
        start_found = pos > 0
        start_key = np.where(start_found, lk[np.maximum(pos - 1, 0)], np.uint64(0))
        start_key_level = l
    # storage: interception slot (1-based, head 0) -> last key <= q
    if levels:
        l2 = levels[2]
        ipos = np.searchsorted(l2, q, side="right")
        islot = np.where(ipos > 0, np.searchsorted(sk, l2[np.maximum(ipos - 1, 0)], side="left") + 1, 0)
    else:
        islot = np.zeros(nq, dtype=np.int64)
    tslot = np.searchsorted(sk, q, side="right")  # slot of the last key <= q (0 = head)
    storage_lines = _distinct_lines((islot + 1) // KEYS_PER_LINE, (tslot + 1) // KEYS_PER_LINE)
    hit = (tslot > 0) & (sk[np.maximum(tslot - 1, 0)] == q) if sk.size else np.zeros(nq, dtype=bool)
    value_lines = np.unique(tslot[hit] // (LINE // VAL_BYTES)).size if with_values else 0
    io = nq * (8 + 4) + nq * (8 + 1)
    total = (index_lines + storage_lines + value_lines) * LINE + lds_bytes + io
    return {"bytes": int(total), "per_query": total / max(nq, 1), "index_lines": int(index_lines),
            "storage_key_lines": int(storage_lines), "value_lines": int(value_lines),
            "lds_bytes": int(lds_bytes), "io_bytes": int(io), "queries": int(nq), "top": int(top)}


# Reference bytes per query of the parts of a batch outside the descent: the
# ordering step as a two-pass key-range partition that reads each query's key
# and op twice (2 x 9 B), writes the ordered key, position and op (13 B) which
# the descent reads back (13 B), and the answers written in arrival order
# (value and status, 9 B).
PARTITION_BYTES_PER_QUERY = 2 * (8 + 1) + (8 + 4 + 1) + (8 + 4 + 1)
ANSWER_BYTES_PER_QUERY = 8 + 1


def batch_bytes(descent, n_queries):
    """Algorithmic bytes of one whole batch (ordering, descent, answers) from
    a ``descent_bytes`` result: its index, storage and value lines (and the
    LDS-staged levels), plus the reference ordering and answer bytes in place
    of the descent's own input and output terms."""
    return int(descent["bytes"] - descent["io_bytes"] +
               n_queries * (PARTITION_BYTES_PER_QUERY + ANSWER_BYTES_PER_QUERY))
