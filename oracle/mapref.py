"""Plain map replay of a query batch -- TEST INFRASTRUCTURE ONLY.

The batched index must give exactly the answers of a serial execution of the
batch in arrival order (paper Section 4.2: one thread owns each data node, so
the parallel result is serializable; Section 3.2.4).  This module writes that
serial execution out directly as a dictionary replay:

  SEARCH k   -> (PRESENT, m[k]) if k in m else (ABSENT, 0)
  INSERT k v -> same answer, then m[k] = v
  DELETE k   -> same answer, then k is removed
  op not in {0,1,2} or k == 2**64-1 -> (INVALID, 0), no effect

``replay_dict`` is the definition on a Python dict.  ``MapState`` keeps the
map as sorted numpy arrays so that large indices (tens of millions of keys)
stay cheap; a batch is still replayed query by query in arrival order, but only
over the keys the batch touches (all other keys are unaffected by definition).
"""
import numpy as np

SEARCH, INSERT, DELETE = 0, 1, 2
ABSENT, PRESENT, INVALID = 0, 1, 255
KEY_MAX = (1 << 64) - 1


def replay_dict(m: dict, ops, keys, vals):
    """Apply a batch to dict ``m`` in place, in arrival order.

    Returns (out_vals, out_status) as Python lists."""
    out_v, out_s = [], []
    for op, k, v in zip(ops, keys, vals):
        op, k, v = int(op), int(k), int(v)
        if op > DELETE or k == KEY_MAX:
            out_v.append(0)
            out_s.append(INVALID)
            continue
        if k in m:
            out_v.append(m[k])
            out_s.append(PRESENT)
        else:
            out_v.append(0)
            out_s.append(ABSENT)
        if op == INSERT:
            m[k] = v
        elif op == DELETE:
            m.pop(k, None)
    return out_v, out_s


def dedupe_last(keys, vals):
    """Sorted unique keys with the value of each key's LAST occurrence
    (bulk load = inserting the pairs in array order)."""
    keys = np.asarray(keys, dtype=np.uint64)
    vals = np.asarray(vals, dtype=np.uint64)
    rk = keys[::-1]
    rv = vals[::-1]
    uk, first_in_reversed = np.unique(rk, return_index=True)
    uv = rv[first_in_reversed]
    keep = uk != np.uint64(KEY_MAX)
    return uk[keep], uv[keep]


class MapState:
    """The index as a map held in two sorted numpy arrays."""

    def __init__(self, keys=None, vals=None):
        if keys is None:
            self.keys = np.zeros(0, dtype=np.uint64)
            self.vals = np.zeros(0, dtype=np.uint64)
        else:
            self.keys, self.vals = dedupe_last(keys, vals)

    def __len__(self):
        return int(self.keys.size)

    def lookup(self, q):
        """Vectorised SEARCH: (status u8[], value u64[]) for keys q."""
        q = np.asarray(q, dtype=np.uint64)
        pos = np.searchsorted(self.keys, q, side="left")
        posc = np.minimum(pos, max(self.keys.size - 1, 0))
        if self.keys.size:
            hit = (pos < self.keys.size) & (self.keys[posc] == q)
        else:
            hit = np.zeros(q.shape, dtype=bool)
        st = np.where(hit, PRESENT, ABSENT).astype(np.uint8)
        val = np.where(hit, self.vals[posc] if self.keys.size else 0, 0).astype(np.uint64)
        return st, val

    def apply_batch(self, ops, keys, vals):
        """Serial replay of one batch; mutates the state.

        Returns (out_vals u64[], out_status u8[]) in arrival order."""
        ops = np.asarray(ops, dtype=np.uint8)
        keys = np.asarray(keys, dtype=np.uint64)
        vals = np.asarray(vals, dtype=np.uint64)
        n = ops.size
        valid = (ops <= DELETE) & (keys != np.uint64(KEY_MAX))
        touched = np.unique(keys[valid])
        st0, v0 = self.lookup(touched)
        # the part of the map the batch can see, as a dict
        m = {int(k): int(v) for k, v, s in zip(touched.tolist(), v0.tolist(), st0.tolist()) if s == PRESENT}
        out_v, out_s = replay_dict(m, ops.tolist(), keys.tolist(), vals.tolist())
        # write back: drop every touched key, then add the survivors
        keep = ~np.isin(self.keys, touched, assume_unique=True)
        ks = self.keys[keep]
        vs = self.vals[keep]
        if m:
            nk = np.fromiter(m.keys(), dtype=np.uint64, count=len(m))
            nv = np.fromiter(m.values(), dtype=np.uint64, count=len(m))
            ks = np.concatenate([ks, nk])
            vs = np.concatenate([vs, nv])
            order = np.argsort(ks, kind="stable")
            ks, vs = ks[order], vs[order]
        self.keys, self.vals = ks, vs
        return (np.asarray(out_v, dtype=np.uint64).reshape(n),
                np.asarray(out_s, dtype=np.uint8).reshape(n))

    def search_batch(self, keys):
        """Answers of an all-SEARCH batch (no state change)."""
        keys = np.asarray(keys, dtype=np.uint64)
        st, val = self.lookup(keys)
        inval = keys == np.uint64(KEY_MAX)
        st = np.where(inval, INVALID, st).astype(np.uint8)
        val = np.where(inval, 0, val).astype(np.uint64)
        return val, st

    def range_batch(self, lo, hi):
        """Range searches on the sorted arrays (the plain definition: every key
        k with lo <= k <= hi): (counts, keys, values), concatenated in range
        order."""
        lo = np.asarray(lo, dtype=np.uint64)
        hi = np.asarray(hi, dtype=np.uint64)
        a = np.searchsorted(self.keys, lo, side="left")
        b = np.searchsorted(self.keys, hi, side="right")
        b = np.where(lo <= hi, np.maximum(a, b), a)
        counts = (b - a).astype(np.uint64)
        idx = np.concatenate([np.arange(x, y) for x, y in zip(a.tolist(), b.tolist())] or
                             [np.zeros(0, dtype=np.int64)]).astype(np.int64)
        return counts, self.keys[idx], self.vals[idx]
