"""Query hand-over between neighbouring workers (paper Algorithm 3, Section
3.2.2) and the latch-free invariant (Section 3.2.4) -- TEST INFRASTRUCTURE ONLY.

Input: the key-sorted query set (Definition 3) with one interception per
query (Definition 4; ``None`` stands for the head of the list).  The sorted
set is first cut into ``n_workers`` consecutive slices of equal size (the
partition step of Algorithm 1; when the size is not divisible the first
``n % n_workers`` slices get one extra query -- the paper leaves this open).

Hand-over, in worker order (the paper notes the adjustment must run in the
order of worker id, Section 3.2.5):
  every worker learns the interception of the FIRST query of the next
  non-empty worker's original slice;
  worker i prepends the queries handed to it by worker i-1, then walks its
  slice backwards and hands every trailing query whose interception equals
  that key to worker i+1, stopping at the first one that differs.

Output: the owning worker of every sorted query.
"""

_HEAD = object()


def _icpt_key(x):
    return _HEAD if x is None else x


def even_partition(n: int, n_workers: int):
    """Slice bounds [(lo, hi)] of the partition step."""
    base, extra = divmod(n, n_workers)
    bounds, lo = [], 0
    for w in range(n_workers):
        hi = lo + base + (1 if w < extra else 0)
        bounds.append((lo, hi))
        lo = hi
    return bounds


def redistribute(interceptions, n_workers: int):
    """Owner worker of each sorted query after the hand-over.

    ``interceptions`` lists, in sorted-query order, the interception key of
    each query (None for the head)."""
    icpt = [_icpt_key(x) for x in interceptions]
    n = len(icpt)
    bounds = even_partition(n, n_workers)
    # first interception of each worker's ORIGINAL slice (exchanged first)
    first = [icpt[lo] if hi > lo else None for lo, hi in bounds]
    slices = [list(range(lo, hi)) for lo, hi in bounds]
    owner = [None] * n
    carried = []
    for w in range(n_workers):
        batch = carried + slices[w]
        # key of the next non-empty worker's first interception
        nxt = None
        for v in range(w + 1, n_workers):
            if bounds[v][1] > bounds[v][0]:
                nxt = first[v]
                break
        carried = []
        if nxt is not None:
            while batch and icpt[batch[-1]] == nxt:
                carried.insert(0, batch.pop())
        for q in batch:
            owner[q] = w
    # the last worker keeps whatever is left over
    for q in carried:
        owner[q] = n_workers - 1
    return owner


def check_latch_free(interceptions, owner):
    """True when no interception is shared by two workers and the owners are
    non-decreasing along the sorted query set, i.e. every worker's queries lie
    between its own first interception and the next worker's (Section 3.2.4)."""
    icpt = [_icpt_key(x) for x in interceptions]
    seen = {}
    for i, (c, w) in enumerate(zip(icpt, owner)):
        if i and owner[i] < owner[i - 1]:
            return False
        key = ("head",) if c is _HEAD else ("k", c)
        if key in seen and seen[key] != w:
            return False
        seen[key] = w
    return True
