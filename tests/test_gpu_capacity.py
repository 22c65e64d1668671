"""GPU tests of the storage capacity: the host's bound on the slots in use
stays an upper bound whatever mix of paths enqueued the batches, a fixed
capacity is enforced before anything is enqueued, and a wrong host bound can
never make a kernel write past the capacity.  Answers against the CPU oracle,
bit-exact."""
import numpy as np
import pytest
import torch

from oracle.skiplist import SkipList
from paper_1601_00159_amd._lib import PI_ERR_CAPACITY, PI_ERR_DEVICE, PiError
from paper_1601_00159_amd.index import Group, Index, to_device_u64, to_device_u8, to_numpy_u64

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.node.name}", flush=True)


def export_np(ix):
    k, v = ix.export()
    return to_numpy_u64(k), to_numpy_u64(v)


def fresh_keys(rng, n, avoid):
    k = np.unique(rng.integers(0, 1 << 63, size=2 * n + 16, dtype=np.uint64))
    k = k[~np.isin(k, avoid)]
    return rng.permutation(k)[:n]


def check_answers(got_v, got_s, want_v, want_s, what):
    got_v, got_s = np.asarray(got_v, dtype=np.uint64), np.asarray(got_s, dtype=np.uint8)
    assert np.array_equal(got_s, np.asarray(want_s, dtype=np.uint8)), what
    assert np.array_equal(got_v, np.asarray(want_v, dtype=np.uint64)), what


def batch_on_device(ops, keys, vals, dev):
    n = ops.size
    return (to_device_u8(ops, dev), to_device_u64(keys, dev), to_device_u64(vals, dev),
            torch.empty(n, dtype=torch.int64, device=dev), torch.empty(n, dtype=torch.uint8, device=dev))


@pytest.mark.parametrize("policy", ["never", "threshold"])
def test_group_and_single_calls_share_the_capacity_bound(policy):
    """A fixed-capacity index used alternately through the many-index call
    and the single-index call: every call that fits is answered as the oracle
    answers it, the first call that does not fit is refused with
    PI_ERR_CAPACITY and leaves the index unchanged, and the storage bound the
    host keeps after a group call covers the single calls made in between
    (a stale bound once let a later group call append past the capacity)."""
    rng = np.random.default_rng({"never": 61, "threshold": 62}[policy])
    dev = torch.device("cuda", 0)
    lk = np.unique(rng.integers(0, 1 << 63, size=1000, dtype=np.uint64))[:1000]
    lv = rng.integers(0, 1 << 64, size=lk.size, dtype=np.uint64, endpoint=False)
    orc = SkipList()
    orc.bulk_load(lk, lv)
    used = set(lk.tolist())

    def inserts(n, n_search=0):
        k = fresh_keys(rng, n, np.array(sorted(used), dtype=np.uint64))
        used.update(k.tolist())
        ops = np.ones(n, dtype=np.uint8)
        keys = k
        if n_search:
            ops = np.concatenate([ops, np.zeros(n_search, dtype=np.uint8)])
            keys = np.concatenate([keys, lk[rng.integers(0, lk.size, n_search)]])
            p = rng.permutation(ops.size)
            ops, keys = ops[p], keys[p]
        vals = rng.integers(0, 1 << 64, size=ops.size, dtype=np.uint64, endpoint=False)
        return ops, keys, vals

    with Index(capacity_hint=1500, rebuild_policy=policy, rebuild_min=1 << 40) as ix, Group() as g:
        ix.bulk_load(lk, lv)                       # slots in use: 1002 of 1500

        def group_call(ops, keys, vals):
            b = batch_on_device(ops, keys, vals, dev)
            g.execute([ix], [b])
            torch.cuda.synchronize()
            return to_numpy_u64(b[3]), b[4].cpu().numpy()

        def single_call(ops, keys, vals):
            ov, os_ = ix.execute(ops, keys, vals)
            torch.cuda.synchronize()
            return to_numpy_u64(ov), os_.cpu().numpy()

        def accepted(call, b, what):
            got = call(*b)
            check_answers(*got, *orc.execute_batch(*b), what)

        def refused(call, b, what):
            before = export_np(ix)
            with pytest.raises(PiError) as e:
                call(*b)
            assert e.value.status == PI_ERR_CAPACITY, what
            after = export_np(ix)
            assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1]), what

        accepted(group_call, inserts(300), "group 300")        # 1302
        accepted(single_call, inserts(150), "single 150")      # 1452
        refused(group_call, inserts(100), "group 100")         # 1552 > 1500
        accepted(single_call, inserts(40, 1960), "single 40 of 2000 (multi-kernel path)")  # 1492
        accepted(group_call, inserts(8), "group 8")            # 1500: full
        refused(single_call, inserts(1), "single 1")
        refused(group_call, inserts(1), "group 1")
        s = np.zeros(5, dtype=np.uint8)
        accepted(single_call, (s, lk[:5], lk[:5]), "searches on a full index")
        ek, ev = export_np(ix)
        ok, ov = orc.export()
        assert np.array_equal(ek, ok) and np.array_equal(ev, ov)
        assert ix.stats()["overflow_nodes"] == 498


@pytest.mark.parametrize("small_log2", [10, 255])
def test_a_wrong_bound_never_writes_past_the_capacity(small_log2):
    """With the host's bound planted far below the truth, a batch whose 600
    new nodes do not fit the 100 free slots passes the host check; the
    kernels (the one-workgroup path, and with small batches off the
    multi-kernel path) then write no new node past the capacity, and the next
    counter read fails the handle with a capacity error instead of corrupting
    memory."""
    rng = np.random.default_rng(70 + small_log2)
    n = 600
    lk = np.unique(rng.integers(0, 1 << 63, size=3000, dtype=np.uint64))
    cap = lk.size + 2 + 100
    with Index(capacity_hint=cap, rebuild_policy="never", small_batch_log2=small_log2) as ix:
        ix.bulk_load(lk, lk)
        ops = np.ones(n, dtype=np.uint8)
        keys = fresh_keys(rng, n, lk)
        ix.set_storage_bound(0)
        ix.execute(ops, keys, keys)                 # accepted: the planted bound says there is room
        torch.cuda.synchronize()
        with pytest.raises(PiError) as e:
            ix.stats()
        assert e.value.status == PI_ERR_DEVICE
        assert "capacity" in str(e.value)
        with pytest.raises(PiError) as e:           # the handle stays failed
            ix.execute(ops[:1], keys[:1], keys[:1])
        assert e.value.status == PI_ERR_DEVICE


def test_serving_capacity_checked_before_the_first_micro_batch():
    """pi_serve on a fixed-capacity index whose stream inserts more keys than
    fit: refused with PI_ERR_CAPACITY before any micro-batch, the index
    unchanged; a stream that fits is served with the oracle's answers."""
    rng = np.random.default_rng(81)
    lk = np.unique(rng.integers(0, 1 << 63, size=2000, dtype=np.uint64))
    orc = SkipList()
    orc.bulk_load(lk, lk)
    with Index(capacity_hint=lk.size + 2 + 200, rebuild_policy="never") as ix:
        ix.bulk_load(lk, lk)
        n = 5000
        ops = np.zeros(n, dtype=np.uint8)
        keys = lk[rng.integers(0, lk.size, n)]
        ins = rng.choice(n, 300, replace=False)
        ops[ins] = 1
        keys[ins] = fresh_keys(rng, 300, lk)
        vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
        arrival = np.sort(rng.random(n)) * 200.0
        before = export_np(ix)
        with pytest.raises(PiError) as e:
            ix.serve(arrival, ops, keys, vals, deadline_us=20.0, max_batch=500)
        assert e.value.status == PI_ERR_CAPACITY
        after = export_np(ix)
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        ops[ins[200:]] = 0                          # 200 inserts: they fit exactly
        gv, gs, done, ends = ix.serve(arrival, ops, keys, vals, deadline_us=20.0, max_batch=500)
        torch.cuda.synchronize()
        check_answers(to_numpy_u64(gv), gs.cpu().numpy(), *orc.execute_batch(ops, keys, vals), "served")
        assert ends[-1] == n
        ek, ev = export_np(ix)
        ok, ov = orc.export()
        assert np.array_equal(ek, ok) and np.array_equal(ev, ov)
