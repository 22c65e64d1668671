"""The seeded generators: determinism, shapes, op mixes, Zipf frequencies."""
import numpy as np

from paper_1601_00159_amd import workloads as W


def test_deterministic_and_unique():
    a = W.plain_pi(scale=12)
    b = W.plain_pi(scale=12)
    assert np.array_equal(a.load_keys, b.load_keys)
    assert np.array_equal(a.batches[0].keys, b.batches[0].keys)
    assert np.unique(a.load_keys).size == a.load_keys.size == 4096
    assert a.load_keys.max() < (1 << 63)
    assert not np.all(np.diff(a.load_keys.astype(np.float64)) > 0)  # shuffled, not sorted


def test_plain_mix_fractions():
    w = W.plain_pi(scale=16)
    ops = w.batches[0].ops
    n = ops.size
    for op, p in ((0, 0.8), (1, 0.1), (2, 0.1)):
        frac = (ops == op).mean()
        assert abs(frac - p) < 6 * np.sqrt(p * (1 - p) / n)
    loaded = np.isin(w.batches[0].keys, w.load_keys).mean()
    assert abs(loaded - 0.5) < 0.02


def test_zipf_pmf_chi_square():
    z = W.Zipf(1000, 0.99)
    rng = W.rng_for(1, 2, 3)
    r = z.sample(200_000, rng)
    assert r.min() >= 0 and r.max() < 1000
    obs = np.bincount(r, minlength=1000)[:50].astype(np.float64)
    exp = z.pmf(np.arange(50)) * r.size
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 49 dof: p ~ 1e-7 cut-off
    # P(r) proportional to (r+1)^-theta
    p = z.pmf(np.arange(3))
    assert abs(p[0] / p[1] - 2 ** 0.99) < 1e-9


def test_write_heavy_shapes():
    w = W.write_heavy(3, 1 << 12, 1 << 14, 2)
    b = w.batches[0]
    ins = b.ops == W.INSERT
    assert abs(ins.mean() - 0.5) < 0.03
    # non-insert keys come from the loaded set
    assert np.isin(b.keys[~ins], w.load_keys).all()
