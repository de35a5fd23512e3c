"""The seeded input generator: determinism, exact counts, distinctness, order,
hot-slice share and the Zipf law it samples."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2507_15121_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lin(idx, dims):
    lin = np.zeros(idx.shape[1], dtype=np.int64)
    for w, d in enumerate(dims):
        lin = lin * int(d) + idx[w].astype(np.int64)
    return lin


@pytest.mark.parametrize("dist,hot", [("uniform", 0.0), ("zipf", 0.0), ("zipf", 0.05)])
def test_counts_distinct_sorted_in_range(dist, hot):
    dims = (3000, 2000, 700)
    nnz = 200_000
    idx, info = synth.coords(dims, nnz, dist, 1.1, hot, seed=5)
    assert idx.shape == (3, nnz) and idx.dtype == np.int32
    for w, d in enumerate(dims):
        assert idx[w].min() >= 0 and idx[w].max() < d
    lin = _lin(idx, dims)
    assert np.all(np.diff(lin) > 0)  # strictly increasing: sorted and distinct
    if hot:
        h = info["hot_index"]
        assert info["hot_nnz"] == round(hot * nnz)
        assert int((idx[0] == h).sum()) == info["hot_nnz"]
        assert h == synth.rank_perm(0, dims[0], seed=5)[dims[0] // 2]


def test_order4_and_order2():
    idx, _ = synth.coords((50, 40, 30, 20), 10_000, "zipf", 1.2, seed=3)
    assert np.all(np.diff(_lin(idx, (50, 40, 30, 20))) > 0)
    idx, _ = synth.coords((100, 90), 2_000, "uniform", seed=3)
    assert np.all(np.diff(_lin(idx, (100, 90))) > 0)


def test_seed_determinism_and_sensitivity():
    a, _ = synth.coords((500, 400, 300), 20_000, "zipf", 1.1, seed=1)
    b, _ = synth.coords((500, 400, 300), 20_000, "zipf", 1.1, seed=1)
    c, _ = synth.coords((500, 400, 300), 20_000, "zipf", 1.1, seed=2)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    np.testing.assert_array_equal(synth.values(1000, seed=1), synth.values(1000, seed=1))


def test_independent_of_thread_count():
    code = ("import hashlib,sys; sys.path.insert(0,%r); from paper_2507_15121_amd import synth; "
            "i,_=synth.coords((30000,20000,5000),300000,'zipf',1.1,0.05,seed=9); "
            "v=synth.factor(1,777,8,seed=9); "
            "print(hashlib.md5(i.tobytes()+v.tobytes()).hexdigest())" % ROOT)
    outs = set()
    for nt in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           check=True)
        outs.add(r.stdout.strip())
    assert len(outs) == 1


def test_rank_perm_is_bijection():
    for I in (1, 2, 3, 17, 1000, 65537):
        p = synth.rank_perm(0, I, seed=4)
        assert np.array_equal(np.sort(p), np.arange(I))
    p1 = synth.rank_perm(0, 1000, seed=4)
    p2 = synth.rank_perm(1, 1000, seed=4)
    assert not np.array_equal(p1, p2)


def test_zipf_sampler_head_frequencies_chi2():
    # P(rank k) = k^-s / H_{I,s}; chi-square over the 20 most likely ranks plus
    # the tail bucket.
    from scipy import stats
    I, s, n = 100_000, 1.1, 2_000_000
    r = synth.zipf_ranks(I, s, n, seed=12)
    assert r.min() >= 0 and r.max() < I
    w = np.arange(1, I + 1, dtype=np.float64) ** -s
    p = w / w.sum()
    head = 20
    obs = np.bincount(r, minlength=I)
    o = np.concatenate([obs[:head], [obs[head:].sum()]])
    e = np.concatenate([p[:head], [p[head:].sum()]]) * n
    chi2 = ((o - e) ** 2 / e).sum()
    assert chi2 < stats.chi2.ppf(0.9999, head)


def test_uniform_values_and_factors_ranges():
    v = synth.values(100_000, seed=2)
    assert v.dtype == np.float32 and v.min() >= 0.0 and v.max() < 1.0
    assert abs(v.mean() - 0.5) < 0.01
    f = synth.factor(0, 1000, 32, seed=2)
    assert f.shape == (1000, 32) and f.min() >= -1.0 and f.max() < 1.0
    assert abs(f.mean()) < 0.01
    # distinct modes use distinct streams
    assert not np.array_equal(synth.factor(0, 10, 4, seed=2), synth.factor(1, 10, 4, seed=2))


def test_uniform_small_workload_matches_recipe():
    t = synth.workload("uniform3-1000x800x600-100k")
    assert t.nnz == 100_000 and t.dims == (1000, 800, 600)
    st = synth.slice_stats(t.idx, t.dims)
    # 100 nonzeros per mode-0 slice on average, every slice touched
    assert st[0]["distinct"] == 1000
