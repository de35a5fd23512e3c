"""The benchmark's CPU-baseline leg (CPU only): the oracle split over threads
must compute exactly what the sequential oracle computes."""
import concurrent.futures

import numpy as np

import bench
import oracle
from paper_2507_15121_amd import synth


def _problem():
    dims = (3000, 1200, 500)
    st = synth.tensor(dims, 40_000, "zipf", 1.1, 0.05, seed=21)
    factors64 = [f.astype(np.float64) for f in synth.factors(dims, 8, seed=21)]
    return st, factors64


def test_row_blocks_reassemble_the_full_output_bit_for_bit():
    st, f64 = _problem()
    for d in range(3):
        full = oracle.mttkrp(st.idx, st.val.astype(np.float64), st.dims, f64, d)
        for parts in (1, 3, 8, 64):
            bounds, jobs = bench.row_block_jobs(st.idx, st.val.astype(np.float64), st.dims, f64, d, parts)
            assert bounds[0] == 0 and bounds[-1] == st.dims[d] and np.all(np.diff(bounds) > 0)
            assert len(jobs) == bounds.size - 1 <= parts
            assert sum(j[1].size for j in jobs) == st.nnz
            got = np.vstack([oracle.mttkrp(*j) for j in jobs])
            # every row's nonzeros stay in one block, in input order: the same fp64 sums
            np.testing.assert_array_equal(got, full)


def test_row_blocks_balance_nonzeros():
    st, f64 = _problem()
    _, jobs = bench.row_block_jobs(st.idx, st.val.astype(np.float64), st.dims, f64, 1, 8)
    sizes = np.array([j[1].size for j in jobs])
    heaviest = np.bincount(st.idx[1]).max()
    # a block exceeds the even share by at most the one row it cannot split
    assert sizes.max() <= st.nnz / 8 + heaviest


def test_empty_sample_gives_equal_row_ranges():
    st, f64 = _problem()
    empty = np.zeros((3, 0), np.int32)
    bounds, jobs = bench.row_block_jobs(empty, np.zeros(0), st.dims, f64, 0, 7)
    assert len(jobs) == 7 and bounds[-1] == st.dims[0]
    got = np.vstack([oracle.mttkrp(*j) for j in jobs])
    assert got.shape == (st.dims[0], 8) and not got.any()


def test_position_split_oracle_rows_match_the_sequential_oracle():
    st, f64 = _problem()
    rows = np.array([0, 5, int(np.argmax(np.bincount(st.idx[0]))), 2999])
    rows = np.unique(rows)
    with concurrent.futures.ThreadPoolExecutor(4) as pool:
        got = bench.oracle_rows(st, f64, 0, rows, 8, pool, 5)
    ref = oracle.mttkrp(st.idx, st.val.astype(np.float64), st.dims, f64, 0)[rows]
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_cpu_baseline_times_a_bounded_sample():
    st, f64 = _problem()
    with concurrent.futures.ThreadPoolExecutor(2) as pool:
        S, t, t_zero = bench.cpu_baseline(st, f64, pool, 2, 0.05)
    assert 0 < S <= st.nnz and t > 0 and t_zero >= 0
