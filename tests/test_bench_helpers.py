"""CPU tests of the benchmark's pure helpers: the row ranges of the polar-trimmed dense GEMM
comparison.  No GPU."""
import numpy as np
import torch

import bench
import oracle


def test_polar_rows_is_the_last_node_above_the_threshold():
    # Q stored transposed per pair (n x l, nodes last); chunks smaller than the pair count
    l = 16
    Q = torch.zeros((5, l, l), dtype=torch.float64)
    Q[0, 0, 3] = 1.0                       # last significant node 3 -> 4 rows
    Q[1, 2, 15] = 2 * bench.POLAR_TRIM     # the last node counts
    Q[2, 1, 7] = bench.POLAR_TRIM          # not above the threshold -> 0 rows
    Q[3, 0, :] = 1.0
    Q[3, 0, 10:] = 0.0                     # -> 10 rows
    assert bench.polar_rows(Q, chunk=2) == [4, 16, 0, 10, 0]


def test_polar_rows_on_legendre_matrices():
    # against the oracle's dense Q^(m,p): every node past the count is negligible, the last
    # one inside is not, and high orders leave out nodes towards the pole
    l = 32
    pairs = [(m, p) for m in range(0, 2 * l, 7) for p in (0, 1)]
    Q = torch.zeros((len(pairs), l, l), dtype=torch.float64)
    for i, (m, p) in enumerate(pairs):
        q = oracle.dense_q(l, m, p)
        Q[i, :q.shape[1], :] = torch.from_numpy(q.T)
    rows = bench.polar_rows(Q, chunk=5)
    for i, (m, p) in enumerate(pairs):
        q = oracle.dense_q(l, m, p)
        if q.shape[1] == 0:
            assert rows[i] == 0
            continue
        r = rows[i]
        assert np.abs(q[r:]).max(initial=0.0) <= bench.POLAR_TRIM
        assert np.abs(q[r - 1]).max() > bench.POLAR_TRIM
    assert rows[0] == l and rows[-2] < l


def test_gemm_runs_pad_to_the_run_maximum():
    ncols = [5, 4, 0, 0, 3, 1, 0]
    rows = [8, 6, 0, 0, 2, 7, 0]
    assert bench.gemm_runs(ncols, rows, run=2) == [(0, 2, 5, 8), (4, 6, 3, 7)]
    assert bench.gemm_runs(ncols, [0] * 7, run=3) == []
