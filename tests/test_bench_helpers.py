"""CPU tests of the benchmark's pure helpers: the row ranges of the polar-trimmed dense GEMM
comparison, the roofline object of the JSON line and the per-step stage totals.  No GPU."""
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


def test_roofline_picks_the_largest_launch_and_its_bound():
    prof = {
        "synth.fft/F64/split32": {"ms": 40.0, "launches": 20, "flops": 1e9, "bytes": 8e9},
        "analysis.final/F64/split32": {"ms": 250.0, "launches": 20, "flops": 1.2e11, "bytes": 1.5e10},
        "synth.level2.c0/F64/split32": {"ms": 100.0, "launches": 20, "flops": 4e11, "bytes": 1e10},
    }
    r = bench.roofline(prof, precision="split32", l=1024, F=64)
    mean_s = 250.0 / 20 / 1e3
    # a Legendre launch at 64 fields is a dense contraction: matrix-core bound, FP64-equivalent
    # flops against the FP32 MFMA peak the split form runs on, its four products per
    # FP64-equivalent product given beside it
    assert r["kernel"] == "analysis.final/F64/split32" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["peak"] == 157.3 and abs(r["achieved"] - 1.2e11 / mean_s / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12 and r["mean_launch_ms"] == 12.5
    assert abs(r["executed_frac"] - 4 * r["frac"]) < 1e-12
    assert r["nonalgorithmic_bytes_per_launch"] == 1.5e10
    r = bench.roofline(prof, precision="fp64", l=1024, F=64)
    assert r["bound"] == "mfma" and r["peak"] == 78.6 and abs(r["executed_frac"] - r["frac"]) < 1e-15
    # an FFT launch that dominates is bound by HBM on the grid bytes it reads or writes once
    prof["synth.fft/F64/split32"]["ms"] = 400.0
    r = bench.roofline(prof, precision="split32", l=1024, F=64)
    gb = 64 * 2048 * 4096 * 16
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["achieved"] - gb / 0.02 / 1e9) < 1e-6 and r["nonalgorithmic_bytes_per_launch"] == 8e9 - gb


def test_roofline_of_a_factor_streaming_launch_is_hbm_bound():
    # one complex field (R = 4): 2 x 4 flops per 8-byte factor word, below the FP64 ridge point
    # (78.6 TFLOP/s over 8 TB/s): bound by HBM on the launch's algorithmic bytes
    prof = {"analysis.final/F1/fp64": {"ms": 2.0, "launches": 10, "flops": 1e8, "bytes": 1.2e8},
            "synth.level1/F1/fp64": {"ms": 1.0, "launches": 10, "flops": 1e8, "bytes": 1.1e8}}
    r = bench.roofline(prof, precision="fp64", l=256, F=1)
    assert r["kernel"] == "analysis.final/F1/fp64" and r["bound"] == "hbm" and r["peak"] == 8000.0
    assert abs(r["achieved"] - 1.2e8 / 2e-4 / 1e9) < 1e-9 and abs(r["frac"] - r["achieved"] / 8000.0) < 1e-15
    # the same launch at 64 columns per factor word is a contraction again
    assert bench.roofline(prof, precision="fp64", l=256, F=1, R=64)["bound"] == "mfma"


def test_step_roofline_sums_every_launch():
    prof = {"a": {"ms": 10.0, "launches": 4, "flops": 2e11, "bytes": 1e9},
            "b": {"ms": 30.0, "launches": 2, "flops": 5e11, "bytes": 3e9}}
    r = bench.step_roofline(prof, steps=2, ms_step=20.0, precision="split32", l=1024, F=64, fac_entries=1e9)
    flops = (4 * 2e11 + 2 * 5e11) / 2
    assert abs(r["flops_per_step"] - flops) < 1 and abs(r["mfma_frac"] - flops / 0.02 / 157.3e12) < 1e-12
    assert abs(r["executed_mfma_frac"] - 4 * r["mfma_frac"]) < 1e-12
    algo = 2 * 1e9 * 8 + 2 * 64 * 4 * 1024 ** 2 * 16 + 2 * 64 * 2048 * 4096 * 16
    assert abs(r["algorithmic_bytes_per_step"] - algo) < 1 and r["layout_bytes_per_step"] == (4e9 + 6e9) / 2


def test_stage_totals_merge_size_classes():
    prof = {"synth.level2.c0/F64/fp64": {"ms": 30.0}, "synth.level2.c1/F64/fp64": {"ms": 10.0},
            "synth.fft/F64/fp64": {"ms": 20.0}}
    assert bench.stage_totals(prof, steps=10) == {"synth.fft/F64/fp64": 2.0, "synth.level2/F64/fp64": 4.0}
