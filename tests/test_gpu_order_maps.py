"""GPU parity of the per-order maps of Section 5 (equations (transform) and (transform2) on the
nodes of Lemma distinct_theorem with the weights of Lemma quadratures), applied by the
butterfly kernels through sht_order_apply, against the oracle's dense matrices
(oracle.gauss_jacobi.matrix, built on the step-one recurrence and numpy's eigensolver).

Error metric: relative l2 per (pair, direction) over the pair's R columns; FP64 gate 1e-11.
"""
import ctypes

import numpy as np
import pytest

from oracle import gauss_jacobi as gj

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _check_pairs(plan, l, R, pairs, seed=0, label=""):
    """Forward and inverse map of random vectors, pair by pair against the oracle."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((plan.rows, R))
    y = plan.apply(_dev(x)).cpu().numpy()
    z = plan.apply(_dev(y), transpose=True).cpu().numpy()
    worst_f = worst_t = worst_rt = 0.0
    for m, p in pairs:
        r0, n = plan.layout(m, p)
        assert n == len(range(m + p, 2 * l, 2))
        if n == 0:
            continue
        A = gj.matrix(m, n, p)
        xs, ys, zs = x[r0:r0 + n], y[r0:r0 + n], z[r0:r0 + n]
        ef = np.linalg.norm(ys - A @ xs) / np.linalg.norm(A @ xs)
        et = np.linalg.norm(zs - A.T @ ys) / np.linalg.norm(A.T @ ys)
        er = np.linalg.norm(zs - xs) / np.linalg.norm(xs)
        assert ef < FP64_TOL and et < FP64_TOL and er < FP64_TOL, (m, p, n, ef, et, er)
        worst_f, worst_t, worst_rt = max(worst_f, ef), max(worst_t, et), max(worst_rt, er)
    print(f"{label} R={R}: forward {worst_f:.2e}, transposed {worst_t:.2e}, round trip {worst_rt:.2e} "
          f"over {len(pairs)} pairs (gate {FP64_TOL:g})", flush=True)
    return x, y, z


def _all_pairs(l):
    return [(m, p) for m in range(2 * l) for p in (0, 1)]


@pytest.mark.parametrize("R", [1, 3, 16, 48])
def test_every_pair_l32(R):
    # leaf width 8: up to two levels above the leaves; R = 1, 3 run the vector kernels, R = 16, 48
    # the FP64 matrix-core level kernels (48: three column tiles)
    from paper_0910_5435_amd import OrderPlan

    plan = OrderPlan(32, eps=1e-13, leaf_width=8)
    assert plan.rows == 32 * 65  # sum over m < 64 of (64 - m)
    _check_pairs(plan, 32, R, _all_pairs(32), seed=R, label="l=32 C=8")


@pytest.mark.parametrize("l,C", [(1, 2), (3, 2), (5, 4)])
def test_small_and_ragged_bandlimits(l, C):
    # l = 1: one-row pairs and an empty one (m = 1, p = 1); l = 3, 5: not powers of two, leaves
    # of ragged width
    from paper_0910_5435_amd import OrderPlan

    plan = OrderPlan(l, eps=1e-14, leaf_width=C)
    assert plan.rows == l * (2 * l + 1)
    for R in (1, 5):
        _check_pairs(plan, l, R, _all_pairs(l), seed=l, label=f"l={l} C={C}")


def test_l256_sampled_orders_and_full_round_trip():
    from paper_0910_5435_amd import OrderPlan

    l = 256
    plan = OrderPlan(l, eps=1e-13, leaf_width=32)
    st = plan.stats()
    print(f"order maps l={l} C=32: k_max {st['k_max']}, k_avg {st['k_avg']:.1f}, k_sd {st['k_sd']:.1f}, "
          f"factor entries {st['factor_entries']:.3e} (dense {st['dense_entries']:.3e})", flush=True)
    assert st["factor_entries"] < st["dense_entries"]
    orders = [0, 1, 37, 100, 255, 256, 300, 510, 511]
    for R in (2, 32):
        x, y, z = _check_pairs(plan, l, R, [(m, p) for m in orders for p in (0, 1)], seed=R, label="l=256 C=32")
        # every pair: the inverse undoes the forward map (A is orthogonal)
        rt = np.linalg.norm(z - x, axis=0) / np.linalg.norm(x, axis=0)
        assert np.all(rt < FP64_TOL), rt.max()
        # and the forward map keeps each pair's norm
        for m in range(0, 2 * l, 17):
            for p in (0, 1):
                r0, n = plan.layout(m, p)
                if n:
                    nx, ny = np.linalg.norm(x[r0:r0 + n]), np.linalg.norm(y[r0:r0 + n])
                    assert abs(ny - nx) <= 1e-12 * nx


def test_order_plan_refuses_sht_calls_and_vice_versa():
    from paper_0910_5435_amd import OrderPlan, Plan, _lib

    lib = _lib.load()
    op = OrderPlan(8, leaf_width=4)
    buf = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert lib.sht_synth(op.handle, p, p, 1, p, 1 << 19, None) == _lib.SHT_EINVAL
    assert lib.sht_workspace_bytes(op.handle, 1, 0) == 0
    assert lib.sht_order_apply(op.handle, p, p, 1, 0, p, 1 << 19, None) == _lib.SHT_EINVAL  # in == out
    assert lib.sht_order_apply(op.handle, p, ctypes.c_void_p(buf.data_ptr() + 8 * 4096), 1, 2, p, 1 << 19,
                               None) == _lib.SHT_EINVAL  # transpose must be 0 or 1
    sp = Plan(8)
    assert lib.sht_order_rows(sp.handle) == _lib.SHT_EINVAL
    assert lib.sht_order_workspace_bytes(sp.handle, 4) == 0
    # the two plans of one bandlimit hold the same pairs with the same sizes
    for m in range(16):
        for par in (0, 1):
            assert op.layout(m, par)[1] == sp.tree(m, par)[1]
