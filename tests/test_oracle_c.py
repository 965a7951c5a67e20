"""The oracle's plain-C Legendre table (oracle/pbar.c) and the fast path built on it.

The C routine evaluates the same definition by the same step-one recurrence as the numpy
oracle; it is pinned here on its own by the pins of the Pbar functions (closed forms from
equation (association), parity, the Sturm-Liouville equation, scipy, exact series in the
underflow band, Unsold's sum, the step-two recurrence, orthonormality under the
Gauss-Legendre rule), the fast transform path by the whole-transform pins (the hand-worked
l = 1 grid, scipy's spherical harmonics, exact round trips, the adjoint identity), and
plausible mistakes planted into a patched copy of the C source must each fail a pin.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import sht_synthetic as syn
from oracle import pbar_c
from tests import test_oracle_pins as pins

C_SRC = os.path.join(os.path.dirname(pbar_c.__file__), "pbar.c")


@pytest.fixture(scope="module", autouse=True)
def _library():
    if not os.path.exists(pbar_c.LIB_PATH):
        from oracle import build

        build.build()
    pbar_c.load()


def _c(lib=None):
    return lambda orders, x, kmax: pbar_c.pbar_orders_c(orders, x, kmax, lib=lib)


PBAR_PINS = [
    ("closed forms", lambda p: pins.test_pbar_closed_forms_low_degree(pbar=p)),
    ("parity m=7", lambda p: pins.test_pbar_parity(7, pbar=p)),
    ("parity m=120", lambda p: pins.test_pbar_parity(120, pbar=p)),
    ("Sturm-Liouville", lambda p: pins.test_pbar_sturm_liouville(pbar=p)),
    ("scipy lpmv", lambda p: pins.test_pbar_vs_scipy_lpmv(pbar=p)),
    ("exact series m=775", lambda p: pins.test_pbar_vs_exact_series_extreme(775, 0.924, [775, 1000, 1400, 2047], pbar=p)),
    ("exact series m=1500", lambda p: pins.test_pbar_vs_exact_series_extreme(1500, 0.95, [1500, 2500, 4095], pbar=p)),
    ("exact series m=3", lambda p: pins.test_pbar_vs_exact_series_extreme(3, 0.3, [3, 500, 2047], pbar=p)),
    ("Unsold x=0.3", lambda p: pins.test_unsold_sum_at_high_degree(0.3, pbar=p)),
    ("Unsold x=0.9999", lambda p: pins.test_unsold_sum_at_high_degree(0.9999, pbar=p)),
    ("step-two recurrence m=50", lambda p: pins.test_step2_recurrence_holds(50, pbar=p)),
]


@pytest.mark.parametrize("name,pin", PBAR_PINS, ids=[c[0] for c in PBAR_PINS])
def test_c_table_meets_pbar_pins(name, pin):
    pin(_c())


def _q_c(l, m, p):
    x, w = oracle.gauss_legendre(2 * l)
    xp, wp = x[l:], w[l:]
    n = oracle.folded_sizes(l, m)[p]
    T = pbar_c.pbar_table_c(m, xp, 2 * l - 1)  # degrees m..2l-1
    cols = T[p : p + 2 * n : 2, :].T
    return np.sqrt(2.0 * wp)[:, None] * cols


@pytest.mark.parametrize("l,orders,tol", [(40, None, 2e-14), (512, [0, 333, 1023], 5e-13),
                                          (1024, [0, 775, 1500, 2047], 1e-12)])
def test_c_table_orthonormal_columns(l, orders, tol):
    # orthonormality of Section 3.3 with parity and the exactness of the Gauss-Legendre rule
    for m in (range(2 * l) if orders is None else orders):
        for p in (0, 1):
            Q = _q_c(l, m, p)
            if Q.shape[1]:
                np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), rtol=0, atol=tol)


FAST_PINS = [
    ("worked grid l=1", lambda: pins.test_worked_example_l1(fast=True)),
    ("scipy spherical harmonics", lambda: pins.test_against_scipy_spherical_harmonics(fast=True)),
    ("round trip complex", lambda: pins.test_round_trip_exact(16, "complex", "fft", fast=True)),
    ("round trip real, paper grid", lambda: pins.test_round_trip_exact(8, "real", "paper", fast=True)),
    ("adjoint identity complex", lambda: pins.test_adjoint_identity("complex", fast=True)),
    ("adjoint identity real", lambda: pins.test_adjoint_identity("real", fast=True)),
]


@pytest.mark.parametrize("name,pin", FAST_PINS, ids=[c[0] for c in FAST_PINS])
def test_fast_path_meets_transform_pins(name, pin):
    pin()


@pytest.mark.parametrize("kind", ["complex", "real"])
def test_fast_path_equals_numpy_path(kind):
    # the C table reproduces the numpy table bit for bit (same recurrence, same operations),
    # so the two paths of every transform agree exactly
    l = 24
    b = syn.coefficients(l, 2, seed=1, kind=kind)
    r = syn.grid(l, 2, seed=2, kind=kind)
    assert np.array_equal(oracle.synth(b, l, kind=kind), oracle.synth(b, l, kind=kind, fast=True))
    assert np.array_equal(oracle.analyze(r, l, kind=kind), oracle.analyze(r, l, kind=kind, fast=True))
    assert np.array_equal(oracle.synth_adjoint(r, l, kind=kind), oracle.synth_adjoint(r, l, kind=kind, fast=True))
    x, _ = oracle.gauss_legendre(2 * l)
    assert np.array_equal(oracle.pbar_orders(range(2 * l), x, 2 * l - 1),
                          pbar_c.pbar_orders_c(range(2 * l), x, 2 * l - 1))


# (description, text in pbar.c, planted replacement, pin that must fail)
PLANTS = [
    ("seed normalisation", "sqrt((2.0 * m + 1.0) / 2.0) * mant", "sqrt((2.0 * m + 2.0) / 2.0) * mant",
     "closed forms"),
    ("seed factor index", "sqrt((2.0 * j - 1.0) / (2.0 * j))", "sqrt((2.0 * j - 1.0) / (2.0 * j + 1.0))",
     "scipy lpmv"),
    ("recurrence coefficient a_k of the wrong degree",
     "const double a_k = k > m ? sqrt((kk * kk - mm * mm)", "const double a_k = k > m ? sqrt((k1 * k1 - mm * mm)",
     "scipy lpmv"),
    ("sign of the three-term recurrence", "(x[i] * cur[i] - a_k * prev[i])", "(x[i] * cur[i] + a_k * prev[i])",
     "Sturm-Liouville"),
    ("exponent lost on rescaling in the recurrence", "ex[i] += STEP;", "ex[i] += STEP - 1;",
     "exact series m=775"),
    ("exponent lost on rescaling the seed", "e -= STEP;", "e -= STEP + 1;", "exact series m=1500"),
]


@pytest.mark.parametrize("name,old,new,pin_name", PLANTS, ids=[c[0] for c in PLANTS])
def test_planted_mistake_in_c_table_is_caught(tmp_path, name, old, new, pin_name):
    src = open(C_SRC).read()
    assert src.count(old) == 1, old
    bad = tmp_path / "pbar_planted.c"
    bad.write_text(src.replace(old, new))
    so = tmp_path / "libpbar_planted.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so), str(bad), "-lm"],
                   check=True)
    lib = pbar_c.load(str(so))
    pin = dict(PBAR_PINS)[pin_name]
    pin(_c())  # the pin passes on the oracle's own table
    with pytest.raises(AssertionError):
        pin(_c(lib))
