"""Plausible mistakes planted in the oracle, on the CPU: each pin must catch the one it is
meant to catch, so a pin that passes is evidence, not an accident.  Every case patches one
piece of the oracle for the duration of the test and runs an existing pin against it."""
import numpy as np
import pytest

import oracle
import oracle.legendre
import oracle.sht
from tests import test_oracle_pins as pins


def _reverse_orders(orig):
    # e^{-i m phi} where the expansion has e^{+i m phi}: the order axis read backwards
    return lambda g, l, grid, direct: orig(g[:, ::-1, :], l, grid, direct)


def _scaled(orig, factor):
    return lambda *a, **k: orig(*a, **k) * factor


def _degree_shift(orig):
    # every order reads the function of the next degree (an index off by one)
    def f(orders, x, kmax):
        P = orig(orders, x, kmax + 1)
        return P[:, 1:, :]
    return f


def _weights_scaled(orig, factor):
    def f(n):
        x, w = orig(n)
        return x, w * factor
    return f


def _no_normalisation(orig):
    # analysis without the 1/N of the longitude sum
    return lambda f, l, grid, direct, normalize: orig(f, l, grid, direct, False)


def _seed_power(orig):
    # the seed (1 - x^2)^{m/2} of Pbar_m^m taken once too often for m >= 1
    def f(orders, x, kmax):
        P = orig(orders, x, kmax)
        s = np.sqrt((1.0 - np.asarray(x)) * (1.0 + np.asarray(x)))
        ms = np.asarray(orders)
        return P * np.where(ms[:, None, None] > 0, s[None, None, :], 1.0)
    return f


def _adjoint_without_factor_two(orig):
    # the real-field adjoint without its factor 2 on the m > 0 orders
    def f(r, l, kind="complex", grid="fft", direct=False, orders=None, **kw):
        out = orig(r, l, kind, grid, direct, orders, **kw)
        if kind == "real":
            out[:, 2 * l:] *= 0.5
        return out
    return f


def _odd_perturbation(orig):
    # a term odd in x slipped into the recurrence (breaks the parity of Section 3.3)
    def f(orders, x, kmax):
        return orig(orders, x, kmax) * (1.0 + 1e-12 * np.asarray(x))[None, None, :]
    return f


CASES = [
    ("seed power of Pbar_m^m", "package", "pbar_orders", _seed_power, pins.test_pbar_closed_forms_low_degree),
    ("seed power (Sturm-Liouville)", "package", "pbar_orders", _seed_power, pins.test_pbar_sturm_liouville),
    ("term odd in x", "package", "pbar_orders", _odd_perturbation, lambda: pins.test_pbar_parity(7)),
    ("real adjoint without the factor 2", "package", "synth_adjoint", _adjoint_without_factor_two,
     lambda: pins.test_adjoint_identity("real")),
    ("phi exponent sign", "sht", "_fourier_sum", _reverse_orders, pins.test_against_scipy_spherical_harmonics),
    ("phi exponent sign (worked grid)", "sht", "_fourier_sum", _reverse_orders, pins.test_worked_example_l1),
    ("Pbar scaled by 1 + 1e-9", "package", "pbar_orders", lambda o: _scaled(o, 1 + 1e-9),
     lambda: pins.test_unsold_sum_at_high_degree(0.3)),
    ("Pbar degree off by one", "sht", "pbar_orders", _degree_shift, pins.test_against_scipy_spherical_harmonics),
    ("weights scaled by 1 + 1e-9", "sht", "gauss_legendre", lambda o: _weights_scaled(o, 1 + 1e-9),
     lambda: pins.test_round_trip_exact(8, "complex", "fft")),
    ("analysis without 1/N", "sht", "_fourier_coeffs", _no_normalisation,
     lambda: pins.test_round_trip_exact(4, "real", "paper")),
]


@pytest.mark.parametrize("name,where,attr,plant,pin", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, name, where, attr, plant, pin):
    pin()  # the pin passes on the oracle as it is
    target = oracle if where == "package" else oracle.sht
    monkeypatch.setattr(target, attr, plant(getattr(target, attr)))
    with pytest.raises(AssertionError):
        pin()
