"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types an oracle formula: each compares the oracle with
an independent source (a closed form derived by hand from equation
(association), a library routine, a high-precision evaluation, an identity of
the functions, a hand-worked grid, or an algebraic property of the maps).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps

import oracle
import sht_synthetic as syn

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Gauss-Legendre grid


def test_gl_small_closed_forms():
    x, w = oracle.gauss_legendre(2)
    np.testing.assert_allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], rtol=0, atol=3e-16)
    np.testing.assert_allclose(w, [1.0, 1.0], rtol=0, atol=1e-15)
    x, w = oracle.gauss_legendre(3)
    np.testing.assert_allclose(x, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], rtol=0, atol=3e-16)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 5, 10, 64, 128, 256])
def test_gl_vs_numpy_leggauss(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, rtol=0, atol=2e-15)
    # numpy's own weights carry ~1e-12 relative error at the ends of the interval
    np.testing.assert_allclose(w, wr, rtol=0, atol=3e-14)


def test_gl_vs_mpmath_high_precision():
    import mpmath as mp

    mp.mp.dps = 40
    n = 64
    x, w = oracle.gauss_legendre(n)
    for i in [0, 1, 2, n // 2, n - 1]:
        xi = mp.findroot(lambda t: mp.legendre(n, t), mp.mpf(x[i]))
        dp = mp.diff(lambda t: mp.legendre(n, t), xi)
        wi = 2 / ((1 - xi ** 2) * dp ** 2)
        assert abs(x[i] - float(xi)) <= 2.3e-16  # one ulp near 1
        assert abs(w[i] - float(wi)) <= 2e-13 * float(wi)


@pytest.mark.parametrize("n", [512, 2048])
def test_gl_vs_scipy_roots(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = sps.roots_legendre(n)
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-15)
    # scipy's weights lose ~1e-9 relative accuracy at the ends; compare absolutely
    np.testing.assert_allclose(w, wr, rtol=0, atol=5e-13)
    assert np.all(np.diff(x) > 0)  # ascending (equation (thetas) ordering)


@pytest.mark.parametrize("l", [4, 32, 128])
def test_gl_exact_to_degree_4l_minus_1(l):
    x, w = oracle.gauss_legendre(2 * l)
    for d in range(0, 4 * l, 1):
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs(np.sum(w * x ** d) - exact) < 1e-14, d


# ---------------------------------------------------------------- Pbar values


def _impl(pbar):
    """The Pbar table routine under test: the numpy oracle unless another is passed."""
    return pbar or oracle.pbar_orders


def test_pbar_closed_forms_low_degree(pbar=None):
    # From equation (association) by hand: no Condon-Shortley phase.
    x = np.linspace(-0.97, 0.97, 23)
    s = np.sqrt(1 - x * x)
    P = _impl(pbar)([0, 1, 2], x, 3)
    forms = {
        (0, 0): np.full_like(x, 1 / math.sqrt(2)),
        (1, 0): math.sqrt(1.5) * x,
        (1, 1): math.sqrt(3) / 2 * s,
        (2, 0): math.sqrt(2.5) * (3 * x * x - 1) / 2,
        (2, 1): math.sqrt(15) / 2 * x * s,
        (2, 2): math.sqrt(15) / 4 * (1 - x * x),
        (3, 0): math.sqrt(3.5) * (5 * x ** 3 - 3 * x) / 2,
    }
    for (k, m), ref in forms.items():
        np.testing.assert_allclose(P[m, k], ref, rtol=0, atol=2e-15, err_msg=f"k={k} m={m}")
    assert np.all(P[0, :, :][[0], :] > 0)


@pytest.mark.parametrize("m", [0, 1, 7, 120])
def test_pbar_parity(m, pbar=None):
    # Section 3.3: Pbar^m_l(-x) = (-1)^(l-m) Pbar^m_l(x).
    x = np.linspace(0.01, 0.99, 37)
    K = m + 400
    Pp = _impl(pbar)([m], x, K)[0]
    Pm = _impl(pbar)([m], -x, K)[0]
    sign = np.where((np.arange(K + 1) - m) % 2 == 0, 1.0, -1.0)[:, None]
    scale = np.max(np.abs(Pp), axis=1, keepdims=True) + 1e-300
    assert np.max(np.abs(Pm - sign * Pp) / scale) <= 1e-15


def test_pbar_sturm_liouville(pbar=None):
    # Lemma (sturm-liouville_Leg): -((1 - x^2) y')' + (m^2 / (1 - x^2) - l(l + 1)) y = 0, with
    # y' and y'' from fourth-order central differences (h = 1e-3; truncation ~1e-7 here).
    x = np.linspace(-0.8, 0.8, 17)
    h = 1e-3
    K = 15
    ms = list(range(K + 1))
    Y = {s: _impl(pbar)(ms, x + s * h, K) for s in (-2, -1, 0, 1, 2)}
    d1 = (Y[-2] - 8 * Y[-1] + 8 * Y[1] - Y[2]) / (12 * h)
    d2 = (-Y[-2] + 16 * Y[-1] - 30 * Y[0] + 16 * Y[1] - Y[2]) / (12 * h * h)
    for m in ms:
        for l in range(m, K + 1):
            y = Y[0][m, l]
            res = -(1 - x * x) * d2[m, l] + 2 * x * d1[m, l] + (m * m / (1 - x * x) - l * (l + 1)) * y
            scale = (1 + l * (l + 1) + m * m / (1 - 0.64)) * np.max(np.abs(y))
            assert np.max(np.abs(res)) <= 1e-6 * scale, (m, l, np.max(np.abs(res)), scale)


def _pbar_scipy(k, m, x):
    # scipy's lpmv carries the Condon-Shortley factor (-1)^m; the paper's function does not.
    norm = math.sqrt((2 * k + 1) / 2 * math.exp(math.lgamma(k - m + 1) - math.lgamma(k + m + 1)))
    return (-1) ** m * norm * sps.lpmv(m, k, x)


def test_pbar_vs_scipy_lpmv(pbar=None):
    x = np.linspace(-0.95, 0.95, 17)
    K = 30
    P = _impl(pbar)(list(range(K + 1)), x, K)
    for m in range(0, K + 1):
        for k in range(m, K + 1):
            ref = _pbar_scipy(k, m, x)
            np.testing.assert_allclose(P[m, k], ref, rtol=0, atol=5e-13 * max(1.0, np.max(np.abs(ref))),
                                       err_msg=f"k={k} m={m}")


def _pbar_exact(k, m, x):
    """Equation (association) evaluated in high precision from the exact power series.

    P_k(x) = 2^-k sum_j (-1)^j C(k, j) C(2k - 2j, k) x^(k - 2j); differentiate m times
    term by term with exact integers, evaluate with enough digits to survive the
    cancellation, multiply by the normalization and (1 - x^2)^(m/2).
    """
    import mpmath as mp

    mp.mp.dps = int(0.75 * k) + 60
    xx = mp.mpf(x)
    total = mp.mpf(0)
    for j in range(0, k // 2 + 1):
        e = k - 2 * j
        if e < m:
            break
        coef = (-1) ** j * math.comb(k, j) * math.comb(2 * k - 2 * j, k)
        coef *= math.factorial(e) // math.factorial(e - m)
        total += mp.mpf(coef) * xx ** (e - m)
    total /= mp.mpf(2) ** k
    norm = mp.sqrt(mp.mpf(2 * k + 1) / 2 * mp.factorial(k - m) / mp.factorial(k + m))
    return norm * (1 - xx * xx) ** (mp.mpf(m) / 2) * total


@pytest.mark.parametrize(
    "m,x,ks",
    [
        (775, 0.924, [775, 1000, 1400, 2047]),  # seed ~1e-323: the underflow band at l = 1024
        (1500, 0.95, [1500, 2500, 4095]),       # seed far below the FP64 range (l = 2048)
        (3, 0.3, [3, 500, 2047]),
    ],
)
def test_pbar_vs_exact_series_extreme(m, x, ks, pbar=None):
    kmax = max(ks)
    P = _impl(pbar)([m], [x], kmax)[0, :, 0]
    for k in ks:
        ref = float(_pbar_exact(k, m, x))
        if abs(ref) < 1e-300:
            assert abs(P[k] - ref) <= 1e-300
        else:
            # purely relative: exponent tracking keeps full relative accuracy at any magnitude
            # in the FP64 range (an absolute slack would hide a lost exponent at 1e-40)
            assert abs(P[k] - ref) <= 1e-12 * abs(ref), (k, P[k], ref)


@pytest.mark.parametrize("x", [0.05, 0.3, 0.924, 0.99, 0.9999])
def test_unsold_sum_at_high_degree(x, pbar=None):
    # sum_{m=-k}^{k} Pbar_k^{|m|}(x)^2 = (2k + 1) / 2 for every k (addition theorem).
    K = 2047
    P = _impl(pbar)(list(range(K + 1)), [x], K)[:, :, 0]  # [m, k]
    for k in [0, 1, 100, 1023, 1500, 2047]:
        s = P[0, k] ** 2 + 2 * np.sum(P[1 : k + 1, k] ** 2)
        assert abs(s - (2 * k + 1) / 2) <= 1e-12 * (2 * k + 1), (k, s)


@pytest.mark.parametrize("m", [0, 1, 3, 50, 400])
def test_step2_recurrence_holds(m, pbar=None):
    # Lemma rec_relation, equations (recurrence0) and (recurrence) with (c_rec), (d_rec).
    x = np.linspace(-0.9, 0.9, 11)
    K = m + 200
    P = _impl(pbar)([m], x, K + 2)[0]
    ls = np.arange(m, K + 1)
    c, d = oracle.step2_coefficients(m, ls)
    cm2, _ = oracle.step2_coefficients(m, ls - 2)
    for idx, l in enumerate(ls):
        lhs = x * x * P[l]
        rhs = d[idx] * P[l] + c[idx] * P[l + 2]
        if l >= m + 2:
            rhs = rhs + cm2[idx] * P[l - 2]
        scale = max(1.0, np.max(np.abs(P[l])))
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13 * scale, err_msg=f"l={l}")


def test_step2_closed_values():
    c, d = oracle.step2_coefficients(0, [0])
    assert abs(c[0] - 2 / (3 * math.sqrt(5))) < 1e-16
    assert abs(d[0] - 1 / 3) < 1e-16
    for m in [0, 4, 17]:
        _, d = oracle.step2_coefficients(m, [m])
        assert abs(d[0] - 1 / (2 * m + 3)) < 1e-15


@pytest.mark.parametrize("m", [0, 1, 5, 300, 2000])
def test_step2_coefficients_are_products_of_step1_coefficients(m):
    # Squaring the step-one recurrence x P_k = a_{k+1} P_{k+1} + a_k P_{k-1},
    # a_k = sqrt((k^2 - m^2) / (4k^2 - 1)), gives (recurrence0)/(recurrence) with
    # c_l = a_{l+1} a_{l+2} and d_l = a_{l+1}^2 + a_l^2 (a_m = 0).
    ls = np.arange(m, m + 300)

    def a(k):
        k = np.asarray(k, dtype=np.float64)
        return np.sqrt(np.maximum(k * k - m * m, 0.0) / (4.0 * k * k - 1.0))

    c, d = oracle.step2_coefficients(m, ls)
    np.testing.assert_allclose(c, a(ls + 1) * a(ls + 2), rtol=1e-15, atol=0)
    np.testing.assert_allclose(d, a(ls + 1) ** 2 + a(ls) ** 2, rtol=1e-15, atol=0)


@pytest.mark.parametrize("l", [4, 16, 40])
def test_orthonormal_columns_all_orders(l):
    for m in range(2 * l):
        for p in (0, 1):
            Q = oracle.dense_q(l, m, p)
            n = Q.shape[1]
            assert n == oracle.folded_sizes(l, m)[p]
            if n:
                np.testing.assert_allclose(Q.T @ Q, np.eye(n), rtol=0, atol=2e-14)


@pytest.mark.parametrize("m", [0, 333, 700, 1023])
def test_orthonormal_columns_l512(m):
    for p in (0, 1):
        Q = oracle.dense_q(512, m, p)
        np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), rtol=0, atol=5e-13)


# ---------------------------------------------------------------- layout


@pytest.mark.parametrize("kind", ["complex", "real"])
def test_coefficient_layout_matches_generator(kind):
    for l in [1, 2, 5]:
        n = oracle.n_coeffs(l, kind)
        ks = syn.degrees_canonical(l, kind)
        ms = syn.orders_canonical(l, kind)
        assert len(ks) == n
        seen = set()
        for pos, (k, m) in enumerate(zip(ks, ms)):
            assert oracle.coeff_index(l, int(k), int(m), kind) == pos
            seen.add((int(k), int(m)))
        assert len(seen) == n


# ---------------------------------------------------------------- whole transform


def test_worked_example_l1(fast=False):
    g = json.load(open(os.path.join(HERE, "golden", "l1_worked_example.json")))
    l = g["l"]
    x, w = oracle.gauss_legendre(2 * l)
    np.testing.assert_allclose(x, g["nodes"], rtol=0, atol=3e-16)
    np.testing.assert_allclose(w, g["weights"], rtol=0, atol=1e-15)
    for case in g["cases"]:
        beta = np.zeros((1, oracle.n_coeffs(l)), dtype=complex)
        beta[0, oracle.coeff_index(l, case["k"], case["m"])] = 1.0
        ref = np.array(case["grid_re"]) + 1j * np.array(case["grid_im"])
        for direct in (False, True):
            f = oracle.synth(beta, l, direct=direct, fast=fast)[0]
            np.testing.assert_allclose(f, ref, rtol=0, atol=1e-15)
        back = oracle.analyze(ref[None], l, fast=fast)
        np.testing.assert_allclose(back, beta, rtol=0, atol=1e-15)


def test_against_scipy_spherical_harmonics(fast=False):
    # Pbar_k^{|m|}(cos t) e^{i m p} = sqrt(2 pi) (-1)^m Y_k^m(t, p) for m >= 0, and the
    # conjugate form for m < 0 (scipy's Y carries the Condon-Shortley phase).
    l = 4
    beta = syn.coefficients(l, 2, seed=3)
    f = oracle.synth(beta, l, fast=fast)
    x, _ = oracle.gauss_legendre(2 * l)
    theta = np.arccos(x)
    phi = oracle.phi_points(l)
    T, PH = np.meshgrid(theta, phi, indexing="ij")
    ref = np.zeros_like(f)
    ks, ms = syn.degrees_canonical(l), syn.orders_canonical(l)
    for pos, (k, m) in enumerate(zip(ks, ms)):
        am = abs(int(m))
        Y = sps.sph_harm_y(int(k), am, T, PH)
        basis = math.sqrt(2 * math.pi) * (-1) ** am * (Y if m >= 0 else np.conj(Y))
        ref += beta[:, pos][:, None, None] * basis[None]
    np.testing.assert_allclose(f, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("l", [1, 2, 3, 5, 8, 16])
@pytest.mark.parametrize("kind", ["complex", "real"])
@pytest.mark.parametrize("grid", ["fft", "paper"])
def test_round_trip_exact(l, kind, grid, fast=False):
    beta = syn.coefficients(l, 3, seed=l, kind=kind)
    f = oracle.synth(beta, l, kind=kind, grid=grid, fast=fast)
    if kind == "real":
        assert np.isrealobj(f)
    back = oracle.analyze(f, l, kind=kind, grid=grid, fast=fast)
    np.testing.assert_allclose(back, beta, rtol=0, atol=1e-13 * np.max(np.abs(beta)))


@pytest.mark.parametrize("l", [2, 8, 32])
def test_fft_equals_direct_sum(l):
    beta = syn.coefficients(l, 2, seed=11)
    f1 = oracle.synth(beta, l, direct=False)
    f2 = oracle.synth(beta, l, direct=True)
    np.testing.assert_allclose(f1, f2, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.analyze(f1, l, direct=True), oracle.analyze(f1, l), rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind", ["complex", "real"])
def test_adjoint_identity(kind, fast=False):
    # <synth(b), r>_R == <b, synth_adjoint(r)>_R  (real inner products)
    l = 6
    b = syn.coefficients(l, 2, seed=5, kind=kind)
    r = syn.grid(l, 2, seed=6, kind=kind)
    lhs = np.sum(np.real(np.conj(oracle.synth(b, l, kind=kind, fast=fast)) * r))
    rhs = np.sum(np.real(np.conj(b) * oracle.synth_adjoint(r, l, kind=kind, fast=fast)))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_subset_routines_agree_with_full():
    l = 8
    beta = syn.coefficients(l, 2, seed=9)
    f = oracle.synth(beta, l)
    rings = [0, 5, 2 * l - 1]
    np.testing.assert_allclose(oracle.ring_values(beta, l, rings), f[:, rings], rtol=0, atol=1e-14)
    keep = [0, 2, 5]
    masked = beta.copy()
    ms = syn.orders_canonical(l)
    masked[:, ~np.isin(np.abs(ms), keep)] = 0.0
    np.testing.assert_allclose(oracle.synth(beta, l, orders=keep), oracle.synth(masked, l), rtol=0, atol=1e-14)
    full = oracle.analyze(f, l)
    part = oracle.analyze_orders(f, l, [0, 3, -7])
    for m in [0, 3, -3, 7, -7]:
        for k in range(abs(m), 2 * l):
            i = oracle.coeff_index(l, k, m)
            assert abs(part[0, i] - full[0, i]) < 1e-14
    adj_full = oracle.synth_adjoint(f, l)
    adj_part = oracle.synth_adjoint(f, l, orders=[0, 3])
    sel = np.isin(np.abs(ms), [0, 3])
    np.testing.assert_allclose(adj_part[:, sel], adj_full[:, sel], rtol=0, atol=1e-13)
    assert np.all(adj_part[:, ~sel] == 0)


@pytest.mark.parametrize("kind", ["complex", "real"])
def test_adjoint_is_gradient_of_squared_misfit(kind):
    # The gradient of L(b) = sum |synth(b) - T|^2 with respect to the real and imaginary
    # parts of every stored coefficient, packed as dL/dRe + i dL/dIm, equals
    # 2 synth_adjoint(synth(b) - T); checked entry by entry with central differences
    # (L is quadratic, so the differences are exact up to rounding).
    l = 4
    b = syn.coefficients(l, 1, seed=11, kind=kind)
    T = syn.grid(l, 1, seed=12, kind=kind)

    def loss(bb):
        d = oracle.synth(bb, l, kind=kind) - T
        return float(np.sum(np.abs(d) ** 2))

    grad = 2.0 * oracle.synth_adjoint(oracle.synth(b, l, kind=kind) - T, l, kind=kind)[0]
    h = 1e-5
    for i in range(b.shape[1]):
        for unit in (1.0, 1j):
            bp = b.copy()
            bm = b.copy()
            bp[0, i] += h * unit
            bm[0, i] -= h * unit
            fd = (loss(bp) - loss(bm)) / (2 * h)
            an = grad[i].real if unit == 1.0 else grad[i].imag
            assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (kind, i, unit, fd, an)
