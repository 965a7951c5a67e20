"""Oracle: Gauss-Legendre nodes and normalized associated Legendre functions.

TEST INFRASTRUCTURE.  Plain, slow, FP64 CPU code.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg use it; the GPU library shares no
code with it.

Definitions followed (Tygert, "Fast algorithms for spherical harmonic
expansions, III"):

* theta grid: the 2l zeros of P_{2l}, ascending (Section 2, equation (thetas)).
* normalized associated Legendre function, no Condon-Shortley phase
  (Section 3.3, equation (association)); orthonormal on (-1, 1) for fixed m.

The functions are evaluated by the classical first-order-in-degree (step-one)
three-term recurrence in its normalized form,

    x P_k = a_{k+1} P_{k+1} + a_k P_{k-1},   a_k = sqrt((k^2 - m^2) / (4 k^2 - 1)),

seeded by the closed forms of P_m^m and P_{m+1}^m that equation (association)
gives.  This is deliberately not the step-two recurrence (recurrence0) /
(recurrence) with the coefficients (c_rec) / (d_rec) that the GPU column
kernel runs: the tests check one against the other.  Underflow of P_m^m at
large m is countered by carrying a separate integer power-of-two exponent per
value (the explicit exponent tracking that Section 5 mentions).
"""
import numpy as np

_BIG = 2.0 ** 400
_SMALL = 2.0 ** -400
_STEP = 400


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on (-1, 1): nodes ascending, weights.

    Newton's method on P_n evaluated by the textbook recurrence
    (k + 1) P_{k+1} = (2k + 1) x P_k - k P_{k-1}; weights
    w = 2 / ((1 - x^2) P_n'(x)^2).  The nodes are the zeros of P_n (equation
    (thetas) with n = 2l).  Antisymmetry of the rule is imposed at the end.
    """
    n = int(n)
    if n < 1:
        raise ValueError("n must be positive")
    i = np.arange(n, dtype=np.float64)
    x = np.cos(np.pi * (i + 0.75) / (n + 0.5))
    for it in range(200):
        p_prev = np.ones_like(x)
        p = x.copy()
        for k in range(1, n):
            p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
        dp = n * (x * p - p_prev) / ((x - 1.0) * (x + 1.0))
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-15 and it > 2:
            break
    # final derivative at the converged nodes
    p_prev = np.ones_like(x)
    p = x.copy()
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    dp = n * (x * p - p_prev) / ((x - 1.0) * (x + 1.0))
    w = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp)
    order = np.argsort(x)
    x, w = x[order], w[order]
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    return x, w


def pbar_orders(orders, x, kmax):
    """P[a, k, i] = normalized P_k^{m_a}(x_i) for k = 0..kmax (0 where k < m_a).

    Vectorised over the orders ``orders`` and points ``x``; degree by degree.
    """
    orders = np.asarray(orders, dtype=np.int64).ravel()
    x = np.asarray(x, dtype=np.float64).ravel()
    A, N = len(orders), len(x)
    out = np.zeros((A, kmax + 1, N))
    if A == 0 or N == 0 or kmax < 0:
        return out
    xx = x[None, :]
    sq = np.sqrt((1.0 - x) * (1.0 + x))[None, :]
    mf = orders.astype(np.float64)[:, None]
    # Running product prod_{j=1..k} sqrt((2j-1)/(2j)) * sqrt(1 - x^2), with exponent.
    r_mant = np.ones((1, N))
    r_exp = np.zeros((1, N), dtype=np.int64)
    prev = np.zeros((A, N))
    cur = np.zeros((A, N))
    ex = np.zeros((A, N), dtype=np.int64)
    for k in range(kmax + 1):
        if k > 0:
            r_mant = r_mant * (np.sqrt((2.0 * k - 1.0) / (2.0 * k)) * sq)
            small = (np.abs(r_mant) < _SMALL) & (r_mant != 0.0)
            r_mant = np.where(small, r_mant * _BIG, r_mant)
            r_exp = np.where(small, r_exp - _STEP, r_exp)
        # orders already started: one step of the recurrence to degree k
        act = (orders < k)[:, None]
        if np.any(act):
            a_k = np.sqrt(np.where(act, (k * k - mf * mf) / (4.0 * k * k - 1.0), 1.0))
            km1 = k - 1
            a_km1 = np.where(
                (orders < km1)[:, None],
                np.sqrt(np.maximum(km1 * km1 - mf * mf, 0.0) / max(4.0 * km1 * km1 - 1.0, 1.0)),
                0.0,
            )
            nxt = (xx * cur - a_km1 * prev) / a_k
            big = act & (np.abs(nxt) > _BIG)
            nxt = np.where(big, nxt * _SMALL, nxt)
            cur_s = np.where(big, cur * _SMALL, cur)
            ex = np.where(big, ex + _STEP, ex)
            prev = np.where(act, cur_s, prev)
            cur = np.where(act, nxt, cur)
        # orders starting at this degree: the seed P_m^m
        start = (orders == k)[:, None]
        if np.any(start):
            seed = np.sqrt((2.0 * k + 1.0) / 2.0) * r_mant
            cur = np.where(start, seed, cur)
            prev = np.where(start, 0.0, prev)
            ex = np.where(start, r_exp, ex)
        live = (orders <= k)[:, None]
        vals = np.ldexp(cur, np.clip(ex, -100000, 100000).astype(np.int32))
        out[:, k, :] = np.where(live, vals, 0.0)
    return out


def pbar_table(m, x, kmax):
    """T[i, j] = normalized P_{m+j}^m(x_i), j = 0..kmax-m."""
    P = pbar_orders([m], x, kmax)
    return P[0, m:, :].T.copy()


def step2_coefficients(m, degrees):
    """(c_l, d_l) of equations (c_rec) and (d_rec) for order m, degrees l."""
    l = np.asarray(degrees, dtype=np.float64)
    m = float(m)
    c = np.sqrt(
        (l - m + 1.0) * (l - m + 2.0) * (l + m + 1.0) * (l + m + 2.0)
        / ((2.0 * l + 1.0) * (2.0 * l + 3.0) ** 2 * (2.0 * l + 5.0))
    )
    d = (2.0 * l * (l + 1.0) - 2.0 * m * m - 1.0) / ((2.0 * l - 1.0) * (2.0 * l + 3.0))
    return c, d
