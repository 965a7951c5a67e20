"""Oracle: the per-order quadratures (Section 3.3) and transforms (Section 5).

TEST INFRASTRUCTURE.  Plain, slow, FP64 CPU code; only the tests use it and the library
shares no code with it.

Definitions followed (Tygert, "Fast algorithms for spherical harmonic expansions, III"):

* nodes: the n positive zeros x_j of Pbar^m_{m+2n} (parity 0) or y_j of Pbar^m_{m+2n+1}
  (parity 1), Lemma distinct_theorem, equations (zeros) and (zeros2);
* weights: rho_j of equation (weights1) and sigma_j of equation (weights2),
      rho_j   = 2 (2m + 4n + 1) / ((1 - x_j^2) Pbar^m_{m+2n}'(x_j)^2),
      sigma_j = 2 (2m + 4n + 3) / ((1 - y_j^2) Pbar^m_{m+2n+1}'(y_j)^2),
  the derivative taken from the textbook identity for normalized functions
      (1 - x^2) Pbar_L'(x) = sqrt((2L + 1)(L^2 - m^2) / (2L - 1)) Pbar_{L-1}(x) - L x Pbar_L(x);
* the matrices of equations (transform) and (transform2): sqrt(w_i) Pbar^m_{m+p+2j}(x_i).

The nodes start from the eigenvalues of the x^2 three-term recurrence of Lemma
rec_relation (numpy's dense symmetric eigensolver) and are then polished by Newton's method
on Pbar_L evaluated with the step-one table of ``legendre.pbar_table``, so the nodes and the
weights rest on the step-one recurrence.  The weights are returned also as
lambda_j = w_j (1 - x_j^2)^m, the weights of Lemma quadratures for the weight function
(1 - x^2)^m.  Meant for moderate m (the values carry (1 - x^2)^{+-m}).
"""
import numpy as np

from .legendre import pbar_table, step2_coefficients


def _degree(m, n, parity):
    return m + parity + 2 * n


def rule(m, n, parity=0):
    """(x, lam, w): nodes ascending in (0, 1), lambda = w (1 - x^2)^m, and w = rho or sigma."""
    m, n, parity = int(m), int(n), int(parity)
    if m < 0 or n < 1 or parity not in (0, 1):
        raise ValueError("need m >= 0, n >= 1, parity 0 or 1")
    L = _degree(m, n, parity)
    lj = m + parity + 2 * np.arange(n)
    c, d = step2_coefficients(m, lj)
    J = np.diag(d) + np.diag(c[:-1], 1) + np.diag(c[:-1], -1)
    x = np.sqrt(np.clip(np.linalg.eigvalsh(J), 0.0, 1.0))
    a = np.sqrt((2.0 * L + 1.0) * (L * L - m * m) / (2.0 * L - 1.0))

    def value_and_derivative(x):
        T = pbar_table(m, x, L)  # T[i, k] = Pbar^m_{m+k}(x_i)
        pL, pL1 = T[:, L - m], T[:, L - 1 - m]
        return pL, (a * pL1 - L * x * pL) / ((1.0 - x) * (1.0 + x))

    for _ in range(8):
        p, dp = value_and_derivative(x)
        step = p / dp
        x = x - step
        if np.max(np.abs(step) / x) < 1e-16:
            break
    _, dp = value_and_derivative(x)
    w = 2.0 * (2.0 * m + 4.0 * n + 1.0 + 2.0 * parity) / ((1.0 - x) * (1.0 + x) * dp * dp)
    lam = w * ((1.0 - x) * (1.0 + x)) ** m
    return x, lam, w


def matrix(m, n, parity=0):
    """The n x n matrix of (transform) (parity 0) or (transform2) (parity 1)."""
    x, _, w = rule(m, n, parity)
    T = pbar_table(m, x, m + parity + 2 * (n - 1))
    return np.sqrt(w)[:, None] * T[:, parity::2][:, :n]


def beta_moment(m, k):
    """Closed form of the integral over (-1, 1) of (1 - x^2)^m x^(2k): B(k + 1/2, m + 1).

    Evaluated from B(1/2, 1) = 2 by the Beta function's recurrences B(a, b + 1) =
    B(a, b) b / (a + b) and B(a + 1, b) = B(a, b) a / (a + b), summed in logarithms; a
    difference of log-gamma values would lose about |lgamma| ulps (1e-13 at m = 10^4)."""
    from math import exp, fsum, log, log1p

    logb = log(2.0) - fsum(log1p(0.5 / j) for j in range(1, m + 1))
    logb += fsum(log((i - 0.5) / (i + m + 0.5)) for i in range(1, k + 1))
    return exp(logb)
