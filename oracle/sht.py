"""Oracle: the spherical harmonic transform written out from its definition.

TEST INFRASTRUCTURE.  Plain FP64 CPU code (numpy); only the tests, the smoke
check and the benchmark's CPU-baseline leg use it.  Nothing here is shared
with the GPU library.

Synthesis (coefficients -> grid) is the regrouped expansion of Section 2,
equation (alternate_expansion):

    f(theta_i, phi_j) = sum_m e^{i m phi_j} g_m(x_i),
    g_m(x)            = sum_{k=|m|}^{2l-1} beta_k^m Pbar_k^{|m|}(x),

with x_i the 2l Gauss-Legendre nodes (equation (thetas)).  The sums over k are
done directly (O(l^3)); the sums over m by a DFT (numpy.fft, or the direct
sum when asked).

Analysis (grid -> coefficients) is its exact inverse on band-limited data:

    G_m(x_i)  = (1/N) sum_j f(theta_i, phi_j) e^{-i m phi_j},
    beta_k^m  = sum_i w_i Pbar_k^{|m|}(x_i) G_m(x_i),

exact because the 2l-point Gauss-Legendre rule integrates polynomials of
degree <= 4l - 1 (products here have degree <= 4l - 2) and the N-point DFT
separates |m - m'| < N.  The adjoint of synthesis (used by autograd) is the
same sum without w_i and without 1/N.

Readings where the paper leaves room (each is listed in the design notes):

* phi grid: N = 4l points phi_j = 2 pi j / (4l) ("fft"); the paper's own
  4l - 1 half-offset points of equation (phis) are available as "paper".
* Pbar has no Condon-Shortley phase and negative orders use Pbar^{|m|}
  unchanged (equations (expansion), (association)); hence real fields obey
  beta_k^{-m} = conj(beta_k^m).
* Storage order of the coefficients: see ``coeff_index``.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .legendre import gauss_legendre, pbar_orders


# ----------------------------------------------------------------------------------------
# storage layout (the oracle's own copy; the GPU library has an independent one)


def n_coeffs(l, kind="complex"):
    return 4 * l * l if kind == "complex" else 2 * l * l + l


def _order_offset(l, am, kind):
    """Index of the first entry of order |m| = am in one field's vector."""
    L2 = 2 * l
    if kind == "real":
        return am * L2 - am * (am - 1) // 2
    if am == 0:
        return 0
    return L2 + 2 * (am - 1) * L2 - (am - 1) * am


def coeff_index(l, k, m, kind="complex"):
    """Position of beta_k^m: orders |m| ascending; +m block then -m; k contiguous."""
    am = abs(m)
    if not (0 <= am <= k <= 2 * l - 1):
        raise IndexError("need |m| <= k <= 2l - 1")
    if kind == "real" and m < 0:
        raise IndexError("real fields store m >= 0 only")
    base = _order_offset(l, am, kind)
    if m < 0:
        base += 2 * l - am
    return base + (k - am)


def _order_slice(l, m, kind):
    start = coeff_index(l, abs(m), m, kind)
    return slice(start, start + 2 * l - abs(m))


def phi_points(l, grid="fft"):
    if grid == "fft":
        N = 4 * l
        return 2.0 * np.pi * np.arange(N) / N
    if grid == "paper":  # equation (phis)
        N = 4 * l - 1
        return 2.0 * np.pi * (np.arange(N) + 0.5) / N
    raise ValueError(grid)


def folded_sizes(l, m):
    """(n_even, n_odd): number of degrees k = m..2l-1 with k - m even / odd."""
    n = 2 * l - m
    return (n + 1) // 2, n // 2


# ----------------------------------------------------------------------------------------
# Legendre sums and their inverses


def _chunks(seq, size):
    for s in range(0, len(seq), size):
        yield seq[s : s + size]


def _workers():
    """Threads of the fast path: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _complex_times_real(A, B):
    """A @ B for complex A and real B as two real products (the real and imaginary parts)."""
    F = A.shape[0]
    R = np.concatenate([A.real, A.imag], axis=0) @ B
    return R[:F] + 1j * R[F:]


def _for_each_order(aorders, x, kmax, fast, fn):
    """Calls fn(m, T) with T[k - m, i] = Pbar_k^m(x_i), k = m..kmax, for every order.

    Default: numpy tables (``pbar_orders``) for chunks of orders, in order.  fast=True: the
    same functions from the C routine of ``pbar_c`` (same recurrence), one order per task
    on a pool of threads (orders are independent; each task writes only its own order's
    outputs, and the products inside a task run single-threaded).
    """
    if not fast:
        chunk = max(1, min(len(aorders), (1 << 24) // max(1, (kmax + 1) * len(x))))
        for ms in _chunks(aorders, chunk):
            P = pbar_orders(ms, x, kmax)
            for a, m in enumerate(ms):
                fn(m, P[a, m:, :])
        return
    from threadpoolctl import threadpool_limits

    from .pbar_c import pbar_table_c

    def task(m):
        fn(m, pbar_table_c(m, x, kmax))

    with threadpool_limits(1), ThreadPoolExecutor(_workers()) as ex:
        for _ in ex.map(task, list(aorders)):
            pass


def legendre_sums(beta, l, x, kind="complex", orders_per_chunk=None, orders=None, fast=False):
    """g[f, m + 2l - 1, i] = sum_k beta_k^m Pbar_k^{|m|}(x_i) for all m.

    For real fields the negative orders are filled in by conjugation.  With
    ``orders`` (a list of |m|) only those orders are summed; the others stay 0,
    i.e. the coefficients of the other orders are treated as zero.  ``fast`` takes the
    tables from the C routine on a pool of threads (see ``_for_each_order``).
    """
    beta = np.atleast_2d(np.asarray(beta, dtype=np.complex128))
    F = beta.shape[0]
    x = np.asarray(x, dtype=np.float64)
    N = len(x)
    L2 = 2 * l
    g = np.zeros((F, 2 * L2 - 1, N), dtype=np.complex128)
    aorders = list(range(L2)) if orders is None else sorted({abs(int(m)) for m in orders})

    def one(m, Pm):  # Pm: (degrees, nodes)
        g[:, m + L2 - 1, :] = _complex_times_real(beta[:, _order_slice(l, m, kind)], Pm)
        if m > 0:
            if kind == "complex":
                g[:, -m + L2 - 1, :] = _complex_times_real(beta[:, _order_slice(l, -m, kind)], Pm)
            else:
                g[:, -m + L2 - 1, :] = np.conj(g[:, m + L2 - 1, :])

    if orders_per_chunk is not None and not fast:
        for ms in _chunks(aorders, orders_per_chunk):
            P = pbar_orders(ms, x, L2 - 1)
            for a, m in enumerate(ms):
                one(m, P[a, m:, :])
    else:
        _for_each_order(aorders, x, L2 - 1, fast, one)
    return g


def _fourier_sum(g, l, grid, direct):
    """f[f, i, j] = sum_m g[f, m, i] e^{i m phi_j}."""
    L2 = 2 * l
    ms = np.arange(-(L2 - 1), L2)
    phi = phi_points(l, grid)
    if grid == "fft" and not direct:
        N = 4 * l
        F, _, Ni = g.shape
        bins = np.zeros((F, Ni, N), dtype=np.complex128)
        bins[:, :, ms % N] = np.transpose(g, (0, 2, 1))
        return np.fft.ifft(bins, axis=-1) * N
    E = np.exp(1j * np.outer(ms, phi))  # (m, j)
    return np.einsum("fmi,mj->fij", g, E)


def _fourier_coeffs(f, l, grid, direct, normalize):
    """G[f, m + 2l - 1, i] = (1/N)^normalize sum_j f[f, i, j] e^{-i m phi_j}."""
    L2 = 2 * l
    ms = np.arange(-(L2 - 1), L2)
    phi = phi_points(l, grid)
    N = len(phi)
    f = np.asarray(f)
    if grid == "fft" and not direct:
        G = np.fft.fft(f, axis=-1)[:, :, ms % N]
    else:
        E = np.exp(-1j * np.outer(phi, ms))  # (j, m)
        G = f @ E
    G = np.transpose(G, (0, 2, 1))
    if normalize:
        G = G / N
    return G


def synth(beta, l, kind="complex", grid="fft", direct=False, orders=None, fast=False):
    """Grid values f[field, ring, j] from coefficients beta[field, :] (canonical order).

    ``orders`` restricts the expansion to the listed |m| (other orders taken as zero);
    ``fast`` takes the Legendre tables from the C routine on a pool of threads.
    """
    x, _ = gauss_legendre(2 * l)
    g = legendre_sums(beta, l, x, kind, orders=orders, fast=fast)
    f = _fourier_sum(g, l, grid, direct)
    return f.real.copy() if kind == "real" else f


def ring_values(beta, l, rings, kind="complex", grid="fft", direct=False):
    """Synthesis restricted to the rings listed (indices into the ascending nodes)."""
    x, _ = gauss_legendre(2 * l)
    g = legendre_sums(beta, l, x[np.asarray(rings)], kind)
    f = _fourier_sum(g, l, grid, direct)
    return f.real.copy() if kind == "real" else f


def _coefficient_sums(G, l, weights, x, kind, orders=None, fast=False):
    """beta_k^m = sum_i weights_i Pbar_k^{|m|}(x_i) G[f, m, i] for the orders asked."""
    F = G.shape[0]
    L2 = 2 * l
    out = np.zeros((F, n_coeffs(l, kind)), dtype=np.complex128)
    aorders = list(range(L2)) if orders is None else sorted({abs(int(m)) for m in orders})

    def one(m, Pm):
        PWT = (Pm * weights[None, :]).T  # (nodes, degrees), a transposed view
        out[:, _order_slice(l, m, kind)] = _complex_times_real(G[:, m + L2 - 1, :], PWT)
        if m > 0 and kind == "complex":
            out[:, _order_slice(l, -m, kind)] = _complex_times_real(G[:, -m + L2 - 1, :], PWT)

    _for_each_order(aorders, x, L2 - 1, fast, one)
    return out


def analyze(f, l, kind="complex", grid="fft", direct=False, fast=False):
    """Coefficients (canonical order) from grid values f[field, ring, j]."""
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None]
    x, w = gauss_legendre(2 * l)
    G = _fourier_coeffs(f.astype(np.complex128), l, grid, direct, normalize=True)
    out = _coefficient_sums(G, l, w, x, kind, fast=fast)
    if kind == "real":
        out[:, : 2 * l] = out[:, : 2 * l].real
    return out


def analyze_orders(f, l, orders, kind="complex", grid="fft", fast=False):
    """Analysis for a subset of orders; entries of other orders are left at zero."""
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None]
    x, w = gauss_legendre(2 * l)
    G = _fourier_coeffs(f.astype(np.complex128), l, grid, False, normalize=True)
    out = _coefficient_sums(G, l, w, x, kind, orders, fast=fast)
    if kind == "real":
        out[:, : 2 * l] = out[:, : 2 * l].real
    return out


def synth_adjoint(r, l, kind="complex", grid="fft", direct=False, orders=None, fast=False):
    """Adjoint of ``synth`` for the real inner products of its input and output.

    Complex fields: gamma_k^m = sum_i Pbar_k^{|m|}(x_i) sum_j r_ij e^{-i m phi_j}
    (the conjugate transpose).  Real fields (m >= 0 stored, beta^{-m} =
    conj(beta^m)): the same sum times 2 for m > 0, real part only at m = 0.
    With ``orders`` (a list of |m|) only those orders are computed; the others are 0.
    """
    r = np.asarray(r)
    if r.ndim == 2:
        r = r[None]
    x, _ = gauss_legendre(2 * l)
    G = _fourier_coeffs(r.astype(np.complex128), l, grid, direct, normalize=False)
    out = _coefficient_sums(G, l, np.ones_like(x), x, kind, orders, fast=fast)
    if kind == "real":
        out *= 2.0
        out[:, : 2 * l] = 0.5 * out[:, : 2 * l].real
    return out


# ----------------------------------------------------------------------------------------
# per-order, per-parity matrices on the positive nodes


def dense_q(l, m, p):
    """Q[i, j] = sqrt(2 w_i) Pbar^m_{m+p+2j}(x_i) over the l positive nodes (ascending).

    Columns are orthonormal (orthonormality of Section 3.3 plus parity and the
    exactness of the Gauss-Legendre rule); this is the analogue on the common
    grid of the paper's unitary per-order maps (transform), (transform2).
    """
    x, w = gauss_legendre(2 * l)
    xp, wp = x[l:], w[l:]
    n = folded_sizes(l, m)[p]
    if n == 0:
        return np.zeros((l, 0))
    T = pbar_orders([m], xp, 2 * l - 1)[0]  # (degrees 0..2l-1, nodes)
    cols = T[m + p : m + p + 2 * n : 2, :].T
    return np.sqrt(2.0 * wp)[:, None] * cols
