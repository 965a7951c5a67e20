"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the transform.  It only draws pseudorandom
numbers in the canonical storage orders that the C ABI documents:

* coefficients, complex fields: per field, orders |m| = 0 .. 2l-1 in turn; for
  |m| > 0 the block of +m comes before the block of -m; inside a block the
  degrees k = |m| .. 2l-1 are contiguous.  4 l^2 complex numbers per field.
* coefficients, real fields (Hermitian symmetry beta_k^{-m} = conj(beta_k^m)):
  only m >= 0 is stored, |m| = 0 .. 2l-1, degrees contiguous.  2 l^2 + l
  complex numbers per field; the imaginary parts at m = 0 are zero.
* grid: per field, ring i = 0 .. 2l-1 (ascending cos(theta)), then the 4l
  equispaced longitudes phi_j = 2 pi j / (4 l).

The coefficient distribution follows the configurations of the transform's
benchmarks: real and imaginary parts i.i.d. N(0, 1), scaled by (1 + k)^-power,
drawn in storage order with numpy's PCG64 generator.
"""
import numpy as np


def degrees_canonical(l, kind="complex"):
    """Degree k of every entry of one field's coefficient vector (int64)."""
    L2 = 2 * l
    parts = []
    for m in range(L2):
        ks = np.arange(m, L2, dtype=np.int64)
        parts.append(ks)
        if kind == "complex" and m > 0:
            parts.append(ks)
    return np.concatenate(parts)


def orders_canonical(l, kind="complex"):
    """Signed order m of every entry of one field's coefficient vector (int64)."""
    L2 = 2 * l
    parts = []
    for m in range(L2):
        n = L2 - m
        parts.append(np.full(n, m, dtype=np.int64))
        if kind == "complex" and m > 0:
            parts.append(np.full(n, -m, dtype=np.int64))
    return np.concatenate(parts)


def n_coeffs(l, kind="complex"):
    return 4 * l * l if kind == "complex" else 2 * l * l + l


def coefficients(l, nfields, seed=0, power=1.0, kind="complex"):
    """Random coefficients, shape (nfields, n_coeffs(l, kind)), complex128."""
    rng = np.random.default_rng(seed)
    n = n_coeffs(l, kind)
    raw = rng.standard_normal((nfields, n, 2))
    beta = raw[..., 0] + 1j * raw[..., 1]
    k = degrees_canonical(l, kind)
    beta *= (1.0 + k) ** (-float(power))
    if kind == "real":
        beta[:, : 2 * l] = beta[:, : 2 * l].real  # m = 0 block is real
    return beta


def grid(l, nfields, seed=0, kind="complex"):
    """Random grid values N(0,1) (complex: both parts), shape (nfields, 2l, 4l)."""
    rng = np.random.default_rng(seed)
    shape = (nfields, 2 * l, 4 * l)
    if kind == "complex":
        raw = rng.standard_normal(shape + (2,))
        return raw[..., 0] + 1j * raw[..., 1]
    return rng.standard_normal(shape)


def unit_vectors(n, count, seed=0):
    """Unit-l2 test vectors with entries uniform on (-1, 1), shape (n, count)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, size=(n, count))
    return v / np.linalg.norm(v, axis=0, keepdims=True)
