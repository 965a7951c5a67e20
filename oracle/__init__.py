"""CPU FP64 oracle for the spherical harmonic transform (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with
it; the two meet only on the seeded inputs of ``sht_synthetic``.
"""
from .legendre import gauss_legendre, pbar_orders, pbar_table, step2_coefficients
from .sht import (
    coeff_index,
    n_coeffs,
    phi_points,
    synth,
    analyze,
    synth_adjoint,
    legendre_sums,
    ring_values,
    analyze_orders,
    dense_q,
    folded_sizes,
)

__all__ = [
    "gauss_legendre",
    "pbar_orders",
    "pbar_table",
    "step2_coefficients",
    "coeff_index",
    "n_coeffs",
    "phi_points",
    "synth",
    "analyze",
    "synth_adjoint",
    "legendre_sums",
    "ring_values",
    "analyze_orders",
    "dense_q",
    "folded_sizes",
]
