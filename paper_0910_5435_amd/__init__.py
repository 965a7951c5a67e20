"""MI355X-native butterfly spherical harmonic transform (Tygert, SHT III).

The compute path lives in ``libsht.so`` (HIP kernels for gfx950 behind a C ABI);
this package only binds it.  Importing the package does not load the library;
the first call that needs it does, and raises ImportError if it was not built.
"""
from .sht import (Batch, Butterfly, OrderPlan, Plan, coeff_index, gauss_jacobi_matrix, gauss_jacobi_rule,
                  gl_nodes, plan_cache_append, plan_cache_check, num_coeffs)

__all__ = ["Plan", "OrderPlan", "Batch", "Butterfly", "coeff_index", "gauss_jacobi_matrix", "gauss_jacobi_rule", "gl_nodes",
           "plan_cache_append", "plan_cache_check",
           "num_coeffs"]
