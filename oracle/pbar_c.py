"""Oracle: ctypes access to the plain-C Legendre table of oracle/pbar.c.

TEST INFRASTRUCTURE.  Same functions and recurrence as ``legendre.pbar_orders`` (the
step-one recurrence from the seeds of equation (association), with exponent tracking),
evaluated node by node in C so that the oracle can sweep every order of the largest
bandlimits.  The library is built by ``oracle/build.py``; without it this module raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbar.so")
_lib = None


def load(path=None):
    """Load the compiled table routine (``path`` overrides the in-tree library)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python oracle/build.py`")
    lib = ctypes.CDLL(p)
    fn = lib.oracle_pbar_table
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                   ctypes.c_void_p]
    if path is None:
        _lib = lib
    return lib


def pbar_table_c(m, x, kmax, lib=None):
    """T[k - m, i] = Pbar_k^m(x_i) for k = m..kmax (C routine; releases the GIL)."""
    lib = lib or load()
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.empty((kmax - m + 1, len(x)))
    if kmax < m:
        return np.zeros((0, len(x)))
    work = np.empty(3 * max(1, len(x)))
    rc = lib.oracle_pbar_table(int(m), int(kmax), x.ctypes.data, len(x), out.ctypes.data, work.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_pbar_table({m}, {kmax}) failed")
    return out


def pbar_orders_c(orders, x, kmax, lib=None):
    """P[a, k, i] = Pbar_k^{m_a}(x_i) for k = 0..kmax (0 where k < m_a): the layout of
    ``legendre.pbar_orders``, filled by the C routine."""
    orders = np.asarray(orders, dtype=np.int64).ravel()
    x = np.asarray(x, dtype=np.float64).ravel()
    out = np.zeros((len(orders), kmax + 1, len(x)))
    for a, m in enumerate(orders):
        if m <= kmax:
            out[a, m:, :] = pbar_table_c(int(m), x, kmax, lib)
    return out
