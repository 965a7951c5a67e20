"""ctypes declarations of the C ABI in include/sht.h (argument marshalling only)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsht.so")

SHT_OK = 0
SHT_EINVAL = -1
SHT_ENOMEM = -2
SHT_EHIP = -3
SHT_EUNSUPPORTED = -4
SHT_EINTERNAL = -5
SHT_ENOTREADY = -6
SHT_ECORRUPT = -7

NOALLOC_SCRATCH_BYTES = 256 << 20  # SHT_NOALLOC_SCRATCH_BYTES of include/sht.h

SHT_FP64 = 0
SHT_SPLIT32 = 1
SHT_FP32 = 2
SHT_INT8 = 3

SHT_COMPLEX = 0
SHT_REAL = 1

SHT_BATCH_SYNTH = 0
SHT_BATCH_ANALYZE = 1
SHT_BATCH_ADJOINT = 2


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("leaf_width", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("field_kind", ctypes.c_int),
        ("host_threads", ctypes.c_int),
        ("device", ctypes.c_int),
        ("split_only", ctypes.c_int),
        ("cache_dir", ctypes.c_char_p),
        ("id_device", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("l", ctypes.c_int),
        ("leaf_width", ctypes.c_int),
        ("max_levels", ctypes.c_int),
        ("k_max", ctypes.c_int),
        ("k_avg", ctypes.c_double),
        ("k_sd", ctypes.c_double),
        ("n_blocks", ctypes.c_longlong),
        ("factor_entries", ctypes.c_longlong),
        ("dense_entries", ctypes.c_longlong),
        ("m_max_words", ctypes.c_longlong),
        ("t_columns_s", ctypes.c_double),
        ("t_compress_s", ctypes.c_double),
        ("t_total_s", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("device_bytes", ctypes.c_longlong),
        ("max_abs_t", ctypes.c_double),
        ("cache_pairs_loaded", ctypes.c_longlong),
        ("cache_rebuilt", ctypes.c_int),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("plan", ctypes.c_void_p),
        ("nfields", ctypes.c_int),
        ("input", ctypes.c_void_p),
        ("output", ctypes.c_void_p),
    ]


class BatchConfig(ctypes.Structure):
    _fields_ = [
        ("column_tile", ctypes.c_int),
        ("wg_per_cu", ctypes.c_int),
        ("queues", ctypes.c_int),
        ("ms", ctypes.c_double),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("groups", ctypes.c_int),
        ("launches", ctypes.c_int),
        ("phases", ctypes.c_int),
        ("items", ctypes.c_longlong),
        ("columns", ctypes.c_longlong),
        ("workspace_bytes", ctypes.c_size_t),
        ("config", BatchConfig),
        ("grid", ctypes.c_int),
    ]


class ShtError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = _lib.sht_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})")


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_S = ctypes.c_size_t
_LL = ctypes.c_longlong
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "sht_default_opts": (None, [ctypes.POINTER(PlanOpts)]),
    "sht_plan": (_I, [_I, _D, ctypes.POINTER(_P)]),
    "sht_plan_ex": (_I, [_I, _D, ctypes.POINTER(PlanOpts), ctypes.POINTER(_P)]),
    "sht_destroy": (None, [_P]),
    "sht_plan_prepare": (_I, [_P, _I, _P]),
    "sht_workspace_bytes": (_S, [_P, _I, _I]),
    "sht_synth": (_I, [_P, _P, _P, _I, _P, _S, _P]),
    "sht_analyze": (_I, [_P, _P, _P, _I, _P, _S, _P]),
    "sht_synth_adjoint": (_I, [_P, _P, _P, _I, _P, _S, _P]),
    "sht_synth_ex": (_I, [_P, _I, _P, _P, _I, _P, _S, _P]),
    "sht_synth_noalloc": (_I, [_P, _P, _P, _I, _P]),
    "sht_analyze_ex": (_I, [_P, _I, _P, _P, _I, _P, _S, _P]),
    "sht_synth_adjoint_ex": (_I, [_P, _I, _P, _P, _I, _P, _S, _P]),
    "sht_plan_stats": (_I, [_P, ctypes.POINTER(Stats)]),
    "sht_batch_create": (_I, [ctypes.POINTER(Request), _I, _I, _I, _S, _P, ctypes.POINTER(_P)]),
    "sht_batch_configure": (_I, [_P, ctypes.POINTER(BatchConfig)]),
    "sht_batch_tune": (_I, [_P, _I, _P, ctypes.POINTER(BatchConfig)]),
    "sht_batch_run": (_I, [_P, _P]),
    "sht_batch_check": (_I, [_P, _P]),
    "sht_batch_get_info": (_I, [_P, ctypes.POINTER(BatchInfo)]),
    "sht_batch_destroy": (None, [_P]),
    "sht_coeff_index": (_LL, [_I, _I, _I, _I]),
    "sht_num_coeffs": (_LL, [_I, _I]),
    "sht_gl_nodes": (_I, [_I, _DP, _DP]),
    "sht_plan_columns": (_I, [_P, _I, _I, _DP, _I]),
    "sht_dense_q": (_I, [_P, _I, _I, _P, _LL, _P]),
    "sht_plan_tree": (_I, [_P, _I, _I, _IP, _IP]),
    "sht_bf_build": (_I, [_DP, _I, _I, _I, _I, _I, _D, ctypes.POINTER(_P)]),
    "sht_bf_destroy": (None, [_P]),
    "sht_plan_cache_check": (_I, [ctypes.c_char_p, _I, _D, _I, ctypes.POINTER(_LL)]),
    "sht_plan_cache_append": (_I, [ctypes.c_char_p, _I, _D, _I, _I, _P]),
    "sht_plan_cache_read": (_I, [ctypes.c_char_p, _I, _D, _I, _I, ctypes.POINTER(_P)]),
    "sht_bf_info": (_I, [_P, _IP, _IP, _DP, _DP, ctypes.POINTER(_LL), ctypes.POINTER(_LL)]),
    "sht_bf_block": (_I, [_P, _I, _I, _I, _IP, _IP, ctypes.POINTER(_IP), ctypes.POINTER(_IP),
                          ctypes.POINTER(_DP)]),
    "sht_bf_final": (_I, [_P, _I, _IP, _IP, _IP, ctypes.POINTER(_DP), ctypes.POINTER(_IP)]),
    "sht_gj_rule": (_I, [_I, _I, _I, _DP, _DP]),
    "sht_gj_matrix": (_I, [_I, _I, _I, _DP, _I]),
    "sht_order_plan": (_I, [_I, _D, ctypes.POINTER(PlanOpts), ctypes.POINTER(_P)]),
    "sht_order_rows": (_LL, [_P]),
    "sht_order_layout": (_I, [_P, _I, _I, ctypes.POINTER(_LL), _IP]),
    "sht_order_workspace_bytes": (_S, [_P, _I]),
    "sht_order_apply": (_I, [_P, _P, _P, _I, _I, _P, _S, _P]),
    "sht_profile_enable": (_I, [_P, _I]),
    "sht_profile_reset": (_I, [_P]),
    "sht_profile_count": (_I, [_P]),
    "sht_profile_get": (_I, [_P, _I, ctypes.POINTER(ctypes.c_char_p), _DP, ctypes.POINTER(_LL), _DP, _DP]),
    "sht_strerror": (ctypes.c_char_p, [_I]),
    "sht_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load the built library; raise ImportError (never fall back) if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_0910_5435_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, what):
    if status != SHT_OK:
        raise ShtError(status, what)
