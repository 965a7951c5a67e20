"""Python binding of the C ABI: plans, transforms on torch device tensors, host helpers.

Every step of the transform runs in the library's HIP kernels; this module only
passes pointers, sizes and the current HIP stream.  PyTorch supplies device
memory and streams.
"""
import ctypes

import numpy as np

from . import _lib as L

PRECISIONS = {"fp64": L.SHT_FP64, "split32": L.SHT_SPLIT32, "fp32": L.SHT_FP32, "int8": L.SHT_INT8}
KINDS = {"complex": L.SHT_COMPLEX, "real": L.SHT_REAL}


def _torch():
    import torch

    return torch


def num_coeffs(l, kind="complex"):
    return int(L.load().sht_num_coeffs(l, KINDS[kind]))


def coeff_index(l, k, m, kind="complex"):
    return int(L.load().sht_coeff_index(l, k, m, KINDS[kind]))


def gl_nodes(n):
    """Host Gauss-Legendre rule computed by the library: (x ascending, w)."""
    lib = L.load()
    x = np.zeros(n)
    w = np.zeros(n)
    L.check(lib.sht_gl_nodes(n, x.ctypes.data_as(L._DP), w.ctypes.data_as(L._DP)), "sht_gl_nodes")
    return x, w


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _used_on(stream, *tensors):
    """Tell torch's caching allocator that tensors it allocated on the current stream are
    used on another stream, so their memory is not handed out again before that work ends."""
    if stream is not None:
        for t in tensors:
            t.record_stream(stream)


class Plan:
    """Butterfly SHT plan for bandlimit l (degrees 0..2l-1) on one GPU."""

    def __init__(self, l, eps=1e-13, leaf_width=64, precision="fp64", kind="complex",
                 host_threads=0, device=None, split_only=False, cache_dir=None, id_device=False):
        lib = L.load()
        opts = L.PlanOpts()
        lib.sht_default_opts(ctypes.byref(opts))
        opts.leaf_width = int(leaf_width)
        opts.precision = PRECISIONS[precision]
        opts.field_kind = KINDS[kind]
        opts.host_threads = int(host_threads)
        opts.split_only = 1 if split_only else 0
        opts.id_device = 1 if id_device else 0
        self._cache_dir = None if cache_dir is None else str(cache_dir).encode()
        opts.cache_dir = self._cache_dir
        if device is None:
            opts.device = -1
        else:
            opts.device = int(device)
        handle = ctypes.c_void_p()
        L.check(lib.sht_plan_ex(int(l), float(eps), ctypes.byref(opts), ctypes.byref(handle)),
                "sht_plan_ex")
        self._h = handle
        self.l = int(l)
        self.eps = float(eps)
        self.kind = kind
        self.precision = precision
        self.leaf_width = int(leaf_width)
        self._ws = {}
        self._prepared = {precision} if split_only else {"fp64", precision}

    def prepare(self, precision, stream=None):
        """Derive the factor copies a split-FP32 / FP32 transform reads (sht_plan_prepare):
        plan-owned device memory; waits for the stream.  The transforms call it on the first
        use of a precision."""
        if precision not in self._prepared:
            L.check(L.load().sht_plan_prepare(self._h, PRECISIONS[precision], _stream_handle(stream)),
                    "sht_plan_prepare")
            self._prepared.add(precision)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().sht_destroy(self._h)
            self._h = None
            self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ info
    @property
    def handle(self):
        return self._h

    def stats(self):
        st = L.Stats()
        L.check(L.load().sht_plan_stats(self._h, ctypes.byref(st)), "sht_plan_stats")
        return {name: getattr(st, name) for name, _ in L.Stats._fields_}

    @property
    def n_coeffs(self):
        return num_coeffs(self.l, self.kind)

    @property
    def grid_shape(self):
        return (2 * self.l, 4 * self.l)

    def profile(self, enable=True):
        L.check(L.load().sht_profile_enable(self._h, 1 if enable else 0), "sht_profile_enable")

    def profile_reset(self):
        L.check(L.load().sht_profile_reset(self._h), "sht_profile_reset")

    def profile_read(self):
        """{stage: {ms, launches, flops, bytes}} accumulated since the last reset."""
        lib = L.load()
        n = lib.sht_profile_count(self._h)
        if n < 0:
            L.check(n, "sht_profile_count")
        out = {}
        for i in range(n):
            name = ctypes.c_char_p()
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            cnt = ctypes.c_longlong()
            L.check(lib.sht_profile_get(self._h, i, ctypes.byref(name), ctypes.byref(ms),
                                        ctypes.byref(cnt), ctypes.byref(fl), ctypes.byref(by)),
                    "sht_profile_get")
            out[name.value.decode()] = {"ms": ms.value, "launches": cnt.value, "flops": fl.value,
                                        "bytes": by.value}
        return out

    def workspace_bytes(self, nfields, precision=None):
        prec = PRECISIONS[precision or self.precision]
        return int(L.load().sht_workspace_bytes(self._h, int(nfields), prec))

    def workspace(self, nfields, precision=None, device=None):
        torch = _torch()
        nb = self.workspace_bytes(nfields, precision)
        key = (nb, str(device))
        ws = self._ws.get(key)
        if ws is None:
            ws = torch.empty(nb + 256, dtype=torch.uint8, device=device or "cuda")
            self._ws = {key: ws}
        return ws

    def columns(self, m, p):
        """Q^{(m,p)} as generated by the device recurrence kernel (host numpy, l x n_p)."""
        lib = L.load()
        lv, nc = ctypes.c_int(), ctypes.c_int()
        L.check(lib.sht_plan_tree(self._h, m, p, ctypes.byref(lv), ctypes.byref(nc)), "sht_plan_tree")
        q = np.zeros((nc.value, self.l))  # column-major l x n
        if nc.value:
            L.check(lib.sht_plan_columns(self._h, m, p, q.ctypes.data_as(L._DP), self.l),
                    "sht_plan_columns")
        return q.T.copy()

    def dense_q(self, out, mp0=0, count=None, stream=None):
        """Dense Q^{(m,p)} of pairs mp0.. into the device tensor out (pairs, l, l) float64:
        out[i] holds pair mp0 + i column-major (out[i][j] = column j); untouched past n_p."""
        torch = _torch()
        if count is None:
            count = out.shape[0]
        if out.dtype != torch.float64 or not out.is_cuda or out.dim() != 3 or \
                tuple(out.shape[1:]) != (self.l, self.l) or not out.is_contiguous() or out.shape[0] < count:
            raise ValueError("out must be a contiguous float64 device tensor (pairs, l, l)")
        L.check(L.load().sht_dense_q(self._h, int(mp0), int(count), ctypes.c_void_p(out.data_ptr()),
                                     self.l * self.l, _stream_handle(stream)), "sht_dense_q")
        return out

    def tree(self, m, p):
        lib = L.load()
        lv, nc = ctypes.c_int(), ctypes.c_int()
        L.check(lib.sht_plan_tree(self._h, m, p, ctypes.byref(lv), ctypes.byref(nc)), "sht_plan_tree")
        return lv.value, nc.value

    # ------------------------------------------------------------------ transforms
    def _check_tensor(self, t, shape_tail, complex_ok, name):
        torch = _torch()
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        want = torch.complex128 if complex_ok else torch.float64
        if t.dtype != want:
            raise ValueError(f"{name} must be {want}, got {t.dtype}")
        if tuple(t.shape[1:]) != tuple(shape_tail):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (F,) + {shape_tail}")

    def _grid_complex(self):
        return self.kind == "complex"

    def synth(self, coeff, out=None, precision=None, stream=None):
        """coeff: complex128 (F, n_coeffs) on the device -> grid (F, 2l, 4l).

        stream (a torch stream; default the current one) is where the kernels run.  Calls on
        one plan share its cached workspace, so calls on different streams must be ordered
        by the caller."""
        torch = _torch()
        if coeff.dim() == 1:
            coeff = coeff.unsqueeze(0)
        self._check_tensor(coeff, (self.n_coeffs,), True, "coeff")
        F = coeff.shape[0]
        if out is None:
            dt = torch.complex128 if self._grid_complex() else torch.float64
            out = torch.empty((F,) + self.grid_shape, dtype=dt, device=coeff.device)
        self._check_tensor(out, self.grid_shape, self._grid_complex(), "grid")
        self.prepare(precision or self.precision, stream)
        prec = PRECISIONS[precision or self.precision]
        ws = self.workspace(F, precision, coeff.device)
        _used_on(stream, ws, out)
        L.check(L.load().sht_synth_ex(self._h, prec, ctypes.c_void_p(coeff.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), F,
                                      ctypes.c_void_p(_align(ws.data_ptr())), ws.numel() - 256,
                                      _stream_handle(stream)), "sht_synth")
        return out

    def _transposed(self, fn, grid, out, precision, stream, what):
        torch = _torch()
        if grid.dim() == 2:
            grid = grid.unsqueeze(0)
        self._check_tensor(grid, self.grid_shape, self._grid_complex(), "grid")
        F = grid.shape[0]
        if out is None:
            out = torch.empty((F, self.n_coeffs), dtype=torch.complex128, device=grid.device)
        self._check_tensor(out, (self.n_coeffs,), True, "coeff")
        self.prepare(precision or self.precision, stream)
        prec = PRECISIONS[precision or self.precision]
        ws = self.workspace(F, precision, grid.device)
        _used_on(stream, ws, out)
        L.check(fn(self._h, prec, ctypes.c_void_p(grid.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                   F, ctypes.c_void_p(_align(ws.data_ptr())), ws.numel() - 256,
                   _stream_handle(stream)), what)
        return out

    def analyze(self, grid, out=None, precision=None, stream=None):
        """grid (F, 2l, 4l) -> coefficients (F, n_coeffs); exact inverse of synth."""
        return self._transposed(L.load().sht_analyze_ex, grid, out, precision, stream, "sht_analyze")

    def synth_adjoint(self, grid_cot, out=None, precision=None, stream=None):
        """Adjoint of synth (real inner products): the backward of synthesis."""
        return self._transposed(L.load().sht_synth_adjoint_ex, grid_cot, out, precision, stream,
                                "sht_synth_adjoint")


def _align(ptr):
    return (ptr + 255) & ~255


class OrderPlan:
    """The per-order maps of Section 5 on the GPU (sht_order_plan): for every order m < 2l and
    parity p, the orthogonal n_p x n_p matrix A^{(m,p)} of (transform) / (transform2) on its own
    Gauss-Jacobi-type nodes, butterfly-compressed.  Vectors live in "pair rows": an
    (rows, R) float64 device array in which pair 2m + p owns rows [row0, row0 + n_p)."""

    def __init__(self, l, eps=1e-13, leaf_width=64, host_threads=0, device=None):
        lib = L.load()
        opts = L.PlanOpts()
        lib.sht_default_opts(ctypes.byref(opts))
        opts.leaf_width = int(leaf_width)
        opts.host_threads = int(host_threads)
        opts.device = -1 if device is None else int(device)
        handle = ctypes.c_void_p()
        L.check(lib.sht_order_plan(int(l), float(eps), ctypes.byref(opts), ctypes.byref(handle)),
                "sht_order_plan")
        self._h = handle
        self.l = int(l)
        self.eps = float(eps)
        self.leaf_width = int(leaf_width)
        self.rows = int(lib.sht_order_rows(handle))
        self._ws = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().sht_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def stats(self):
        st = L.Stats()
        L.check(L.load().sht_plan_stats(self._h, ctypes.byref(st)), "sht_plan_stats")
        return {name: getattr(st, name) for name, _ in L.Stats._fields_}

    def layout(self, m, p):
        """(row0, n_p) of pair (m, p)."""
        r0, n = ctypes.c_longlong(), ctypes.c_int()
        L.check(L.load().sht_order_layout(self._h, int(m), int(p), ctypes.byref(r0), ctypes.byref(n)),
                "sht_order_layout")
        return r0.value, n.value

    def profile(self, enable=True):
        L.check(L.load().sht_profile_enable(self._h, 1 if enable else 0), "sht_profile_enable")

    profile_reset = Plan.profile_reset
    profile_read = Plan.profile_read

    def apply(self, x, out=None, transpose=False, stream=None):
        """out = A x (coefficients -> node values) for every pair, or A^T x with transpose=True
        (the inverse).  x: float64 (rows, R) or (rows,) on the device, contiguous."""
        torch = _torch()
        squeeze = x.dim() == 1
        if squeeze:
            x = x.unsqueeze(1)
        if not x.is_cuda or not x.is_contiguous() or x.dtype != torch.float64 or x.shape[0] != self.rows:
            raise ValueError(f"x must be a contiguous float64 device tensor with {self.rows} rows")
        R = x.shape[1]
        if out is None:
            out = torch.empty_like(x)
        elif out.shape != x.shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor shaped like x")
        nb = int(L.load().sht_order_workspace_bytes(self._h, int(R)))
        if self._ws is None or self._ws.numel() < nb + 256 or self._ws.device != x.device:
            self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=x.device)
        _used_on(stream, self._ws, out)
        L.check(L.load().sht_order_apply(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         int(R), 1 if transpose else 0, ctypes.c_void_p(_align(self._ws.data_ptr())),
                                         self._ws.numel() - 256, _stream_handle(stream)), "sht_order_apply")
        return out[:, 0] if squeeze else out


BATCH_OPS = {"synth": L.SHT_BATCH_SYNTH, "analyze": L.SHT_BATCH_ANALYZE, "adjoint": L.SHT_BATCH_ADJOINT}


class Batch:
    """Many requests (plan, input, output) run by one persistent launch replayed from a graph.

    op: "synth" (coefficients -> grid), "analyze" or "adjoint" (grid -> coefficients).
    Inputs and outputs are device tensors in the plan's layouts with a leading field axis;
    the batch keeps references to them (their addresses are baked into the graph).  The
    plans must outlive the batch.
    """

    def __init__(self, requests, op="synth", precision="fp64", workspace_limit=0, stream=None):
        lib = L.load()
        self.op = op
        self.precision = precision
        self._keep = []
        arr = (L.Request * len(requests))()
        for i, (plan, inp, out) in enumerate(requests):
            if op == "synth":
                plan._check_tensor(inp, (plan.n_coeffs,), True, "coeff")
                plan._check_tensor(out, plan.grid_shape, plan._grid_complex(), "grid")
            else:
                plan._check_tensor(inp, plan.grid_shape, plan._grid_complex(), "grid")
                plan._check_tensor(out, (plan.n_coeffs,), True, "coeff")
            if inp.shape[0] != out.shape[0]:
                raise ValueError("input and output field counts differ")
            arr[i].plan = plan.handle
            arr[i].nfields = int(inp.shape[0])
            arr[i].input = inp.data_ptr()
            arr[i].output = out.data_ptr()
            self._keep.append((plan, inp, out))
        h = ctypes.c_void_p()
        L.check(lib.sht_batch_create(arr, len(requests), BATCH_OPS[op], PRECISIONS[precision],
                                     int(workspace_limit), _stream_handle(stream), ctypes.byref(h)),
                "sht_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            L.load().sht_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, stream=None):
        L.check(L.load().sht_batch_run(self._h, _stream_handle(stream)), "sht_batch_run")

    def check(self, stream=None):
        """Wait for the stream and raise if the last run's persistent kernel gave up."""
        L.check(L.load().sht_batch_check(self._h, _stream_handle(stream)), "sht_batch_check")

    def configure(self, column_tile=0, wg_per_cu=0, queues=0):
        c = L.BatchConfig(column_tile, wg_per_cu, queues, 0.0)
        L.check(L.load().sht_batch_configure(self._h, ctypes.byref(c)), "sht_batch_configure")

    def tune(self, reps=3, stream=None):
        """Autotune tile, residency and queue layout; returns the chosen configuration."""
        c = L.BatchConfig()
        L.check(L.load().sht_batch_tune(self._h, int(reps), _stream_handle(stream), ctypes.byref(c)),
                "sht_batch_tune")
        return {"column_tile": c.column_tile, "wg_per_cu": c.wg_per_cu, "queues": c.queues, "ms": c.ms}

    def info(self):
        i = L.BatchInfo()
        L.check(L.load().sht_batch_get_info(self._h, ctypes.byref(i)), "sht_batch_get_info")
        return {"groups": i.groups, "launches": i.launches, "phases": i.phases, "items": i.items,
                "columns": i.columns, "workspace_bytes": i.workspace_bytes, "grid": i.grid,
                "config": {"column_tile": i.config.column_tile, "wg_per_cu": i.config.wg_per_cu,
                           "queues": i.config.queues}}


def plan_cache_check(cache_dir, l, eps, leaf_width=64):
    """(status, intact leading records) of the plan cache file of (l, eps, leaf_width):
    status 0 (every record present intact), SHT_ECORRUPT or SHT_EINVAL (no file); host only."""
    n = ctypes.c_longlong()
    rc = L.load().sht_plan_cache_check(str(cache_dir).encode(), int(l), float(eps), int(leaf_width), ctypes.byref(n))
    return rc, n.value


def plan_cache_append(cache_dir, l, eps, leaf_width, mp, butterfly):
    """Append a host-built Butterfly of pair mp = 2m + p as the next plan cache record."""
    L.check(L.load().sht_plan_cache_append(str(cache_dir).encode(), int(l), float(eps), int(leaf_width), int(mp),
                                           butterfly._h), "sht_plan_cache_append")


def gauss_jacobi_rule(m, n, parity=0):
    """Nodes x (ascending, positive) and weights lambda = rho (1 - x^2)^m (parity 0) or
    sigma (1 - x^2)^m (parity 1) of the per-order quadratures of Section 3.3 (Lemma
    quadratures); host only."""
    lib = L.load()
    x = np.empty(int(n))
    w = np.empty(int(n))
    L.check(lib.sht_gj_rule(int(m), int(n), int(parity), x.ctypes.data_as(L._DP), w.ctypes.data_as(L._DP)),
            "sht_gj_rule")
    return x, w


def gauss_jacobi_matrix(m, n, parity=0):
    """The n x n orthogonal matrix of equation (transform) (parity 0) or (transform2)
    (parity 1): A[i, j] = sqrt(w_i) Pbar^m_{m+parity+2j}(x_i); host only."""
    lib = L.load()
    a = np.empty((int(n), int(n)), order="F")
    L.check(lib.sht_gj_matrix(int(m), int(n), int(parity), a.ctypes.data_as(L._DP), int(n)), "sht_gj_matrix")
    return a


class Butterfly:
    """Host-only multilevel ID of a dense matrix (Section 3.2 built per Section 4)."""

    def __init__(self, a, leaf_width, eps, levels=-1):
        lib = L.load()
        a = np.asfortranarray(np.asarray(a, dtype=np.float64))
        rows, cols = a.shape
        self._a = a
        h = ctypes.c_void_p()
        L.check(lib.sht_bf_build(a.ctypes.data_as(L._DP), rows, cols, rows, int(leaf_width),
                                 int(levels), float(eps), ctypes.byref(h)), "sht_bf_build")
        self._h = h
        self.rows, self.cols, self.C = rows, cols, int(leaf_width)
        self._read_info()

    @classmethod
    def from_plan_cache(cls, cache_dir, l, eps, leaf_width, mp):
        """The butterfly of pair mp = 2m + p read back from a plan cache file (host only)."""
        h = ctypes.c_void_p()
        L.check(L.load().sht_plan_cache_read(str(cache_dir).encode(), int(l), float(eps), int(leaf_width), int(mp),
                                             ctypes.byref(h)), "sht_plan_cache_read")
        self = cls.__new__(cls)
        self._h = h
        self._a = None
        self.C = int(leaf_width)
        self.rows = int(l)
        m, n = mp // 2, 2 * int(l) - mp // 2
        self.cols = (n + 1) // 2 if mp % 2 == 0 else n // 2
        self._read_info()
        return self

    def _read_info(self):
        lib = L.load()
        h = self._h
        lv, km = ctypes.c_int(), ctypes.c_int()
        ka, ks = ctypes.c_double(), ctypes.c_double()
        fe, mm = ctypes.c_longlong(), ctypes.c_longlong()
        L.check(lib.sht_bf_info(h, ctypes.byref(lv), ctypes.byref(km), ctypes.byref(ka),
                                ctypes.byref(ks), ctypes.byref(fe), ctypes.byref(mm)), "sht_bf_info")
        self.levels = lv.value
        self.k_max = km.value
        self.k_avg = ka.value
        self.k_sd = ks.value
        self.factor_entries = fe.value
        self.m_max_words = mm.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().sht_bf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def block(self, t, r, c):
        """(skel, red, T) with T of shape (k, K - k): w = in[skel] + T @ in[red]."""
        lib = L.load()
        k, K = ctypes.c_int(), ctypes.c_int()
        sp, rp, tp = L._IP(), L._IP(), L._DP()
        L.check(lib.sht_bf_block(self._h, t, r, c, ctypes.byref(k), ctypes.byref(K),
                                 ctypes.byref(sp), ctypes.byref(rp), ctypes.byref(tp)), "sht_bf_block")
        k, K = k.value, K.value
        skel = np.ctypeslib.as_array(sp, shape=(k,)).copy() if k else np.zeros(0, dtype=np.int32)
        red = np.ctypeslib.as_array(rp, shape=(K - k,)).copy() if K - k else np.zeros(0, dtype=np.int32)
        if k and K - k:
            T = np.ctypeslib.as_array(tp, shape=(K - k, k)).T.copy()
        else:
            T = np.zeros((k, K - k))
        return skel, red, T

    def final(self, r):
        """(row0, S, cols): rows [row0, row0 + h) = S @ w_{L, r}."""
        lib = L.load()
        row0, h, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        sp, cp = L._DP(), L._IP()
        L.check(lib.sht_bf_final(self._h, r, ctypes.byref(row0), ctypes.byref(h), ctypes.byref(k),
                                 ctypes.byref(sp), ctypes.byref(cp)), "sht_bf_final")
        h, k = h.value, k.value
        S = np.ctypeslib.as_array(sp, shape=(k, h)).T.copy() if h and k else np.zeros((h, k))
        cols = np.ctypeslib.as_array(cp, shape=(k,)).copy() if k else np.zeros(0, dtype=np.int32)
        return row0.value, S, cols
