"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Error metric: relative l2 over the whole output array of each field; FP64 gate 1e-11.
"""
import numpy as np
import pytest

import oracle
import sht_synthetic as syn

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11


def _plan(l, C=64, eps=1e-13, kind="complex", precision="fp64"):
    from paper_0910_5435_amd import Plan

    return Plan(l, eps=eps, leaf_width=C, kind=kind, precision=precision)


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    F = a.shape[0]
    out = []
    for f in range(F):
        den = np.linalg.norm(b[f])
        out.append(np.linalg.norm(a[f] - b[f]) / (den if den > 0 else 1.0))
    return np.array(out)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# Tolerance on Q entries: the oracle's own step-one recurrence loses ~1e-10 relative on
# Pbar near x = 1 at degree ~2000 (measured against exact-series values), i.e. ~3e-13
# after the sqrt(2 w) ~ 2e-3 row factor; at l <= 256 both sides agree to ~1e-14.
@pytest.mark.parametrize("l,C,orders,tol", [(32, 8, None, 2e-14), (256, 64, [0, 1, 77, 255, 256, 400, 510, 511], 1e-13),
                                            (1024, 64, [0, 775, 1500, 2047], 1e-12)])
def test_column_kernel_matches_oracle(l, C, orders, tol):
    P = _plan(l, C)
    if orders is None:
        orders = range(2 * l)
    worst = 0.0
    for m in orders:
        for p in (0, 1):
            q = P.columns(m, p)
            ref = oracle.dense_q(l, m, p)
            assert q.shape == ref.shape
            if ref.size:
                err = np.max(np.abs(q - ref))
                worst = max(worst, err)
                assert err < tol, (m, p, err)
    print(f"columns l={l}: max abs diff vs oracle {worst:.3e}")


# F % 4 == 0 selects the FP64 matrix-core kernels (R = 4F a multiple of 16), the rest the
# vector kernels; the column tile is 64, 32 or 16 wide depending on R.
@pytest.mark.parametrize("l,C,F", [(32, 8, 1), (32, 8, 3), (256, 64, 1), (64, 16, 5),
                                   (64, 16, 4), (128, 32, 8), (256, 64, 16)])
def test_synth_matches_oracle(l, C, F):
    P = _plan(l, C)
    beta = syn.coefficients(l, F, seed=0, power=1.0)
    ref = oracle.synth(beta, l)
    got = P.synth(_dev(beta)).cpu().numpy()
    torch.cuda.synchronize()
    err = _rel(got, ref)
    print(f"synth l={l} C={C} F={F} rel_l2 max={err.max():.3e}")
    assert err.max() < FP64_TOL


@pytest.mark.parametrize("l,C,F", [(32, 8, 1), (32, 8, 3), (256, 64, 1), (64, 16, 5),
                                   (64, 16, 4), (128, 32, 8), (256, 64, 16)])
def test_analyze_matches_oracle(l, C, F):
    P = _plan(l, C)
    g = syn.grid(l, F, seed=1)  # any grid: analysis is a linear map on all of them
    ref = oracle.analyze(g, l)
    got = P.analyze(_dev(g)).cpu().numpy()
    err = _rel(got, ref)
    print(f"analyze l={l} C={C} F={F} rel_l2 max={err.max():.3e}")
    assert err.max() < FP64_TOL


@pytest.mark.parametrize("l,C,F", [(32, 8, 2), (128, 32, 1), (64, 16, 4)])
def test_adjoint_matches_oracle(l, C, F):
    P = _plan(l, C)
    r = syn.grid(l, F, seed=2)
    ref = oracle.synth_adjoint(r, l)
    got = P.synth_adjoint(_dev(r)).cpu().numpy()
    err = _rel(got, ref)
    assert err.max() < FP64_TOL


@pytest.mark.parametrize("l,C", [(1, 64), (2, 1), (4, 2), (8, 64), (16, 4)])
def test_tiny_bandlimits(l, C):
    P = _plan(l, C)
    beta = syn.coefficients(l, 2, seed=l)
    ref = oracle.synth(beta, l)
    got = P.synth(_dev(beta)).cpu().numpy()
    assert _rel(got, ref).max() < FP64_TOL
    back = P.analyze(_dev(ref)).cpu().numpy()
    assert _rel(back, beta).max() < FP64_TOL


def test_worked_example_l1_on_gpu():
    import json, os

    here = os.path.dirname(os.path.abspath(__file__))
    g = json.load(open(os.path.join(here, "golden", "l1_worked_example.json")))
    P = _plan(1, 64)
    for case in g["cases"]:
        beta = np.zeros((1, 4), dtype=complex)
        beta[0, oracle.coeff_index(1, case["k"], case["m"])] = 1.0
        ref = np.array(case["grid_re"]) + 1j * np.array(case["grid_im"])
        got = P.synth(_dev(beta)).cpu().numpy()[0]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("l,C,F", [(32, 8, 2), (128, 64, 1), (64, 16, 8)])
def test_real_fields(l, C, F):
    P = _plan(l, C, kind="real")
    beta = syn.coefficients(l, F, seed=4, kind="real")
    ref = oracle.synth(beta, l, kind="real")
    got = P.synth(_dev(beta)).cpu().numpy()
    assert _rel(got, ref).max() < FP64_TOL
    back = P.analyze(_dev(ref)).cpu().numpy()
    assert _rel(back, beta).max() < FP64_TOL
    r = syn.grid(l, F, seed=5, kind="real")
    adj = P.synth_adjoint(_dev(r)).cpu().numpy()
    assert _rel(adj, oracle.synth_adjoint(r, l, kind="real")).max() < FP64_TOL


def test_round_trip_gpu_only():
    l, C, F = 128, 32, 4
    P = _plan(l, C)
    beta = _dev(syn.coefficients(l, F, seed=8))
    back = P.analyze(P.synth(beta))
    err = _rel(back.cpu().numpy(), beta.cpu().numpy())
    assert err.max() < FP64_TOL


# --------------------------------------------------------------------- precision variants
# split: FP64 operands cut into an exactly-multiplied leading slice plus an FP32 remainder
# on the FP32 matrix cores, accumulated in FP64 every four K-steps (gate 1e-9); FP32: plain
# single precision (error reported, loose sanity bound only).
SPLIT_TOL = 1e-9


@pytest.mark.parametrize("l,C,F", [(64, 16, 4), (128, 32, 8), (256, 64, 16)])
def test_split_precision_matches_oracle(l, C, F):
    P = _plan(l, C, eps=1e-12)
    beta = syn.coefficients(l, F, seed=0, power=1.5)
    ref = oracle.synth(beta, l)
    got = P.synth(_dev(beta), precision="split32").cpu().numpy()
    es = _rel(got, ref)
    g = syn.grid(l, F, seed=1)
    ga = P.analyze(_dev(g), precision="split32").cpu().numpy()
    ea = _rel(ga, oracle.analyze(g, l))
    f32 = P.synth(_dev(beta), precision="fp32").cpu().numpy()
    e32 = _rel(f32, ref)
    print(f"split l={l} F={F}: synth {es.max():.2e} analysis {ea.max():.2e}; fp32 synth {e32.max():.2e}")
    assert es.max() < SPLIT_TOL and ea.max() < SPLIT_TOL
    assert e32.max() < 1e-4


# int8-slice form: FP64 operands as five 8-bit fixed-point digits on the int8 matrix cores,
# exact int32 sums combined in FP64; the same 1e-9 gate as the split form.
INT8_TOL = 1e-9


@pytest.mark.parametrize("l,C,F", [(64, 16, 4), (128, 32, 8), (256, 64, 16), (64, 8, 12)])
def test_int8_matches_oracle(l, C, F):
    P = _plan(l, C, eps=1e-12)
    beta = syn.coefficients(l, F, seed=0, power=1.5)
    es = _rel(P.synth(_dev(beta), precision="int8").cpu().numpy(), oracle.synth(beta, l))
    g = syn.grid(l, F, seed=1)
    ea = _rel(P.analyze(_dev(g), precision="int8").cpu().numpy(), oracle.analyze(g, l))
    r = syn.grid(l, F, seed=2)
    ej = _rel(P.synth_adjoint(_dev(r), precision="int8").cpu().numpy(), oracle.synth_adjoint(r, l))
    print(f"int8 l={l} C={C} F={F}: synth {es.max():.2e} analysis {ea.max():.2e} adjoint {ej.max():.2e}")
    assert es.max() < INT8_TOL and ea.max() < INT8_TOL and ej.max() < INT8_TOL


def test_int8_real_fields_and_plan_default():
    from paper_0910_5435_amd import Plan

    l, C, F = 64, 16, 8
    P = Plan(l, eps=1e-12, leaf_width=C, kind="real", precision="int8")
    beta = syn.coefficients(l, F, seed=3, kind="real", power=1.5)
    ref = oracle.synth(beta, l, kind="real")
    assert _rel(P.synth(_dev(beta)).cpu().numpy(), ref).max() < INT8_TOL
    assert _rel(P.analyze(_dev(ref)).cpu().numpy(), beta).max() < INT8_TOL
    r = syn.grid(l, F, seed=4, kind="real")
    assert _rel(P.synth_adjoint(_dev(r)).cpu().numpy(), oracle.synth_adjoint(r, l, kind="real")).max() < INT8_TOL


def test_prepare_and_split_only_plans():
    # A split-FP32 transform needs the split copies of the factors: SHT_ENOTREADY until
    # sht_plan_prepare derived them (the transforms themselves never allocate).  A split-only
    # plan frees its FP64 copies: FP64 transforms on it are refused, split ones match the oracle.
    import ctypes

    from paper_0910_5435_amd import Plan, _lib

    lib = _lib.load()
    l, C, F = 64, 16, 4
    P = _plan(l, C, eps=1e-12)
    beta = _dev(syn.coefficients(l, F, seed=0, power=1.5))
    grid = torch.empty((F, 2 * l, 4 * l), dtype=torch.complex128, device="cuda")
    ws = P.workspace(F)
    wp = (ws.data_ptr() + 255) & ~255

    def call(plan, prec):
        rc = lib.sht_synth_ex(plan.handle, prec, ctypes.c_void_p(beta.data_ptr()),
                              ctypes.c_void_p(grid.data_ptr()), F, ctypes.c_void_p(wp), ws.numel() - 256, None)
        torch.cuda.synchronize()
        return rc

    assert call(P, _lib.SHT_SPLIT32) == _lib.SHT_ENOTREADY
    assert call(P, _lib.SHT_INT8) == _lib.SHT_ENOTREADY
    assert lib.sht_plan_prepare(P.handle, _lib.SHT_SPLIT32, None) == _lib.SHT_OK
    assert call(P, _lib.SHT_INT8) == _lib.SHT_ENOTREADY
    assert lib.sht_plan_prepare(P.handle, _lib.SHT_INT8, None) == _lib.SHT_OK
    assert call(P, _lib.SHT_INT8) == _lib.SHT_OK
    assert call(P, _lib.SHT_SPLIT32) == _lib.SHT_OK
    ref = oracle.synth(beta.cpu().numpy(), l)
    assert _rel(grid.cpu().numpy(), ref).max() < SPLIT_TOL
    S = Plan(l, eps=1e-12, leaf_width=C, precision="split32", split_only=True)
    assert S.stats()["device_bytes"] < P.stats()["device_bytes"]
    assert call(S, _lib.SHT_FP64) == _lib.SHT_ENOTREADY
    assert lib.sht_plan_prepare(S.handle, _lib.SHT_FP64, None) == _lib.SHT_ENOTREADY
    assert _rel(S.synth(beta, precision="split32").cpu().numpy(), ref).max() < SPLIT_TOL
    with pytest.raises(_lib.ShtError) as ei:
        Plan(l, eps=1e-12, leaf_width=C, precision="fp64", split_only=True)
    assert ei.value.status == _lib.SHT_EINVAL


def test_plan_cache_round_trip_resume_and_rebuild(tmp_path):
    # A plan built with a cache directory writes every pair's butterfly; the next plan reads
    # them all back and transforms bit for bit like the first; a cache cut at a record boundary
    # resumes there, and one with a flipped byte is cut at that record and rebuilt.
    from paper_0910_5435_amd import Plan, _lib, plan_cache_check

    l, C, eps, F = 64, 16, 1e-13, 4
    npairs = 4 * l
    beta = _dev(syn.coefficients(l, F, seed=9))
    grid = _dev(syn.grid(l, F, seed=10))

    def build():
        P = Plan(l, eps=eps, leaf_width=C, cache_dir=tmp_path)
        st = P.stats()
        out = (P.synth(beta).cpu().numpy(), P.analyze(grid).cpu().numpy())
        P.close()
        return st, out

    st0, ref = build()
    assert st0["cache_pairs_loaded"] == 0 and st0["cache_rebuilt"] == 0
    assert plan_cache_check(tmp_path, l, eps, C) == (_lib.SHT_OK, npairs)
    st1, got = build()
    assert st1["cache_pairs_loaded"] == npairs and st1["factor_entries"] == st0["factor_entries"]
    assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    path = next(p for p in tmp_path.iterdir() if p.suffix == ".cache")
    data = bytearray(path.read_bytes())
    offs, off = [], 36
    while off < len(data):
        offs.append(off)
        off += 16 + int.from_bytes(data[off + 4:off + 12], "little")
    path.write_bytes(bytes(data[:offs[100]]))  # an interrupted build: 100 pairs done
    st2, got = build()
    assert st2["cache_pairs_loaded"] == 100 and st2["cache_rebuilt"] == 0
    assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    assert plan_cache_check(tmp_path, l, eps, C) == (_lib.SHT_OK, npairs)
    data = bytearray(path.read_bytes())
    data[offs[37] + 40] ^= 0x04
    path.write_bytes(bytes(data))
    assert plan_cache_check(tmp_path, l, eps, C) == (_lib.SHT_ECORRUPT, 37)
    st3, got = build()
    assert st3["cache_pairs_loaded"] == 37 and st3["cache_rebuilt"] == 1
    assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    assert plan_cache_check(tmp_path, l, eps, C) == (_lib.SHT_OK, npairs)


def test_split_precision_real_fields_and_adjoint():
    l, C, F = 64, 16, 8
    P = _plan(l, C, eps=1e-12, kind="real")
    beta = syn.coefficients(l, F, seed=3, kind="real", power=1.5)
    got = P.synth(_dev(beta), precision="split32").cpu().numpy()
    assert _rel(got, oracle.synth(beta, l, kind="real")).max() < SPLIT_TOL
    r = syn.grid(l, F, seed=4, kind="real")
    adj = P.synth_adjoint(_dev(r), precision="split32").cpu().numpy()
    assert _rel(adj, oracle.synth_adjoint(r, l, kind="real")).max() < SPLIT_TOL


_MAG_CASE = {}


@pytest.mark.parametrize("scale", [1e-60, 1e-20, 1e20, 1e60])
def test_split_precision_any_magnitude(scale):
    # the split slices of the vectors live on their columns' grids as integers plus a bounded
    # FP32 remainder, so fields far outside FP32's range transform as well as unit ones (the
    # oracle's map is linear: its output for the scaled input is the scaled output); l = 256
    # with C = 64 gives final blocks of more than 128 rows, which the analysis takes in two
    # chunks with grids of their own
    l, C, F = 256, 64, 4
    P = _plan(l, C, eps=1e-12)
    if not _MAG_CASE:
        beta = syn.coefficients(l, F, seed=5, power=1.5)
        grid = syn.grid(l, F, seed=6)
        _MAG_CASE.update(beta=beta, grid=grid, ref_s=oracle.synth(beta, l), ref_a=oracle.analyze(grid, l))
    beta, grid, ref_s, ref_a = (_MAG_CASE[k] for k in ("beta", "grid", "ref_s", "ref_a"))
    got_s = P.synth(_dev(beta * scale), precision="split32").cpu().numpy() / scale
    got_a = P.analyze(_dev(grid * scale), precision="split32").cpu().numpy() / scale
    es, ea = _rel(got_s, ref_s).max(), _rel(got_a, ref_a).max()
    print(f"split at scale {scale:g}: synthesis {es:.2e}, analysis {ea:.2e}", flush=True)
    assert es < SPLIT_TOL and ea < SPLIT_TOL


def test_split_precision_needs_matrix_core_widths():
    from paper_0910_5435_amd import _lib

    P = _plan(32, 8)
    beta = _dev(syn.coefficients(32, 1, seed=0))
    with pytest.raises(_lib.ShtError) as ei:
        P.synth(beta, precision="split32")
    assert ei.value.status == _lib.SHT_EUNSUPPORTED


def test_dense_q_export_matches_oracle():
    # the comparison baseline's dense matrices come from the same column kernel
    l = 16
    P = _plan(l, 4)
    Q = torch.zeros((4 * l, l, l), dtype=torch.float64, device="cuda")
    P.dense_q(Q)
    Qh = Q.cpu().numpy()
    for mp in range(4 * l):
        m, p = mp // 2, mp % 2
        ref = oracle.dense_q(l, m, p)  # l x n_p
        n = ref.shape[1]
        np.testing.assert_allclose(Qh[mp][:n].T, ref, rtol=0, atol=2e-14)
        assert np.all(Qh[mp][n:] == 0)


_STAGED_SCRIPT = r"""
import sys
import numpy as np
import torch
import sht_synthetic as syn
from paper_0910_5435_amd import Plan

l, C, F = 256, 64, 16
P = Plan(l, eps=1e-12, leaf_width=C, precision="split32")
grid = torch.from_numpy(syn.grid(l, F, seed=21)).to("cuda")
np.save(sys.argv[1], P.analyze(grid, precision="split32").cpu().numpy())
"""


def test_split_staged_vectors_match_global_reads(tmp_path):
    # the split transposed levels read their vectors from global memory by default; the
    # staged form (SHT_SPLIT_WLDS_KB, read once per process, so it runs in a child process)
    # adds the same terms in an order that cannot change the result: bit-identical output
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = {}
    for cap in ("0", "76"):
        env = dict(os.environ, SHT_SPLIT_WLDS_KB=cap, PYTHONPATH=root)
        path = tmp_path / f"a{cap}.npy"
        r = subprocess.run([sys.executable, "-c", _STAGED_SCRIPT, str(path)], env=env, cwd=root,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        outs[cap] = np.load(path)
    assert np.array_equal(outs["0"], outs["76"])
    l, F = 256, 16
    ref = oracle.analyze(syn.grid(l, F, seed=21), l)
    assert _rel(outs["0"], ref).max() < SPLIT_TOL
