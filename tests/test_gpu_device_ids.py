"""The device ID builder (sht_plan_opts.id_device): every interpolative decomposition of the
plan computed on the GPU, level by level for a batch of pairs at once.

Checked three ways: the butterflies it builds (read back through the plan cache as host
trees) against the oracle's dense Q^{(m,p)} with the paper's eps_fwd / eps_inv and the bound
|T| <= 2 of Remark QR_algorithm, block by block, in numpy (no GPU kernel involved); the
transforms of a device-built plan against the oracle; and its statistics against the host
builder's (ranks, factor counts, depth-first memory figure)."""
import numpy as np
import pytest

import oracle
import sht_synthetic as syn
from tests import bf_reference as bfr

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return max(float(np.linalg.norm(a[f] - b[f]) / np.linalg.norm(b[f])) for f in range(a.shape[0]))


@pytest.mark.parametrize("l,C", [(16, 4), (64, 16)])
def test_device_built_butterflies_match_dense_q(tmp_path, l, C):
    from paper_0910_5435_amd import Butterfly, Plan, _lib, plan_cache_check

    eps = 1e-13
    P = Plan(l, eps=eps, leaf_width=C, cache_dir=tmp_path, id_device=True)
    st = P.stats()
    P.close()
    assert plan_cache_check(tmp_path, l, eps, C) == (_lib.SHT_OK, 4 * l)
    worst_f = worst_i = worst_t = 0.0
    for mp in range(4 * l):
        m, p = mp // 2, mp % 2
        Q = oracle.dense_q(l, m, p)
        n = Q.shape[1]
        bf = Butterfly.from_plan_cache(tmp_path, l, eps, C, mp)
        if n == 0:
            continue
        # every block: an ID of its input (skeleton + redundant = all columns), |T| <= 2 except
        # where an exchange would have left the residual above eps
        for t in range(bf.levels + 1):
            for r in range(2 ** t):
                for c in range(2 ** (bf.levels - t)):
                    skel, red, T = bf.block(t, r, c)
                    assert sorted(np.concatenate([skel, red]).tolist()) == list(range(len(skel) + len(red)))
                    if T.size:
                        worst_t = max(worst_t, float(np.max(np.abs(T))))
        X = syn.unit_vectors(n, 4, seed=mp)
        Y = bfr.apply(bf, X)
        worst_f = max(worst_f, float(np.max(np.abs(Y - Q @ X))))
        worst_i = max(worst_i, float(np.max(np.abs(bfr.apply_t(bf, Y) - X))))
    print(f"device IDs l={l} C={C}: eps_fwd {worst_f:.1e}, eps_inv {worst_i:.1e}, max|T| {worst_t:.2f} "
          f"(stats {st['max_abs_t']:.2f}), k_avg {st['k_avg']:.1f}, IDs {st['t_compress_s']:.2f} s", flush=True)
    assert worst_f < 1e-13 and worst_i < 1e-12
    assert worst_t <= 2.5 and abs(worst_t - st["max_abs_t"]) < 1e-12


@pytest.mark.parametrize("l,C,F", [(32, 8, 3), (128, 32, 4)])
def test_device_built_plan_transforms_match_oracle(l, C, F):
    from paper_0910_5435_amd import Plan

    P = Plan(l, eps=1e-13, leaf_width=C, id_device=True)
    beta = syn.coefficients(l, F, seed=3)
    grid = syn.grid(l, F, seed=4)
    es = _rel(P.synth(_dev(beta)).cpu().numpy(), oracle.synth(beta, l))
    ea = _rel(P.analyze(_dev(grid)).cpu().numpy(), oracle.analyze(grid, l))
    print(f"device-built plan l={l} C={C} F={F}: synthesis {es:.2e}, analysis {ea:.2e}", flush=True)
    assert es < FP64_TOL and ea < FP64_TOL
    if 4 * F % 16 == 0:
        ss = _rel(P.synth(_dev(beta), precision="split32").cpu().numpy(), oracle.synth(beta, l))
        assert ss < 1e-9


def test_device_and_host_builders_agree_at_l1024():
    # the benchmark's plan (eps 1e-12, C = 64): same statistics up to pivot ties, and the
    # device-built plan's transforms of the benchmark's shape against the oracle on every order
    # of one field
    from paper_0910_5435_amd import Plan

    l, F = 1024, 16
    host = Plan(l, eps=1e-12, leaf_width=64)
    hs = host.stats()
    host.close()
    torch.cuda.empty_cache()
    dev = Plan(l, eps=1e-12, leaf_width=64, id_device=True)
    ds = dev.stats()
    print(f"l=1024 host: plan {hs['t_total_s']:.1f} s (IDs {hs['t_compress_s']:.1f} s), k_avg {hs['k_avg']:.2f}, "
          f"factors {hs['factor_entries']:.4e}, m_max {hs['m_max_words']}, max|T| {hs['max_abs_t']:.2f}", flush=True)
    print(f"l=1024 device: plan {ds['t_total_s']:.1f} s (columns {ds['t_columns_s']:.1f} s, IDs "
          f"{ds['t_compress_s']:.1f} s), k_avg {ds['k_avg']:.2f}, factors {ds['factor_entries']:.4e}, "
          f"m_max {ds['m_max_words']}, max|T| {ds['max_abs_t']:.2f}", flush=True)
    assert abs(ds["k_avg"] - hs["k_avg"]) < 0.01 * hs["k_avg"]
    assert abs(ds["factor_entries"] - hs["factor_entries"]) < 0.01 * hs["factor_entries"]
    assert ds["k_max"] <= hs["k_max"] + 2 and ds["max_abs_t"] <= 2.5
    beta = syn.coefficients(l, F, seed=0, power=1.5)
    beta[1:] = 0.0
    f_ref = oracle.synth(beta[:1], l, fast=True)
    g = dev.synth(_dev(beta)).cpu().numpy()
    e = float(np.linalg.norm(g[0] - f_ref[0]) / np.linalg.norm(f_ref[0]))
    a = dev.analyze(_dev(np.concatenate([f_ref, np.zeros((F - 1,) + f_ref.shape[1:])]))).cpu().numpy()
    a_ref = oracle.analyze(f_ref, l, fast=True)
    ea = float(np.linalg.norm(a[0] - a_ref[0]) / np.linalg.norm(a_ref[0]))
    print(f"l=1024 device-built plan, every order, one field: synthesis {e:.2e}, analysis {ea:.2e}", flush=True)
    assert e < FP64_TOL and ea < FP64_TOL


def test_device_builder_resumes_an_interrupted_cache(tmp_path):
    # a cache cut after pair 100 (an interrupted build): the device builder takes over at pair
    # 100 and the plan transforms bit for bit like the one built in one go
    from paper_0910_5435_amd import Plan, _lib, plan_cache_check

    l, C, eps, F = 64, 16, 1e-13, 4
    beta = _dev(syn.coefficients(l, F, seed=9))

    def build():
        P = Plan(l, eps=eps, leaf_width=C, cache_dir=tmp_path, id_device=True)
        st = P.stats()
        out = P.synth(beta).cpu().numpy()
        P.close()
        return st, out

    st0, ref = build()
    path = next(p for p in tmp_path.iterdir() if p.suffix == ".cache")
    data = path.read_bytes()
    offs, off = [], 36
    while off < len(data):
        offs.append(off)
        off += 16 + int.from_bytes(data[off + 4:off + 12], "little")
    path.write_bytes(data[:offs[100]])
    st1, got = build()
    assert st0["cache_pairs_loaded"] == 0 and st1["cache_pairs_loaded"] == 100
    assert np.array_equal(got, ref)
    assert plan_cache_check(tmp_path, l, eps, C) == (_lib.SHT_OK, 4 * l)
