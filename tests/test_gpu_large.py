"""GPU parity at the largest sizes: the benchmark's batch on every order, bandlimit 2048, and the
mixed-request workload at its own bandlimits.  Everything runs through the C ABI and is compared
with the CPU oracle (relative l2 per field; FP64 gate 1e-11, split-FP32 and int8-slice gate 1e-9).

The tests of this module share their plans (an l = 2048 plan takes tens of seconds to build and
tens of GB of device memory): plans of one form (FP64 only, or split-FP32 only) are kept until a
test asks for the other form, which frees them first.
"""
import math

import numpy as np
import pytest

import oracle
import sht_synthetic as syn

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
SPLIT_TOL = 1e-9

_PLANS = {}


def _plan(l, form, eps=1e-12, C=None):
    """Cached plan of bandlimit l holding the factor copies of one form ("fp64" or "split32")."""
    from paper_0910_5435_amd import Plan

    C = C or min(64, max(4, l // 2))
    for key in [k for k in _PLANS if k[1] != form]:
        _PLANS.pop(key).close()
    key = (l, form, eps, C)
    if key not in _PLANS:
        if form == "fp64":
            _PLANS[key] = Plan(l, eps=eps, leaf_width=C)
        else:
            _PLANS[key] = Plan(l, eps=eps, leaf_width=C, precision=form, split_only=True)
        st = _PLANS[key].stats()
        print(f"plan l={l} {form}: {st['t_total_s']:.1f} s, k_max {st['k_max']}, "
              f"{st['factor_entries']:.3e} factor entries, {st['device_bytes'] / 2**30:.1f} GiB", flush=True)
    return _PLANS[key]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    for key in list(_PLANS):
        _PLANS.pop(key).close()
    torch.cuda.empty_cache()


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    out = []
    for f in range(a.shape[0]):
        den = np.linalg.norm(b[f])
        out.append(np.linalg.norm(a[f] - b[f]) / (den if den > 0 else 1.0))
    return np.array(out)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _only_orders(beta, l, orders):
    """beta with every order outside `orders` (a list of |m|) set to zero."""
    mask = np.isin(np.abs(syn.orders_canonical(l)), orders)
    return np.where(mask[None, :], beta, 0.0), mask


# ------------------------------------------------------------------------ l = 1024, 64 fields
CHECK_FIELDS = [0, 21, 42, 63]


@pytest.mark.timeout(600)
def test_l1024_64_fields_every_order():
    # The benchmark's batch and launch configuration (l = 1024, 64 complex fields, eps 1e-12,
    # leaf width 64, R = 256 columns) in FP64 and split-FP32; four fields spread over the
    # batch are compared with the oracle on every order, in both directions.  Synthesis: the
    # benchmark's coefficients.  Analysis: seeded grids (every field of the batch is random;
    # the four checked ones come from sht_synthetic).
    from paper_0910_5435_amd import Plan

    l, C, F = 1024, 64, 64
    P = Plan(l, eps=1e-12, leaf_width=C, precision="split32")  # keeps its FP64 copies too
    P.prepare("int8")
    beta = syn.coefficients(l, F, seed=0, power=1.5)
    g4 = syn.grid(l, len(CHECK_FIELDS), seed=1)
    f_ref = oracle.synth(beta[CHECK_FIELDS], l, fast=True)
    a_ref = oracle.analyze(g4, l, fast=True)
    print("l=1024 oracle done", flush=True)
    db = _dev(beta)
    del beta
    gen = torch.Generator(device="cuda").manual_seed(1)
    dg = torch.randn((F, 2 * l, 4 * l), dtype=torch.complex128, device="cuda", generator=gen)
    dg[CHECK_FIELDS] = _dev(g4)
    for prec, tol in (("fp64", FP64_TOL), ("split32", SPLIT_TOL), ("int8", SPLIT_TOL)):
        es = _rel(P.synth(db, precision=prec)[CHECK_FIELDS].cpu().numpy(), f_ref)
        ea = _rel(P.analyze(dg, precision=prec)[CHECK_FIELDS].cpu().numpy(), a_ref)
        print(f"l=1024 F=64 {prec}, every order, fields {CHECK_FIELDS}: synthesis {es.max():.2e}, "
              f"analysis {ea.max():.2e} (gate {tol:.0e})", flush=True)
        assert es.max() < tol and ea.max() < tol
    P.close()
    del db, dg
    torch.cuda.empty_cache()


# ------------------------------------------------------------------------------ l = 2048
L_TOP = 2048
TOP_ORDERS = [0, 1, 517, 1500, 2047, 2048, 3000, 3700, 4094, 4095]


# The column kernel against the oracle's Q at the top bandlimit: the orders where the seeds
# Pbar_m^m fall below the FP64 range over most of the nodes (m >= ~1500 at x near the
# equator: exponent tracking), and the last orders.  The oracle's own step-one recurrence
# carries ~2e-10 relative error near x = 1 at degree ~4000 (about twice its l = 1024 figure:
# the error grows linearly with the degree there), i.e. ~4e-13 after the sqrt(2 w) row factor.
@pytest.mark.timeout(600)
def test_l2048_column_kernel_matches_oracle():
    P = _plan(L_TOP, "fp64", C=64)
    worst = 0.0
    for m in [0, 1500, 3000, 4095]:
        for p in (0, 1):
            q = P.columns(m, p)
            ref = oracle.dense_q(L_TOP, m, p)
            assert q.shape == ref.shape
            if ref.size:
                err = float(np.max(np.abs(q - ref)))
                worst = max(worst, err)
                assert err < 2e-12, (m, p, err)
    print(f"l=2048 columns: max abs diff vs oracle {worst:.3e}", flush=True)


def _top_parity(form, tol, precision=None):
    # l = 2048, four complex fields (R = 16: the matrix-core kernels), sampled orders:
    # synthesis of coefficients that vanish outside the sample (whole grids compared) and the
    # sampled orders of the analysis of a seeded grid.
    P = _plan(L_TOP, form, C=64)
    if precision:
        P.prepare(precision)
    form = precision or form
    F = 4
    beta_s, mask = _only_orders(syn.coefficients(L_TOP, F, seed=0, power=1.5), L_TOP, TOP_ORDERS)
    f_ref = oracle.synth(beta_s, L_TOP, orders=TOP_ORDERS, fast=True)
    es = _rel(P.synth(_dev(beta_s), precision=form).cpu().numpy(), f_ref)
    del f_ref
    g = syn.grid(L_TOP, F, seed=1)
    a_ref = oracle.analyze_orders(g, L_TOP, TOP_ORDERS, fast=True)[:, mask]
    ea = _rel(P.analyze(_dev(g), precision=form).cpu().numpy()[:, mask], a_ref)
    print(f"l=2048 F=4 {form}, orders {TOP_ORDERS}: synthesis {es.max():.2e}, analysis {ea.max():.2e} "
          f"(gate {tol:.0e})", flush=True)
    assert es.max() < tol and ea.max() < tol


@pytest.mark.timeout(600)
def test_l2048_fp64_matches_oracle():
    _top_parity("fp64", FP64_TOL)



# ---------------------------------------------------------------- mixed-request workload
C4_BANDLIMITS = [64, 128, 256, 512, 1024, 2048]
# Field counts at the two largest bandlimits are divided so that inputs, outputs, plans and
# workspace fit one GPU's 288 GB (the draw's 137 fields at l = 2048 alone need ~150 GB of
# coefficients and grids).
C4_DIVISOR = {1024: 4, 2048: 8}


def _c4_spec():
    """96 requests, bandlimit uniform over C4_BANDLIMITS, 1..16 complex fields (default_rng(0)),
    the counts at l = 1024 / 2048 divided by C4_DIVISOR (rounded up)."""
    rng = np.random.default_rng(0)
    ls = rng.choice(C4_BANDLIMITS, 96)
    fs = rng.integers(1, 17, 96)
    return [(int(l), int(math.ceil(f / C4_DIVISOR.get(int(l), 1)))) for l, f in zip(ls, fs)]


def _c4_orders(l):
    return sorted({0, 1, l // 3, l - 1, l, 2 * l - 1})


def _c4(form, tol):
    # One persistent launch per direction (more if the workspace limit cuts it), every request's
    # first field against the oracle on sampled orders (its coefficients vanish outside them),
    # every field's round trip analysis(synthesis(beta)) = beta.
    from paper_0910_5435_amd import Batch

    spec = _c4_spec()
    plans = {l: _plan(l, form) for l in sorted({l for l, _ in spec})}
    reqs = []
    for i, (l, F) in enumerate(spec):
        beta = syn.coefficients(l, F, seed=1000 + i, power=1.5)
        beta[:1], _ = _only_orders(beta[:1], l, _c4_orders(l))
        x = _dev(beta)
        y = torch.empty((F, 2 * l, 4 * l), dtype=torch.complex128, device="cuda")
        reqs.append((plans[l], x, y))
    limit = 32 << 30
    b = Batch(reqs, op="synth", precision=form, workspace_limit=limit)
    b.run()
    b.check()
    info_s = b.info()
    b.close()
    back = [(P, y, torch.empty((y.shape[0], P.n_coeffs), dtype=torch.complex128, device="cuda"))
            for (P, _, y) in reqs]
    a = Batch(back, op="analyze", precision=form, workspace_limit=limit)
    a.run()
    a.check()
    info_a = a.info()
    a.close()
    print(f"C4 {form}: {len(spec)} requests, {sum(F for _, F in spec)} fields; synthesis {info_s}; "
          f"analysis launches {info_a['launches']}", flush=True)
    worst_s = worst_a = worst_r = 0.0
    for i, ((P, x, y), (_, _, z)) in enumerate(zip(reqs, back)):
        l = P.l
        orders = _c4_orders(l)
        x0 = x[:1].cpu().numpy()
        y0 = y[:1].cpu().numpy()
        worst_s = max(worst_s, _rel(y0, oracle.synth(x0, l, orders=orders, fast=True)).max())
        _, mask = _only_orders(x0, l, orders)
        a_ref = oracle.analyze_orders(y0, l, orders, fast=True)[:, mask]
        worst_a = max(worst_a, _rel(z[:1].cpu().numpy()[:, mask], a_ref).max())
        worst_r = max(worst_r, _rel(z.cpu().numpy(), x.cpu().numpy()).max())
        if i % 16 == 15:
            print(f"C4 {form}: {i + 1} requests checked", flush=True)
    print(f"C4 {form}: synthesis vs oracle {worst_s:.2e}, analysis vs oracle {worst_a:.2e}, "
          f"round trip {worst_r:.2e} (gate {tol:.0e})", flush=True)
    assert worst_s < tol and worst_a < tol and worst_r < 2 * tol
    del reqs, back
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_c4_full_bandlimits_fp64():
    _c4("fp64", FP64_TOL)


@pytest.mark.timeout(600)
def test_l2048_int8_matches_oracle():
    # the int8-slice digits derived on the FP64 plan (after the mixed workload freed its data)
    _top_parity("fp64", SPLIT_TOL, precision="int8")


@pytest.mark.timeout(600)
def test_l2048_split_matches_oracle():
    _top_parity("split32", SPLIT_TOL)


@pytest.mark.timeout(900)
def test_c4_full_bandlimits_split():
    _c4("split32", SPLIT_TOL)
