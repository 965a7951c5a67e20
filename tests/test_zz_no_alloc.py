"""The no-allocation synthesis entry point through the C ABI: sht_synth_noalloc (workspace in the
library's fixed device array) against sht_synth (caller's workspace) on the same plans and
inputs.  Same kernels, same launch shapes: the outputs must agree bit for bit, on consecutive
calls that reuse the array with smaller inputs."""
import ctypes

import numpy as np
import pytest

import sht_synthetic as syn

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _noalloc(lib, plan, coeff, grid):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.sht_synth_noalloc(plan.handle, ctypes.c_void_p(coeff.data_ptr()), ctypes.c_void_p(grid.data_ptr()),
                               int(coeff.shape[0]), stream)
    torch.cuda.synchronize()
    return rc


def test_noalloc_synthesis_matches_sht_synth():
    from paper_0910_5435_amd import Plan, _lib

    lib = _lib.load()
    p128 = Plan(128, eps=1e-13, leaf_width=32)
    p64 = Plan(64, eps=1e-13, leaf_width=16)
    s64 = Plan(64, eps=1e-12, leaf_width=16, precision="split32")
    # consecutive calls, each smaller than the one before: matrix-core width (R = 32), vector
    # kernels (R = 8), a smaller plan (R = 4), then the split form on the matrix cores (R = 16)
    cases = [(p128, 8, 0), (p128, 2, 1), (p64, 1, 2), (s64, 4, 3)]
    for plan, F, seed in cases:
        assert plan.workspace_bytes(F) <= _lib.NOALLOC_SCRATCH_BYTES
        coeff = torch.from_numpy(syn.coefficients(plan.l, F, seed=seed, power=1.5)).cuda()
        want = plan.synth(coeff)
        got = torch.full_like(want, complex("nan+nanj"))
        assert _noalloc(lib, plan, coeff, got) == _lib.SHT_OK
        assert torch.equal(got, want), (plan.l, F, float((got - want).abs().max()))
        print(f"noalloc l={plan.l} F={F} {plan.precision}: identical to sht_synth", flush=True)
    # a workspace beyond the fixed array is refused before anything runs
    big = Plan(256, eps=1e-13, leaf_width=64)
    F = 64
    assert big.workspace_bytes(F) > _lib.NOALLOC_SCRATCH_BYTES
    coeff = torch.zeros((F, big.n_coeffs), dtype=torch.complex128, device="cuda")
    grid = torch.empty((F,) + big.grid_shape, dtype=torch.complex128, device="cuda")
    assert _noalloc(lib, big, coeff, grid) == _lib.SHT_EUNSUPPORTED
    for plan in (p128, p64, s64, big):
        plan.close()
