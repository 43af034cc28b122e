"""fab_sketch_apply_noalloc (for callers that cannot allocate device memory) against
fab_sketch_apply, the workspace entry point it is a variant of: the same kernels and grid, so the
same bits; two calls in a row, the second with a smaller input (the static scratch keeps the last
call's contents, which must not leak into the next result); d beyond the static scratch rejected."""
import ctypes

import numpy as np
import pytest

pytest.importorskip("torch")
import torch  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fab():
    import paper_2503_22631_amd as fab_mod
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fab_mod


@pytest.fixture(scope="module")
def ctx(fab):
    return fab.Context()


def _noalloc(ctx, x, d, zeta, seed):
    out = torch.full((d,), float("nan"), dtype=torch.float64, device=ctx.device)
    dt = 0 if x.dtype == torch.float64 else 1
    st = ctx.lib.fab_sketch_apply_noalloc(ctx.handle, x.numel(), d, zeta, seed, dt, ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()))
    return st, out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_sketch_matches_workspace_entry_point(fab, ctx, dtype):
    g = torch.Generator(device="cpu").manual_seed(5)
    for n, d, zeta in ((1_000_003, 256, 8), (70_001, 80, 4)):  # the second call smaller
        x = torch.randn(n, generator=g, dtype=torch.float64).to(dtype).to(ctx.device)
        ref = fab.sketch_apply(ctx, x, d, zeta, 11)
        st, got = _noalloc(ctx, x, d, zeta, 11)
        torch.cuda.synchronize()
        assert st == 0
        assert torch.equal(got, ref), (n, d, float((got - ref).abs().max()))
        assert np.isfinite(got.cpu().numpy()).all()


def test_noalloc_sketch_rejects_sizes_beyond_its_scratch(fab, ctx):
    x = torch.ones(1000, dtype=torch.float64, device=ctx.device)
    st, _ = _noalloc(ctx, x, 257, 8, 1)
    assert st == -2  # FAB_E_UNSUPPORTED: d beyond the static scratch
    st, _ = _noalloc(ctx, x, 80, 0, 1)
    assert st == -1
