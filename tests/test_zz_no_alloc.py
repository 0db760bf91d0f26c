"""GPU test of psms_apply_dw_noalloc, the stencil entry point that allocates nothing
(its internal fields live in a fixed device array): through the C-ABI it must give
what psms_apply_dw gives on the same inputs, on two calls in a row (the second with
fewer right-hand sides, so stale scratch contents would show), in FP64 and in mixed
precision, and must refuse host memory and requests larger than its scratch."""
import sys

import numpy as np
import pytest

from paper_1204_1306_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def psms():
    from paper_1204_1306_amd import psms as m

    m.load_library()
    return m


def test_noalloc_matches_apply_dw_on_two_calls(psms):
    import torch

    dev = torch.device("cuda:0")
    L, b, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.15
    ctx = psms.Context(L, b, kappa, stream=torch.cuda.current_stream().cuda_stream)
    ctx.gauge_load(0, torch.from_numpy(synth.gauge_field(L, 0.6, 2001)).to(dev))
    for prec, tol in ((psms.F64, 0.0), (psms.MIXED, 0.0)):
        for nrhs, seed in ((3, 71), (1, 72)):
            say(f"case noalloc prec={prec} nrhs={nrhs} seed={seed}")
            psi = torch.from_numpy(synth.gaussian_noise(L, nrhs, seed)).to(dev)
            ref = ctx.apply_dw(0, psi, prec)
            out = torch.full_like(psi, float("nan"))
            ctx.apply_dw_noalloc(0, psi, out, prec)
            torch.cuda.synchronize()
            diff = float((out - ref).abs().max())
            say(f"  max |noalloc - apply_dw| = {diff:.3e} (same kernels and launch: bitwise expected)")
            assert torch.isfinite(out).all()
            assert diff <= tol
    # host memory is refused (staging would need buffers)
    h = synth.gaussian_noise(L, 1, 73)
    s = ctx._lib.psms_apply_dw_noalloc(ctx._h, 0, psms._ptr(h), psms._ptr(np.empty_like(h)), 1, psms.F64)
    assert s == -1
    # more right-hand sides than the 64 MiB scratch holds: 2 x 192 B x 4096 sites = 1.5 MiB per field
    big = torch.zeros((44,) + tuple(psi.shape[1:]), dtype=psi.dtype, device=dev)
    s = ctx.apply_dw_noalloc(0, big, torch.empty_like(big), psms.F64, check=False)
    assert s == -1
    assert "scratch" in ctx._lib.psms_last_error(ctx._h).decode()
    ctx.close()


def test_noalloc_second_context_shares_the_device_array(psms):
    """Two contexts of different lattices on one device use the same array in turn."""
    import torch

    dev = torch.device("cuda:0")
    outs = []
    for L, seed in (((8, 8, 8, 8), 81), ((4, 4, 4, 8), 82)):
        say(f"case noalloc context L={L}")
        ctx = psms.Context(L, (2, 2, 2, 2), 0.13, stream=torch.cuda.current_stream().cuda_stream)
        ctx.gauge_load(0, torch.from_numpy(synth.gauge_field(L, 0.5, seed)).to(dev))
        psi = torch.from_numpy(synth.gaussian_noise(L, 2, seed + 1)).to(dev)
        out = torch.empty_like(psi)
        ctx.apply_dw_noalloc(0, psi, out, psms.F64)
        ref = ctx.apply_dw(0, psi, psms.F64)
        torch.cuda.synchronize()
        outs.append(float((out - ref).abs().max()))
        ctx.close()
    say(f"  differences {outs}")
    assert max(outs) == 0.0
