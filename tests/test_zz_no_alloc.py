"""dfacto_mttkrp_noalloc -- the MTTKRP with the library's fixed scratch
array instead of allocated workspace -- against dfacto_mttkrp, which runs
the same kernels: results must be bitwise equal.  Two calls in a row, the
second with a smaller input (the array keeps the first call's contents),
on a relabeled tensor (carries and permuted tables in the array) and a
plain one (carries only), FP32 and BF16; a call that needs more than the
array holds is refused."""
import numpy as np
import pytest
import torch

from gpu_util import build, factors_to_dev, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu


def _both(ctx, t, m, Fd, R):
    out = torch.full((t.info()["dims"][m], R), float("nan"), device=DEV)
    dfacto.mttkrp_noalloc(ctx, t, m, Fd, out)
    ref = dfacto.mttkrp(ctx, t, m, Fd)
    torch.cuda.synchronize()
    return out, ref


def test_noalloc_equals_mttkrp_two_calls_shrinking():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = dfacto.Context(0)
    big = gen.zipf_distinct((20_000, 12_000, 8_000), 600_000, 1.1, seed=91)
    small = gen.zipf_distinct((3_000, 2_000, 1_500), 40_000, 1.1, seed=92)
    tb = build(ctx, big, relabel=True)
    ts = build(ctx, small, relabel=False)
    assert tb.info()["relabeled"] and not ts.info()["relabeled"]
    cases = [(tb, big, 32, "f32"), (ts, small, 16, "bf16"), (tb, big, 10, "bf16"),
             (ts, small, 8, "f32")]
    for t, coo, R, dt in cases:
        Fd, _ = factors_to_dev(gen.init_factors(coo.dims, R, seed=93 + R), dt)
        for m in range(3):
            got, ref = _both(ctx, t, m, Fd, R)
            assert torch.equal(got, ref), (coo.nnz, R, dt, m)
    tb.close()
    ts.close()
    ctx.close()


def test_noalloc_refuses_beyond_the_array():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = dfacto.Context(0)
    # relabeled: mode 0 gathers a 1,000,000 x 32 FP32 table (128 MB) > 64 MiB
    coo = gen.zipf_distinct((4_000, 1_000_000, 500), 50_000, 1.1, seed=94)
    t = build(ctx, coo, relabel=True)
    Fd, _ = factors_to_dev(gen.init_factors(coo.dims, 32, seed=95), "f32")
    out = torch.empty((coo.dims[0], 32), device=DEV)
    with pytest.raises(dfacto.DfactoError) as e:
        dfacto.mttkrp_noalloc(ctx, t, 0, Fd, out)
    assert e.value.status == dfacto.E_UNSUPPORTED and "scratch" in ctx.last_error()
    # the context and the array stay usable
    small = gen.zipf_distinct((500, 400, 300), 5_000, 1.1, seed=96)
    ts = build(ctx, small)
    Fs, _ = factors_to_dev(gen.init_factors(small.dims, 4, seed=97), "f32")
    got, ref = _both(ctx, ts, 1, Fs, 4)
    assert torch.equal(got, ref)
    t.close()
    ts.close()
    ctx.close()
