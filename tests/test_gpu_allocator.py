"""The caller's allocator (dfacto_allocator) on the GPU: with torch's caching
allocator behind it, the flattenings, build temporaries, workspaces and group
workspaces are torch memory (seen by torch.cuda.memory_allocated while they
live, all returned after close), and every result is bitwise equal to the
one computed on a context that allocates by itself.  An allocator that
cannot serve a request turns it into DFACTO_E_NOMEM."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import build, factors_to_dev, say, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def problem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    coo = gen.zipf_distinct((900, 700, 500), 60_000, 1.1, seed=71)
    return coo, gen.init_factors(coo.dims, 16, seed=72)


class CountingTorchAllocator:
    """TorchAllocator that also counts the calls and the live bytes."""

    def __init__(self, fail=False):
        self.allocs = self.frees = 0
        self.live = {}

        def _alloc(nbytes, stream, user):
            if fail:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream or 0)
            self.allocs += 1
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, stream, user):
            self.frees += 1
            self.live.pop(ptr)
            torch.cuda.caching_allocator_delete(ptr)

        self._fns = (dfacto._ALLOC_FN(_alloc), dfacto._FREE_FN(_free))
        self.struct = dfacto._Allocator(self._fns[0], self._fns[1], None)


def _run_all(ctx, coo, F0):
    """MTTKRP of every mode, three ALS iterations, a GD gradient and two
    grouped ALS iterations; returns every result on the host."""
    t = build(ctx, coo)
    out = {}
    Fd, _ = factors_to_dev(F0, "f32")
    for m in range(3):
        M = torch.empty((coo.dims[m], 16), device=DEV)
        dfacto.mttkrp(ctx, t, m, Fd, M)
        out[f"mttkrp{m}"] = M
    Fa, _ = factors_to_dev(F0, "f32")
    lam = torch.zeros(16, dtype=torch.float64, device=DEV)
    fit = torch.zeros(1, dtype=torch.float64, device=DEV)
    for _ in range(3):
        dfacto.als_iter(ctx, t, Fa, lam, fit)
    out.update(alsA=Fa[0], alsB=Fa[1], alsC=Fa[2], lam=lam, fit=fit)
    G = [torch.empty((d, 16), device=DEV) for d in coo.dims]
    f = torch.zeros(1, dtype=torch.float64, device=DEV)
    dfacto.gd_grad(ctx, t, Fd, G, f, 0.1)
    out.update(g0=G[0], g1=G[1], g2=G[2], f=f)
    Fg, _ = factors_to_dev(F0, "f32")
    lg = torch.zeros(16, dtype=torch.float64, device=DEV)
    fg = torch.zeros(1, dtype=torch.float64, device=DEV)
    grp = dfacto.Group(ctx, [t], [Fg], [lg], fg)
    grp.als(2)
    torch.cuda.synchronize()
    out.update(grpA=Fg[0], grp_fit=fg)
    info = t.info()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    return t, grp, info, res


def test_torch_allocator_results_and_accounting(problem):
    coo, F0 = problem
    ref_ctx = dfacto.Context(0)
    t_ref, g_ref, _, ref = _run_all(ref_ctx, coo, F0)
    g_ref.close()
    t_ref.close()
    ref_ctx.close()

    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    alloc = CountingTorchAllocator()
    ctx = dfacto.Context(0, allocator=alloc)
    t, grp, info, got = _run_all(ctx, coo, F0)
    live = sum(alloc.live.values())
    say(f"  torch allocator: {alloc.allocs} allocations, {alloc.frees} frees, "
        f"{live} bytes live, tensor {info['bytes']} bytes")
    # the flattenings (and the workspaces) are torch memory while they live
    assert live >= info["bytes"]
    assert torch.cuda.memory_allocated(0) - base >= info["bytes"]
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    grp.close()
    t.close()
    ctx.close()
    torch.cuda.synchronize()
    # everything went back
    assert alloc.allocs == alloc.frees and not alloc.live
    say(f"  after close: torch allocated {torch.cuda.memory_allocated(0) - base} bytes above base")


def test_named_torch_allocator(problem):
    coo, F0 = problem
    ctx = dfacto.Context(0, allocator="torch")
    assert isinstance(ctx.allocator, dfacto.TorchAllocator)
    t = build(ctx, coo)
    Fd, _ = factors_to_dev(F0, "f32")
    M = torch.empty((coo.dims[0], 16), device=DEV)
    dfacto.mttkrp(ctx, t, 0, Fd, M)
    torch.cuda.synchronize()
    assert torch.isfinite(M).all()
    t.close()
    ctx.close()


def test_failing_allocator_reports_nomem(problem):
    coo, _ = problem
    alloc = CountingTorchAllocator(fail=True)
    ctx = dfacto.Context(0, allocator=alloc)
    with pytest.raises(dfacto.DfactoError) as e:
        build(ctx, coo)
    assert e.value.status == dfacto.E_NOMEM
    assert alloc.allocs == alloc.frees == 0
    ctx.close()
