"""CP-ALS and the GD gradient captured in a HIP graph: the calls fork part of
their work onto the context's second stream and join it back by events, and
enqueue no memset or copy, so a captured step replays exactly.  One step
(three ALS iterations, then the GD gradient at the result) is captured on a
torch stream the context is bound to, then replayed three times with eager
work and synchronizations between the replays; every replay must equal, bit
for bit, the same step run eagerly from the same state."""
import numpy as np
import pytest
import torch

from gpu_util import build, say, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu


def _bits(x):
    return x.view(torch.int16) if x.dtype == torch.bfloat16 else x


# relabel: gathers from rank-ordered copies of the factors, which at R = 10
# are padded to 16 columns (the copies, the padded output and its narrowing
# are launched inside the capture too)
@pytest.mark.parametrize("R,dtype,relabel", [(32, "f32", False), (16, "bf16", False),
                                             (10, "f32", True), (10, "bf16", True)])
def test_captured_step_replays_bitwise(R, dtype, relabel):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    coo = gen.zipf_distinct((20_000, 15_000, 10_000), 300_000, 1.1, seed=81)
    F0 = gen.init_factors(coo.dims, R, seed=82)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    ctx = dfacto.Context(0)
    T = build(ctx, coo, relabel=relabel)
    assert T.info()["relabeled"] == relabel
    F = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(DEV).to(tdt) for f in F0]
    G = [torch.empty((d, R), dtype=torch.float32, device=DEV) for d in coo.dims]
    lam = torch.zeros(R, dtype=torch.float64, device=DEV)
    fit = torch.zeros(1, dtype=torch.float64, device=DEV)
    fv = torch.zeros(1, dtype=torch.float64, device=DEV)
    state = (*F, lam, fit)
    outs = (*F, lam, fit, *G, fv)

    def step():
        for _ in range(3):
            dfacto.als_iter(ctx, T, F, lam, fit)
        dfacto.gd_grad(ctx, T, F, G, fv, 0.05)

    start = [x.clone() for x in state]
    # eager reference: three steps from the start (this also sizes every
    # workspace, so nothing allocates during the capture)
    eager = []
    for _ in range(3):
        step()
        torch.cuda.synchronize()
        eager.append([x.clone() for x in outs])
    for x, y in zip(state, start):
        x.copy_(y)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    main = torch.cuda.current_stream()
    try:
        with torch.cuda.graph(g, stream=side):
            ctx.set_stream(side)
            step()
    finally:
        ctx.set_stream(main)
    torch.cuda.synchronize()
    # the capture ran nothing: restore the start state before the replays
    for x, y in zip(state, start):
        x.copy_(y)
    torch.cuda.synchronize()
    scratch = torch.empty((coo.dims[0], R), device=DEV)
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = [x.clone() for x in outs]
        same = [torch.equal(_bits(a), _bits(b)) for a, b in zip(got, eager[k])]
        say(f"  R={R} {dtype}: replay {k + 1} equal to eager step {k + 1}: {all(same)} "
            f"(fit {float(fit):.6f})")
        assert all(same), [i for i, s in enumerate(same) if not s]
        # eager library work between the replays (it must not disturb them)
        dfacto.mttkrp(ctx, T, 0, F, scratch)
        torch.cuda.synchronize()
    del g
    T.close()
    ctx.close()


def test_frozen_context_refuses_to_grow_workspaces():
    """After dfacto_ctx_freeze a call that needs larger workspaces fails with
    E_INVALID (so addresses recorded in a graph stay valid); calls at the
    sizes already reserved still run, and unfreezing restores growth."""
    from gpu_util import build, factors_to_dev
    ctx = dfacto.Context(0)
    small = gen.uniform_distinct((50, 40, 30), 2_000, seed=31)
    big = gen.zipf_distinct((4000, 3000, 2000), 200_000, 1.1, seed=32)
    t1, t2 = build(ctx, small), build(ctx, big)
    R = 8
    F1, _ = factors_to_dev(gen.init_factors(small.dims, R, seed=33), "f32")
    lam = torch.zeros(R, dtype=torch.float64, device="cuda:0")
    fit = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    dfacto.als_iter(ctx, t1, F1, lam, fit)  # sizes the workspaces for t1
    ctx.freeze(True)
    dfacto.als_iter(ctx, t1, F1, lam, fit)  # same sizes: runs
    F2, _ = factors_to_dev(gen.init_factors(big.dims, R, seed=34), "f32")
    with pytest.raises(dfacto.DfactoError) as e:
        dfacto.als_iter(ctx, t2, F2, lam, fit)
    assert e.value.status == dfacto.E_INVALID and "frozen" in ctx.last_error()
    ctx.freeze(False)
    dfacto.als_iter(ctx, t2, F2, lam, fit)  # grows now
    torch.cuda.synchronize()
    # the same iteration on a fresh context: bitwise the same factors
    ctx2 = dfacto.Context(0)
    F3, _ = factors_to_dev(gen.init_factors(big.dims, R, seed=34), "f32")
    lam2 = torch.zeros_like(lam)
    fit2 = torch.zeros_like(fit)
    dfacto.als_iter(ctx2, t2, F3, lam2, fit2)
    torch.cuda.synchronize()
    for a, b in zip(F2, F3):
        assert torch.equal(a, b)
    assert fit.item() == fit2.item()
    for t in (t1, t2):
        t.close()
    ctx.close()
    ctx2.close()


def test_frozen_context_runs_padded_relabeled_calls():
    """A relabeled tensor at R = 10 (rank-ordered copies padded to 16
    columns, a padded output per MTTKRP): once CP-ALS and the GD gradient have
    run, every workspace they use is reserved, so the same calls on a frozen
    context run, with bitwise the same results."""
    from gpu_util import build, factors_to_dev
    ctx = dfacto.Context(0)
    coo = gen.zipf_distinct((6000, 4000, 3000), 150_000, 1.1, seed=35)
    t = build(ctx, coo, relabel=True)
    assert t.info()["relabeled"]
    R = 10
    F0 = gen.init_factors(coo.dims, R, seed=36)
    lam = torch.zeros(R, dtype=torch.float64, device="cuda:0")
    fit = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    fv = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    G = [torch.empty((d, R), dtype=torch.float32, device="cuda:0") for d in coo.dims]
    outs = []
    for frozen in (False, True):
        F, _ = factors_to_dev(F0, "f32")
        ctx.freeze(frozen)
        dfacto.als_iter(ctx, t, F, lam, fit)
        dfacto.gd_grad(ctx, t, F, G, fv, 0.05)
        torch.cuda.synchronize()
        outs.append([x.clone() for x in (*F, lam, fit, *G, fv)])
    ctx.freeze(False)
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    t.close()
    ctx.close()
