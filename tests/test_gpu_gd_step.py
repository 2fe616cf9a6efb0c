"""GPU parity of the full GD iteration (dfacto_gd_step: gradients, Armijo
backtracking line search, simultaneous update) against the FP64 oracle's
gd_step: the same trial count, step and acceptance, and factors and
objective values within the single-call tolerances, over several
consecutive steps, for FP32 and BF16 factor storage."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import build, factors_to_dev, rel_fro, say, to_host64, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu

BF16_REL = 2.0 ** -8


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dfacto.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


CASES = {
    "uniform": lambda: gen.small_uniform(),
    "zipf": lambda: (lambda coo: (coo, 16, gen.init_factors(coo.dims, 16, seed=61)))(
        gen.zipf_distinct((700, 400, 250), 40_000, 1.1, seed=60)),
}


@pytest.mark.parametrize("case,dtype,reg", [("uniform", "f32", 0.0), ("zipf", "f32", 0.2),
                                            ("uniform", "bf16", 0.0), ("zipf", "bf16", 0.0)])
def test_gd_step_matches_oracle(ctx, case, dtype, reg):
    coo, R, F0 = CASES[case]()
    t = build(ctx, coo)
    Fd, Fw = factors_to_dev(F0, dtype)
    grads = [torch.empty((d, R), device=DEV) for d in coo.dims]
    ref = Fw
    tol_f = 1e-5 if dtype == "f32" else BF16_REL
    store = "f64" if dtype == "f32" else "bf16"
    for step in range(4):
        info = dfacto.gd_step(ctx, t, Fd, grads, reg, alpha0=1.0, shrink=0.5, c=1e-4, max_trials=40)
        torch.cuda.synchronize()
        A, B, C, oinfo = oracle.gd_step(*coo.arrays64(), coo.dims, ref, reg, alpha0=1.0, shrink=0.5,
                                        c=1e-4, max_trials=40, store=store)
        errs = [rel_fro(to_host64(Fd[m]), x) for m, x in enumerate((A, B, C))]
        say(f"  {case} {dtype} reg={reg} step {step}: trials {info['trials']}/{oinfo['trials']}, "
            f"alpha {info['alpha']:.3e}/{oinfo['alpha']:.3e}, f {info['f']:.8e}/{oinfo['f']:.8e}, "
            f"factor err {max(errs):.2e}")
        assert info["accepted"] == oinfo["accepted"]
        assert info["trials"] == oinfo["trials"]
        assert info["alpha"] == oinfo["alpha"]
        assert abs(info["f0"] - oinfo["f0"]) <= 1e-6 * abs(oinfo["f0"])
        assert abs(info["f"] - oinfo["f"]) <= 1e-6 * abs(oinfo["f0"])
        assert abs(info["gnorm2"] - oinfo["gnorm2"]) <= 1e-5 * oinfo["gnorm2"]
        assert max(errs) <= tol_f
        assert info["f"] <= info["f0"]
        ref = [A, B, C]
    t.close()


def test_gd_step_no_trial_passes(ctx):
    """A first step far too long with one trial: nothing passes and the
    factors stay bitwise as they were."""
    coo, R, F0 = gen.small_uniform()
    t = build(ctx, coo)
    Fd, _ = factors_to_dev(F0, "f32")
    before = [f.clone() for f in Fd]
    grads = [torch.empty((d, R), device=DEV) for d in coo.dims]
    info = dfacto.gd_step(ctx, t, Fd, grads, alpha0=1e8, max_trials=1)
    torch.cuda.synchronize()
    assert not info["accepted"] and info["trials"] == 1 and info["alpha"] == 0.0
    assert info["f"] == info["f0"]
    for a, b in zip(Fd, before):
        assert torch.equal(a, b)
    t.close()


def test_gd_step_argument_errors(ctx):
    coo, R, F0 = gen.small_uniform()
    t = build(ctx, coo)
    Fd, _ = factors_to_dev(F0, "f32")
    grads = [torch.empty((d, R), device=DEV) for d in coo.dims]
    for kw in (dict(alpha0=0.0), dict(alpha0=float("inf")), dict(shrink=1.0), dict(shrink=0.0),
               dict(c=0.0), dict(c=1.0), dict(max_trials=0), dict(max_trials=1001)):
        with pytest.raises(dfacto.DfactoError) as e:
            dfacto.gd_step(ctx, t, Fd, grads, **kw)
        assert e.value.status == dfacto.E_INVALID, kw
    # the context is still usable
    info = dfacto.gd_step(ctx, t, Fd, grads)
    assert info["accepted"]
    t.close()
