"""GPU parity on the paper's synthetic tensor model (preferential
attachment, Section 5) at a reduced size of its first sweep: I = J = K =
10,000 with 100,000 nonzeros, R = 10, FP32 factors.  Nearly every fiber
holds one nonzero here, the case where DFacTo's fiber compression saves
least."""
import pytest
import torch

import oracle
from gpu_util import build, factors_to_dev, rel_fro, say, to_host64, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu


def test_preferential_tensor_mttkrp_als_gd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = dfacto.Context(0)
    coo = gen.preferential_distinct((10_000, 10_000, 10_000), 100_000, seed=70)
    R = 10
    F0 = gen.init_factors(coo.dims, R, seed=71)
    t = build(ctx, coo)
    info = t.info()
    say(f"  fibers per mode {info['nfib']} for {info['nnz']:,} nonzeros")
    Fd, Fw = factors_to_dev(F0, "f32")
    x = coo.arrays64()
    for m in range(3):
        out = torch.empty((coo.dims[m], R), device=DEV)
        dfacto.mttkrp(ctx, t, m, Fd, out)
        torch.cuda.synchronize()
        assert rel_fro(to_host64(out), oracle.mttkrp(*x, coo.dims, Fw, m)) <= 1e-5
    grads = [torch.empty((d, R), device=DEV) for d in coo.dims]
    f = torch.zeros(1, dtype=torch.float64, device=DEV)
    dfacto.gd_grad(ctx, t, Fd, grads, f)
    torch.cuda.synchronize()
    gref, fref = oracle.gd_grad(*x, coo.dims, Fw)
    assert max(rel_fro(to_host64(grads[m]), gref[m]) for m in range(3)) <= 1e-5
    assert abs(f.item() - fref) <= 1e-6 * abs(fref)
    lam = torch.zeros(R, dtype=torch.float64, device=DEV)
    fit = torch.zeros(1, dtype=torch.float64, device=DEV)
    dfacto.als_iter(ctx, t, Fd, lam, fit)
    torch.cuda.synchronize()
    A, B, C, lam_ref, oinfo = oracle.als_iter(*x, coo.dims, Fw)
    errs = [rel_fro(to_host64(Fd[m]), ref) for m, ref in enumerate((A, B, C))]
    say(f"  ALS factor errors {errs}, fit {fit.item():.6f} vs {oinfo['fit']:.6f}")
    assert max(errs) <= 1e-5
    assert abs(fit.item() - oinfo["fit"]) <= 1e-4
    t.close()
    ctx.close()
