"""Parity at the benchmark's full size, in the launch configuration the
benchmark times: zipf50m (1M x 500K x 200K, 50M distinct Zipf(1.1)
coordinates, R = 32), FP32 and BF16 factor storage.

An output row of mode n depends only on the nonzeros whose mode-n index is
that row, and on the whole factors through the R x R Gram matrices.  So the
FP64 oracle, run on the sub-tensor of the sampled rows' nonzeros with the
full factors, gives those rows exactly.  Sampled per mode: the heaviest row
(millions of nonzeros, split over thousands of work chunks: the long-run
carry fix-up), the 10th and 1000th heaviest rows, 40 random nonempty rows,
and empty rows (which must come out exactly zero)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import build, factors_to_dev, rel_fro, say, to_host64, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu

# BF16-stored inputs are exact in the oracle's input (widened), so the
# FP32-accumulation tolerance applies to both storage dtypes
TOL = 1e-5


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("  generating zipf50m (50M distinct coordinates)")
    coo, R, F0 = gen.zipf_50m()
    ctx = dfacto.Context(0)
    t = build(ctx, coo)
    coords = (coo.i, coo.j, coo.k)
    rng = np.random.default_rng(77)
    samples = []
    for m in range(3):
        cnt = np.bincount(coords[m], minlength=coo.dims[m])
        order = np.argsort(cnt, kind="stable")[::-1]
        nonempty = np.flatnonzero(cnt)
        rows = [order[0], order[10], order[1000]]
        rows += list(rng.choice(nonempty, 40, replace=False))
        rows += list(np.flatnonzero(cnt == 0)[:4])
        rows = np.unique(np.array(rows, dtype=np.int64))
        sel = np.zeros(coo.dims[m], bool)
        sel[rows] = True
        keep = sel[coords[m]]
        samples.append(dict(rows=rows, empty=rows[cnt[rows] == 0],
                            sub=tuple(np.ascontiguousarray(a[keep]) for a in coo.arrays64())))
        say(f"  mode {m}: {len(rows)} sampled rows, {int(keep.sum()):,} of their nonzeros, "
            f"heaviest {int(cnt[order[0]]):,}")
    yield coo, R, F0, ctx, t, samples
    t.close()
    ctx.close()


def _check_rows(got, ref, rows, empty, what):
    err = rel_fro(got, ref)
    say(f"  {what}: sampled rows err {err:.2e}")
    assert np.isfinite(got).all()
    assert err <= TOL
    # per row as well, so one bad row cannot hide in the heavy rows' norm
    for r in range(len(rows)):
        assert rel_fro(got[r], ref[r]) <= 10 * TOL or np.linalg.norm(ref[r]) == 0
    for r in np.searchsorted(rows, empty):
        assert (got[r] == 0).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fullsize_mttkrp_sampled_rows(full, dtype):
    coo, R, F0, ctx, t, samples = full
    Fd, Fw = factors_to_dev(F0, dtype)
    outs = [torch.full((d, R), float("nan"), device=DEV) for d in coo.dims]
    for m in range(3):
        dfacto.mttkrp(ctx, t, m, Fd, outs[m])
    torch.cuda.synchronize()
    for m in range(3):
        s = samples[m]
        ref = oracle.mttkrp(*s["sub"], coo.dims, Fw, m)[s["rows"]]
        _check_rows(to_host64(outs[m])[s["rows"]], ref, s["rows"], s["empty"],
                    f"{dtype} MTTKRP mode {m}")


def test_fullsize_gd_sampled_rows(full):
    """GD gradient rows of every mode, FP32 factors (the oracle computes all
    three gradients of the sub-tensor per call; the row of the sampled mode
    is exact)."""
    coo, R, F0, ctx, t, samples = full
    Fd, Fw = factors_to_dev(F0, "f32")
    grads = [torch.full((d, R), float("nan"), device=DEV) for d in coo.dims]
    f = torch.zeros(1, dtype=torch.float64, device=DEV)
    dfacto.gd_grad(ctx, t, Fd, grads, f, 0.0)
    torch.cuda.synchronize()
    for m in range(3):
        s = samples[m]
        gref = oracle.gd_grad(*s["sub"], coo.dims, Fw)[0][m][s["rows"]]
        got = to_host64(grads[m])[s["rows"]]
        err = rel_fro(got, gref)
        say(f"  gradient mode {m}: sampled rows err {err:.2e}")
        assert np.isfinite(got).all() and err <= TOL


def test_fullsize_als_mode0_sampled_rows(full):
    """One CP-ALS iteration: the new mode-0 factor's sampled rows equal
    M_0 H^-1 (H = B^T B * C^T C from the initial factors) up to the positive
    column scaling the normalization applies."""
    coo, R, F0, ctx, t, samples = full
    Fd, Fw = factors_to_dev(F0, "f32")
    lam = torch.zeros(R, dtype=torch.float64, device=DEV)
    fit = torch.zeros(1, dtype=torch.float64, device=DEV)
    dfacto.als_iter(ctx, t, Fd, lam, fit)
    torch.cuda.synchronize()
    s = samples[0]
    rows = s["rows"]
    M = oracle.mttkrp(*s["sub"], coo.dims, Fw, 0)[rows]
    H = (Fw[1].T @ Fw[1]) * (Fw[2].T @ Fw[2])
    U = np.linalg.solve(H, M.T).T
    A = to_host64(Fd[0])[rows]
    d = np.einsum("rc,rc->c", A, U) / np.einsum("rc,rc->c", U, U)
    err = rel_fro(A, U * d)
    say(f"  ALS mode 0 rows: err {err:.2e}, column scales in [{d.min():.3e}, {d.max():.3e}], "
        f"fit {fit.item():.6f}")
    assert (d > 0).all()
    assert err <= TOL
    assert np.isfinite(fit.item()) and 0.0 <= fit.item() <= 1.0
