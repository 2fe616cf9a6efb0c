"""Parity at the paper-shape full size, in the launch configuration the
benchmark times: 6.5M x 2.5M x 1.5M with 1.2B distinct Zipf(1.2)
coordinates (drawn and deduplicated on the device, as the benchmark does),
R = 32, FP32 factors (and BF16 for mode 0).

An output row of mode n depends only on the nonzeros whose mode-n index is
that row, so the FP64 oracle, run on the sub-tensor of the sampled rows'
nonzeros with the full factors, gives those rows exactly.  Sampled per mode
(on the device, from the row counts): the 10th and 1000th heaviest rows
(millions and tens of thousands of nonzeros, split over many work chunks),
40 random nonempty rows, and empty rows (which must come out exactly
zero)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import factors_to_dev, rel_fro, say, to_host64, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu

DIMS = (6_500_000, 2_500_000, 1_500_000)
NNZ = 1_200_000_000
R = 32
TOL = 1e-5


@pytest.fixture(scope="module")
def paper():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("  generating the paper-shape tensor (1.2B distinct coordinates) on the device")
    i, j, k, v = gen.zipf_distinct_torch(DIMS, NNZ, 1.2, seed=3, device=DEV, batch=1 << 28)
    # the generator's temporaries go back to the device before the build
    # allocates (the library does not draw from torch's cache)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ctx = dfacto.Context(0)
    t = dfacto.build_flattenings(ctx, DIMS, i, j, k, v)
    torch.cuda.synchronize()
    say(f"  built: {t.info()['nnz']:,} nonzeros, {t.info()['bytes'] / 1e9:.1f} GB")
    coords = (i, j, k)
    gen_dev = torch.Generator(device=DEV)
    gen_dev.manual_seed(77)
    samples = []
    for m in range(3):
        cnt = torch.bincount(coords[m], minlength=DIMS[m])
        order = torch.argsort(cnt, descending=True, stable=True)
        nonempty = torch.nonzero(cnt).flatten()
        pick = torch.randint(0, nonempty.numel(), (40,), device=DEV, generator=gen_dev)
        empty = torch.nonzero(cnt == 0).flatten()[:4]
        rows = torch.unique(torch.cat([order[10:11], order[1000:1001], nonempty[pick], empty]))
        mark = torch.zeros(DIMS[m], dtype=torch.bool, device=DEV)
        mark[rows] = True
        keep = mark[coords[m]]  # a lookup per nonzero (no broadcast comparison)
        sub = tuple(a[keep].cpu().numpy() for a in (i, j, k, v))
        rows_h = rows.cpu().numpy().astype(np.int64)
        cnt_h = cnt[rows].cpu().numpy()
        samples.append(dict(rows=rows_h, empty=rows_h[cnt_h == 0],
                            sub=(sub[0].view(np.uint32), sub[1].view(np.uint32),
                                 sub[2].view(np.uint32), sub[3].astype(np.float64))))
        say(f"  mode {m}: {len(rows_h)} sampled rows, {len(sub[3]):,} of their nonzeros, "
            f"10th heaviest {int(cnt[order[10]]):,}")
        del cnt, order, nonempty, keep, mark
    del i, j, k, v, coords
    torch.cuda.empty_cache()
    F0 = gen.init_factors(DIMS, R, seed=1003)
    yield ctx, t, samples, F0
    t.close()
    ctx.close()
    torch.cuda.empty_cache()


def _check(got, ref, rows, empty, what):
    err = rel_fro(got, ref)
    say(f"  {what}: sampled rows err {err:.2e}")
    assert np.isfinite(got).all() and err <= TOL
    for r in range(len(rows)):
        assert rel_fro(got[r], ref[r]) <= 10 * TOL or np.linalg.norm(ref[r]) == 0
    for r in np.searchsorted(rows, empty):
        assert (got[r] == 0).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_paper_shape_mttkrp_sampled_rows(paper, dtype):
    ctx, t, samples, F0 = paper
    Fd, Fw = factors_to_dev(F0, dtype)
    modes = range(3) if dtype == "f32" else [0]
    for m in modes:
        out = torch.full((DIMS[m], R), float("nan"), device=DEV)
        dfacto.mttkrp(ctx, t, m, Fd, out)
        s = samples[m]
        got = to_host64(out[torch.from_numpy(s["rows"]).to(DEV)])
        del out
        ref = oracle.mttkrp(*s["sub"], DIMS, Fw, m)[s["rows"]]
        _check(got, ref, s["rows"], s["empty"], f"{dtype} MTTKRP mode {m}")
    del Fd
    torch.cuda.empty_cache()
