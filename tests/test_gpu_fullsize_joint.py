"""Joint ALS at the benchmark's full size, in its launch configuration:
X = zipf50m (1M x 500K x 200K, 50M distinct Zipf(1.1) coordinates) as
users x items x words, Y = 10M distinct Zipf(1.1) ratings over its 1M users x
500K items, R = 32, FP32 factors, mu = 1, lam = 0.1, one iteration.

A user's new row depends only on that user's nonzeros of X and ratings of Y
and on the whole factors through R x R Grams, so the oracle's per-row
solution (oracle.joint_als_rows) on the sub-tensor and sub-ratings of the
sampled users, with the full factors, gives those rows exactly.  Users are
sampled on every path of the device: the heaviest (split into work
segments), heavy (thousands of ratings), dozens of ratings (Cholesky), 1 to 7
ratings (Woodbury identity) and none.  Items likewise, from the device's
updated users (the items' block uses the new A)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import build, factors_to_dev, rel_fro, say, to_host64, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu

MU, LAM = 1.0, 0.1
TOL = 1e-5


def _sample(cnt, rng):
    """Rows by rating count: the heaviest, ranks 50 and 2000, 8 rows with
    20-60 ratings, 8 with 1-7, 4 with none."""
    order = np.argsort(cnt, kind="stable")[::-1]
    rows = [order[0], order[50], order[2000]]
    for lo, hi, n in ((20, 60, 8), (1, 7, 8)):
        pool = np.flatnonzero((cnt >= lo) & (cnt <= hi))
        rows += list(rng.choice(pool, min(n, len(pool)), replace=False))
    rows += list(np.flatnonzero(cnt == 0)[:4])
    return np.unique(np.array(rows, dtype=np.int64))


@pytest.fixture(scope="module")
def joint():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("  generating zipf50m and 10M ratings")
    coo, R, F0 = gen.zipf_50m()
    yc = gen.zipf_distinct((coo.dims[0], coo.dims[1], 1), 10_000_000, 1.1, seed=31)
    ctx = dfacto.Context(0)
    X = build(ctx, coo)
    Y = dfacto.build_ratings(ctx, coo.dims[:2],
                             *[torch.from_numpy(a.view(np.int32)).to(DEV) for a in (yc.i, yc.j)],
                             torch.from_numpy(yc.val).to(DEV))
    Fd, Fw = factors_to_dev(F0, "f32")
    dfacto.joint_als_iter(ctx, X, Y, Fd, MU, LAM)
    torch.cuda.synchronize()
    new = [to_host64(f) for f in Fd]
    yield coo, yc, Fw, new
    X.close()
    Y.close()
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_fullsize_joint_rows(joint, mode):
    coo, yc, Fw, new = joint
    own = yc.i if mode == 0 else yc.j
    rows = _sample(np.bincount(own, minlength=coo.dims[mode]), np.random.default_rng(33 + mode))
    sel = np.zeros(coo.dims[mode], bool)
    sel[rows] = True
    xs = (coo.i, coo.j)[mode]
    kx, ky = sel[xs], sel[own]
    sub_x = (coo.i[kx], coo.j[kx], coo.k[kx], coo.val[kx].astype(np.float64))
    sub_y = (yc.i[ky], yc.j[ky], yc.val[ky].astype(np.float64))
    # the items' block starts from the device's new users
    factors = Fw if mode == 0 else [new[0], Fw[1], Fw[2]]
    ref = oracle.joint_als_rows(*sub_x, coo.dims, *sub_y, factors, MU, LAM, mode, rows)
    got = new[mode][rows]
    cnt = np.bincount(own, minlength=coo.dims[mode])[rows]
    err = rel_fro(got, ref)
    say(f"  {'users' if mode == 0 else 'items'}: {len(rows)} rows with {cnt.min()}..{cnt.max()} "
        f"ratings, {int(kx.sum()):,} tensor nonzeros; error {err:.2e}")
    assert np.isfinite(got).all() and err <= TOL
    for q in range(len(rows)):
        assert rel_fro(got[q], ref[q]) <= 10 * TOL, (rows[q], cnt[q])
