"""GPU tests of served solves (dfacto_server_*): continuous batching must not
change any result -- each request gives bitwise the same factors, weights,
fit and iteration count alone and in a mix -- and those results are the ones
of dfacto_als_iter repeated on the request alone and agree with the FP64
oracle's CP-ALS trajectory from the same start; admission respects the slot
count and the memory budget."""
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_util import rel_fro, say, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu

SPECS = [
    ((900, 700, 500), 20_000, 8, "f32"),
    ((3000, 1000, 400), 60_000, 16, "f32"),
    ((500, 1500, 800), 30_000, 32, "bf16"),
    ((2000, 2000, 2000), 100_000, 32, "f32"),
    ((700, 300, 200), 8_000, 16, "bf16"),
    ((1200, 900, 600), 40_000, 8, "f32"),
]


@pytest.fixture(scope="module")
def requests():
    out = []
    for s, (dims, nnz, R, dt) in enumerate(SPECS):
        coo = gen.zipf_distinct(dims, nnz, 1.1, seed=900 + s)
        init = [f.astype(np.float32) for f in gen.init_factors(coo.dims, R, seed=950 + s)]
        out.append(dict(coo=coo, R=R, dtype=dt, init=init))
    return out


def _submit(srv, r, tol=1e-4, max_iters=12):
    c = r["coo"]
    return srv.submit(c.dims, c.i, c.j, c.k, c.val, r["R"], r["init"], dtype=r["dtype"], tol=tol,
                      max_iters=max_iters)


def _alone(requests, **kw):
    srv = dfacto.Server(0, max_slots=1)
    res = [srv.wait(_submit(srv, r, **kw)) for r in requests]
    srv.close()
    return res


def _same(a, b):
    assert a["status"] == b["status"] == dfacto.OK
    assert a["iters"] == b["iters"]
    assert a["fit"] == b["fit"]
    for m in range(3):
        assert np.array_equal(a["factors"][m], b["factors"][m])
    assert np.array_equal(a["lam"], b["lam"])


def test_served_results_same_alone_and_in_mix(requests):
    alone = _alone(requests)
    srv = dfacto.Server(0, max_slots=8)
    ids = []
    for q, r in enumerate(requests):  # staggered arrivals: later ones join running work
        ids.append(_submit(srv, r))
        if q % 2 == 1:
            time.sleep(0.01)
    mix = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    say(f"  server stats: {st}; iterations per request {[m['iters'] for m in mix]}")
    assert st["peak_active"] >= 2, "the requests never overlapped"
    for a, b in zip(alone, mix):
        _same(a, b)


@pytest.mark.parametrize("which", [1, 2])  # an FP32 and a BF16 request
def test_served_result_equals_repeated_als_iter(requests, which):
    """The served solve equals dfacto_als_iter repeated on the request alone;
    for BF16 storage the server's rounding of the initial factors is torch's
    (nearest, ties to even) and its widening of the results is exact."""
    r = requests[which]
    res = _alone([r])[0]
    c = r["coo"]
    ctx = dfacto.Context(0)
    from gpu_util import build
    t = build(ctx, c)
    F = [torch.from_numpy(f.copy()).to(DEV) for f in r["init"]]
    if r["dtype"] == "bf16":
        F = [f.to(torch.bfloat16) for f in F]
    lam = torch.zeros(r["R"], dtype=torch.float64, device=DEV)
    fit = torch.zeros(1, dtype=torch.float64, device=DEV)
    for _ in range(res["iters"]):
        dfacto.als_iter(ctx, t, F, lam, fit)
    torch.cuda.synchronize()
    assert fit.item() == res["fit"]
    for m in range(3):
        assert np.array_equal(F[m].float().cpu().numpy(), res["factors"][m])
    assert np.array_equal(lam.cpu().numpy(), res["lam"])
    t.close()
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_served_large_request_staged_in_chunks(dtype):
    """A request whose COO arrays (36 MB each) and factors (38 MB) exceed one
    32 MB pinned staging buffer, so uploads and downloads run in several
    chunks through both buffers: the served result equals dfacto_als_iter
    repeated on the request from the same start, bitwise."""
    coo = gen.uniform_distinct((300_000, 250_000, 600), 9_000_000, seed=41)
    R = 32
    init = [f.astype(np.float32) for f in gen.init_factors(coo.dims, R, seed=42)]
    srv = dfacto.Server(0, max_slots=2)
    res = srv.wait(srv.submit(coo.dims, coo.i, coo.j, coo.k, coo.val, R, init, dtype=dtype,
                              tol=0.0, max_iters=3))
    srv.close()
    assert res["status"] == dfacto.OK and res["iters"] == 3
    ctx = dfacto.Context(0)
    from gpu_util import build
    t = build(ctx, coo)
    F = [torch.from_numpy(f.copy()).to(DEV) for f in init]
    if dtype == "bf16":
        F = [f.to(torch.bfloat16) for f in F]
    lam = torch.zeros(R, dtype=torch.float64, device=DEV)
    fit = torch.zeros(1, dtype=torch.float64, device=DEV)
    for _ in range(3):
        dfacto.als_iter(ctx, t, F, lam, fit)
    torch.cuda.synchronize()
    say(f"  {dtype} large served request: fit {res['fit']:.9f}")
    assert fit.item() == res["fit"]
    for m in range(3):
        assert np.array_equal(F[m].float().cpu().numpy(), res["factors"][m])
    assert np.array_equal(lam.cpu().numpy(), res["lam"])
    t.close()
    ctx.close()


def test_admission_limits(requests):
    # one slot: never more than one active
    srv = dfacto.Server(0, max_slots=1)
    ids = [_submit(srv, r, max_iters=3) for r in requests[:3]]
    res = [srv.wait(i) for i in ids]
    assert srv.stats()["peak_active"] == 1
    srv.close()
    assert all(x["status"] == dfacto.OK for x in res)
    # a 1-byte budget admits one request at a time (the first always fits)
    srv = dfacto.Server(0, hbm_budget=1, max_slots=8)
    ids = [_submit(srv, r, max_iters=3) for r in requests[:4]]
    res = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    assert st["peak_active"] == 1
    assert all(x["status"] == dfacto.OK for x in res)
    # admission follows arrival order
    admits = [x["t_admit"] for x in res]
    assert admits == sorted(admits)


def test_submit_errors(requests):
    srv = dfacto.Server(0, max_slots=2)
    r = requests[0]
    c = r["coo"]
    init5 = [np.zeros((d, 5), np.float32) for d in c.dims]
    with pytest.raises(dfacto.DfactoError) as e:
        srv.submit(c.dims, c.i, c.j, c.k, c.val, 5, init5)
    assert e.value.status == dfacto.E_UNSUPPORTED
    with pytest.raises(dfacto.DfactoError) as e:
        srv.submit(c.dims, c.i, c.j, c.k, c.val, r["R"], r["init"], max_iters=0)
    assert e.value.status == dfacto.E_INVALID
    # an out-of-range coordinate fails the request, not the server
    bad = c.i.copy()
    bad[0] = c.dims[0]
    rid = srv.submit(c.dims, bad, c.j, c.k, c.val, r["R"], r["init"], max_iters=2)
    assert srv.wait(rid)["status"] == dfacto.E_RANGE
    ok = srv.wait(_submit(srv, r, max_iters=2))
    assert ok["status"] == dfacto.OK and ok["iters"] == 2
    srv.close()


def _oracle_solve(coo, init, R, dtype, tol, max_iters):
    """The oracle's CP-ALS from the served start (the factors as stored:
    FP32, or BF16 rounded to nearest even), with the served stopping rule:
    stop after the iteration whose fit differs from the previous one by less
    than tol, or after max_iters.  Returns factors, lambda, fits."""
    store = "f64" if dtype == "f32" else "bf16"
    F = gen.round_factors(init, dtype)
    fits = []
    for it in range(max_iters):
        A, B, C, lam, info = oracle.als_iter(*coo.arrays64(), coo.dims, F, store=store)
        F = [A, B, C]
        fits.append(info["fit"])
        if it > 0 and abs(fits[-1] - fits[-2]) < tol:
            break
    return F, lam, fits


SERVED_ORACLE = {  # (fit, factors and lambda) bounds per storage dtype
    "f32": (1e-6, 1e-5),
    "bf16": (1e-4, 2.0 ** -8),
}


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_served_results_match_oracle(dtype):
    """Served solves run to the served stopping rule (fit change < 1e-4 or 50
    iterations): the iteration count, final factors, weights and fit equal
    the oracle's trajectory from the same start.  A planted rank-4 tensor
    plus noise (every entry stored: its fit converges to about 0.74) and a
    Zipf tensor capped at 12 iterations, submitted together."""
    coo_p, _ = gen.planted_dense_noisy((40, 30, 25), 4, seed=21, noise=0.1)
    init_p = [f.astype(np.float32) for f in gen.init_factors(coo_p.dims, 4, seed=22)]
    coo_z = gen.zipf_distinct((900, 700, 500), 20_000, 1.1, seed=900)
    init_z = [f.astype(np.float32) for f in gen.init_factors(coo_z.dims, 8, seed=950)]
    cases = [(coo_p, init_p, 4, 50), (coo_z, init_z, 8, 12)]
    srv = dfacto.Server(0, max_slots=4)
    ids = [srv.submit(c.dims, c.i, c.j, c.k, c.val, R, init, dtype=dtype, tol=1e-4,
                      max_iters=mi) for c, init, R, mi in cases]
    got = [srv.wait(i) for i in ids]
    srv.close()
    ftol, rtol = SERVED_ORACLE[dtype]
    for (c, init, R, mi), res in zip(cases, got):
        assert res["status"] == dfacto.OK
        F, lam, fits = _oracle_solve(c, init, R, dtype, 1e-4, mi)
        errs = [rel_fro(res["factors"][m], F[m]) for m in range(3)]
        say(f"  {dtype} R={R}: served {res['iters']} iterations, oracle {len(fits)}; fit "
            f"{res['fit']:.9f} vs {fits[-1]:.9f}; factors {max(errs):.2e} lambda "
            f"{rel_fro(res['lam'], lam):.2e}")
        assert res["iters"] == len(fits)
        assert abs(res["fit"] - fits[-1]) <= ftol
        assert max(errs) <= rtol
        assert rel_fro(res["lam"], lam) <= rtol
