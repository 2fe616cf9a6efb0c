"""GPU tests of grouped CP-ALS (dfacto_group_*): a group of uneven tensors
must give, member by member, bitwise the results of dfacto_als_iter run on
each member alone (same kernels, same work split, same reduction order), with
or without graph replay and autotuning, and must match the FP64 oracle at the
single-tensor tolerances."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import build, factors_to_dev, rel_fro, say, to_host64, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu

# (dims, nnz, R): uneven shapes and ranks, Zipf(1.1) coordinates
SPECS = [
    ((900, 700, 500), 20_000, 8),
    ((3000, 1000, 400), 60_000, 16),
    ((500, 1500, 800), 30_000, 32),
    ((2000, 2000, 2000), 100_000, 32),
    ((700, 300, 200), 8_000, 16),
    ((1200, 900, 600), 40_000, 8),
    ((400, 350, 300), 12_000, 4),
    ((1500, 800, 700), 50_000, 12),
]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dfacto.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def members(ctx):
    out = []
    for s, (dims, nnz, R) in enumerate(SPECS):
        coo = gen.zipf_distinct(dims, nnz, 1.1, seed=700 + s)
        out.append((coo, build(ctx, coo), R, gen.init_factors(coo.dims, R, seed=800 + s)))
    return out


def _state(members, dtype):
    Fs, lams = [], []
    for coo, t, R, F0 in members:
        Fs.append(factors_to_dev(F0, dtype)[0])
        lams.append(torch.zeros(R, dtype=torch.float64, device=DEV))
    fits = torch.zeros(len(members), dtype=torch.float64, device=DEV)
    return Fs, lams, fits


def _same(a, b):
    return torch.equal(a.view(torch.int16) if a.dtype == torch.bfloat16 else a,
                       b.view(torch.int16) if b.dtype == torch.bfloat16 else b)


def _edge_members(ctx):
    """Members that stress the combined tables: no nonzeros (no chunks, every
    row empty), one nonzero, one row of 20,000 nonzeros (long carry runs)
    next to light rows, and a full 12 x 11 x 10 tensor (no empty row)."""
    rng = np.random.default_rng(901)
    u32 = lambda a: np.asarray(a, dtype=np.uint32)
    coos = [gen.Coo((50, 40, 30), u32([]), u32([]), u32([]), np.zeros(0, np.float32)),
            gen.Coo((60, 50, 40), u32([7]), u32([3]), u32([39]), np.ones(1, np.float32))]
    lin = rng.choice(300 * 200, 20_000, replace=False)
    extra = rng.choice(400 * 300 * 200, 5_000, replace=False)
    ei, ej, ek = extra // (300 * 200), (extra // 200) % 300, extra % 200
    keep = ei != 5
    coos.append(gen.Coo((400, 300, 200), u32(np.concatenate([np.full(20_000, 5), ei[keep]])),
                        u32(np.concatenate([lin // 200, ej[keep]])),
                        u32(np.concatenate([lin % 200, ek[keep]])),
                        rng.standard_normal(20_000 + int(keep.sum())).astype(np.float32)))
    g = np.indices((12, 11, 10)).reshape(3, -1)
    coos.append(gen.Coo((12, 11, 10), u32(g[0]), u32(g[1]), u32(g[2]),
                        rng.standard_normal(g.shape[1]).astype(np.float32)))
    return [(c, build(ctx, c), R, gen.init_factors(c.dims, R, seed=910 + s))
            for s, (c, R) in enumerate(zip(coos, (8, 16, 32, 4)))]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_group_edge_members_bitwise(ctx, dtype):
    members = _edge_members(ctx)
    Fg, lg, fg = _state(members, dtype)
    Fs, ls, fs = _state(members, dtype)
    g = dfacto.Group(ctx, [m[1] for m in members], Fg, lg, fg)
    g.als(2)
    for k, (coo, t, R, _) in enumerate(members):
        fit = torch.zeros(1, dtype=torch.float64, device=DEV)
        for _ in range(2):
            dfacto.als_iter(ctx, t, Fs[k], ls[k], fit)
        fs[k] = fit[0]
    torch.cuda.synchronize()
    say(f"  edge members: nnz {[m[0].nnz for m in members]}, fits {fg.tolist()}")
    for k in range(len(members)):
        for m in range(3):
            assert _same(Fg[k][m], Fs[k][m]), f"member {k} factor {m} differs"
        assert torch.equal(lg[k], ls[k]) and torch.equal(fg[k], fs[k]), f"member {k}"
    g.close()
    for m in members:
        m[1].close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_group_bitwise_equals_single(ctx, members, dtype):
    Fg, lg, fg = _state(members, dtype)
    Fs, ls, fs = _state(members, dtype)
    g = dfacto.Group(ctx, [m[1] for m in members], Fg, lg, fg, graph=False)
    say(f"  group info: {g.info()}")
    iters = 3
    g.als(iters)
    for k, (coo, t, R, _) in enumerate(members):
        fit = torch.zeros(1, dtype=torch.float64, device=DEV)
        for _ in range(iters):
            dfacto.als_iter(ctx, t, Fs[k], ls[k], fit)
        fs[k] = fit[0]
    torch.cuda.synchronize()
    for k in range(len(members)):
        for m in range(3):
            assert _same(Fg[k][m], Fs[k][m]), f"member {k} factor {m} differs"
        assert torch.equal(lg[k], ls[k]), f"member {k} lambda differs"
        assert torch.equal(fg[k], fs[k]), f"member {k} fit differs"
    g.close()


def test_group_graph_replays(ctx, members):
    """A captured iteration replayed several times, with eager library work
    and synchronizations between the replays, equals the eager group after
    every replay."""
    Fa, la, fa = _state(members, "f32")
    Fb, lb, fb = _state(members, "f32")
    tensors = [m[1] for m in members]
    ga = dfacto.Group(ctx, tensors, Fa, la, fa, graph=True, tune=True)
    gb = dfacto.Group(ctx, tensors, Fb, lb, fb, graph=False, tune=False)
    say(f"  tuned: {ga.info()}")
    scratch = torch.empty((members[0][0].dims[0], members[0][2]), device=DEV)
    for rep in range(4):
        ga.als(1)
        gb.als(1)
        # eager work between replays
        dfacto.mttkrp(ctx, tensors[0], 0, Fb[0], scratch)
        torch.cuda.synchronize()
        for k in range(len(members)):
            for m in range(3):
                assert _same(Fa[k][m], Fb[k][m]), f"replay {rep}: member {k} factor {m}"
            assert torch.equal(la[k], lb[k])
        assert torch.equal(fa, fb)
    ga.close()
    gb.close()


@pytest.mark.parametrize("graph", [False, True])
def test_group_on_context_stream(ctx, members, graph):
    """A group launching on its context's stream gives bitwise the results of
    one with its own stream; a context with another stream is refused."""
    Fa, la, fa = _state(members, "bf16")
    Fb, lb, fb = _state(members, "bf16")
    tensors = [m[1] for m in members]
    torch.cuda.synchronize()
    sctx = dfacto.Context(0, stream=torch.cuda.Stream())  # capture needs a created stream
    ga = dfacto.Group(sctx, tensors, Fa, la, fa, graph=graph, ctx_stream=True)
    gb = dfacto.Group(ctx, tensors, Fb, lb, fb)
    for _ in range(3):
        ga.als(1)
        gb.als(1)
    sctx.synchronize()
    torch.cuda.synchronize()
    for k in range(len(members)):
        for m in range(3):
            assert _same(Fa[k][m], Fb[k][m]), f"member {k} factor {m}"
        assert torch.equal(la[k], lb[k])
    assert torch.equal(fa, fb)
    other = dfacto.Context(0, stream=torch.cuda.Stream())
    with pytest.raises(dfacto.DfactoError) as e:
        other.check(dfacto.load().dfacto_group_als(other.handle, ga.handle, 1))
    assert e.value.status == dfacto.E_INVALID
    other.close()
    ga.close()
    gb.close()
    sctx.close()


@pytest.mark.parametrize("graph", [False, True])
def test_group_bf16_reused_grams_bitwise(ctx, members, graph):
    """BF16 storage: iterations after the first of a call, and with
    own_factors every iteration after the group's first, reuse the stored
    factors' Grams of the previous iteration instead of forming them again.
    Four calls of 1, 2, 1 and 3 iterations equal seven dfacto_als_iter calls
    per member, bitwise, with and without graph replay."""
    Fg, lg, fg = _state(members, "bf16")
    Fo, lo, fo = _state(members, "bf16")
    Fs, ls, fs = _state(members, "bf16")
    tensors = [m[1] for m in members]
    g = dfacto.Group(ctx, tensors, Fg, lg, fg, graph=graph)
    go = dfacto.Group(ctx, tensors, Fo, lo, fo, graph=graph, own_factors=True)
    for it in (1, 2, 1, 3):
        g.als(it)
        go.als(it)
        torch.cuda.synchronize()
    for k, (coo, t, R, _) in enumerate(members):
        fit = torch.zeros(1, dtype=torch.float64, device=DEV)
        for _ in range(7):
            dfacto.als_iter(ctx, t, Fs[k], ls[k], fit)
        fs[k] = fit[0]
    torch.cuda.synchronize()
    for k in range(len(members)):
        for m in range(3):
            assert _same(Fg[k][m], Fs[k][m]), f"member {k} factor {m}"
            assert _same(Fo[k][m], Fs[k][m]), f"own_factors: member {k} factor {m}"
        assert torch.equal(lg[k], ls[k]) and torch.equal(lo[k], ls[k])
    assert torch.equal(fg, fs) and torch.equal(fo, fs)
    g.close()
    go.close()


def test_group_tuning_keeps_results(ctx, members):
    """Tuned persistent grid sizes do not change any result."""
    Fa, la, fa = _state(members, "f32")
    Fb, lb, fb = _state(members, "f32")
    tensors = [m[1] for m in members]
    ga = dfacto.Group(ctx, tensors, Fa, la, fa, tune=True)
    gb = dfacto.Group(ctx, tensors, Fb, lb, fb, tune=False)
    say(f"  tuned: {ga.info()['mttkrp_grid']} default: {gb.info()['mttkrp_grid']}")
    ga.als(2)
    gb.als(2)
    torch.cuda.synchronize()
    for k in range(len(members)):
        for m in range(3):
            assert _same(Fa[k][m], Fb[k][m]), f"member {k} factor {m}"
        assert torch.equal(la[k], lb[k])
    assert torch.equal(fa, fb)
    ga.close()
    gb.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_group_every_launch_form(ctx, members, dtype):
    """Every launch form the tuner may pick (columns per lane, lanes per
    group, chunks per lane group), at several persistent grid sizes, gives
    bitwise the default form's iteration; a captured graph is captured
    again after a form changes."""
    Fa, la, fa = _state(members, dtype)
    Fb, lb, fb = _state(members, dtype)
    init = [[f.clone() for f in F] for F in Fa]
    tensors = [m[1] for m in members]
    ga = dfacto.Group(ctx, tensors, Fa, la, fa, graph=True, tune=True)
    gb = dfacto.Group(ctx, tensors, Fb, lb, fb, tune=False)
    inf = ga.info()
    say(f"  {dtype} forms per class {inf['mttkrp_forms']}, tuned cpl {inf['mttkrp_cpl']} "
        f"lanes {inf['mttkrp_lanes']} chunks/group {inf['mttkrp_chunks_per_group']} "
        f"grid {inf['mttkrp_grid']}")
    assert gb.info()["mttkrp_forms"] == [1] * gb.info()["mttkrp_classes"]
    assert max(inf["mttkrp_forms"]) > 1
    seen = set()
    for f in range(max(inf["mttkrp_forms"])):
        grid = (1, 5, 1000)[f % 3]
        for c in range(inf["mttkrp_classes"]):
            ga.set_form(c, min(f, inf["mttkrp_forms"][c] - 1), grid)
        now = ga.info()
        seen.update(zip(now["mttkrp_cpl"], now["mttkrp_lanes"], now["mttkrp_chunks_per_group"]))
        for F, G, I in zip(Fa, Fb, init):
            for m in range(3):
                F[m].copy_(I[m])
                G[m].copy_(I[m])
        ga.als(1)
        gb.als(1)
        torch.cuda.synchronize()
        for k in range(len(members)):
            for m in range(3):
                assert _same(Fa[k][m], Fb[k][m]), f"form {f}: member {k} factor {m}"
            assert torch.equal(la[k], lb[k])
        assert torch.equal(fa, fb)
    say(f"  forms run (cpl, lanes, chunks per group): {sorted(seen)}")
    with pytest.raises(dfacto.DfactoError):
        ga.set_form(inf["mttkrp_classes"], 0, 1)
    with pytest.raises(dfacto.DfactoError):
        ga.set_form(0, inf["mttkrp_forms"][0], 1)
    with pytest.raises(dfacto.DfactoError):
        ga.set_form(0, 0, 0)
    ga.close()
    gb.close()


def test_group_members_match_oracle(ctx, members):
    """One grouped iteration against the FP64 oracle, member by member."""
    Fg, lg, fg = _state(members, "f32")
    g = dfacto.Group(ctx, [m[1] for m in members], Fg, lg, fg)
    g.als(1)
    torch.cuda.synchronize()
    for k, (coo, t, R, F0) in enumerate(members):
        Fw = factors_to_dev(F0, "f32")[1]
        A, B, C, lam_ref, info = oracle.als_iter(*coo.arrays64(), coo.dims, Fw)
        errs = [rel_fro(to_host64(Fg[k][m]), ref) for m, ref in enumerate((A, B, C))]
        say(f"  member {k} R={R}: factor err {max(errs):.2e} fit {fg[k].item():.6f} "
            f"vs {info['fit']:.6f}")
        assert max(errs) <= 1e-5
        assert rel_fro(lg[k].cpu().numpy(), lam_ref) <= 1e-5
        assert abs(fg[k].item() - info["fit"]) <= 1e-4
    g.close()


def test_group_argument_errors(ctx, members):
    coo, t, R, F0 = members[0]
    Fd = factors_to_dev(F0, "f32")[0]
    lam = torch.zeros(R, dtype=torch.float64, device=DEV)
    fits = torch.zeros(1, dtype=torch.float64, device=DEV)
    # a rank without a grouped row map
    F5 = factors_to_dev(gen.init_factors(coo.dims, 5, seed=1), "f32")[0]
    with pytest.raises(dfacto.DfactoError) as e:
        dfacto.Group(ctx, [t], [F5], [torch.zeros(5, dtype=torch.float64, device=DEV)], fits)
    assert e.value.status == dfacto.E_UNSUPPORTED
    # misaligned factors
    buf = torch.empty(Fd[0].numel() + 8, device=DEV)
    mis = buf[1:1 + Fd[0].numel()].view(Fd[0].shape)
    with pytest.raises(dfacto.DfactoError) as e:
        dfacto.Group(ctx, [t], [[mis, Fd[1], Fd[2]]], [lam], fits)
    assert e.value.status == dfacto.E_INVALID
    # the context is still usable
    g = dfacto.Group(ctx, [t], [Fd], [lam], fits)
    g.als(1)
    torch.cuda.synchronize()
    assert np.isfinite(fits.item())
    g.close()
