"""Relabeled gathers.

A relabeled build stores each gathered row's rank in the order of
decreasing gather count instead of its index, and the MTTKRP reads the
factors through copies permuted into that order.  The nonzeros' order,
every chunk's arithmetic and every value gathered are the same, so results
must be BITWISE equal to those of a plain build -- for every rank class and
storage dtype, for ALS, GD and grouped ALS -- and the flattening exported
back to factor rows must equal the plain one exactly.  The oracle
comparison at the end checks the common answer itself."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import build, factors_to_dev, rel_fro, say, to_host64, DEV
from paper_1406_4519_amd import dfacto, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = dfacto.Context(0)
    coo = gen.zipf_distinct((6000, 4000, 2500), 400_000, 1.1, seed=61)
    plain = build(ctx, coo, relabel=False)
    rel = build(ctx, coo, relabel=True)
    assert rel.info()["relabeled"] and not plain.info()["relabeled"]
    yield ctx, coo, plain, rel
    plain.close()
    rel.close()
    ctx.close()


def _bits(x):
    return x.view(torch.int16) if x.dtype == torch.bfloat16 else x


def test_relabeled_structure_exports_the_same(pair):
    ctx, coo, plain, rel = pair
    a, b = plain.info(), rel.info()
    for key in ("nnz", "nfib", "nroot", "nentry", "nchunk"):
        assert a[key] == b[key], key
    for m in range(3):
        ea, eb = dfacto.tensor_export(ctx, plain, m), dfacto.tensor_export(ctx, rel, m)
        for key in ea:
            assert np.array_equal(ea[key], eb[key]), (m, key)


@pytest.mark.parametrize("R", [1, 3, 8, 10, 16, 32, 64, 100])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_relabeled_mttkrp_bitwise(pair, R, dtype):
    ctx, coo, plain, rel = pair
    Fd, _ = factors_to_dev(gen.init_factors(coo.dims, R, seed=62 + R), dtype)
    for m in range(3):
        ref = dfacto.mttkrp(ctx, plain, m, Fd)
        got = dfacto.mttkrp(ctx, rel, m, Fd)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (m, R, dtype)


def test_relabeled_misaligned_factors_bitwise(pair):
    ctx, coo, plain, rel = pair
    R = 16
    Fd, _ = factors_to_dev(gen.init_factors(coo.dims, R, seed=70), "f32")
    mis = []
    for f in Fd:  # rows start 4 bytes past a 16-byte boundary
        buf = torch.empty(f.numel() + 8, device=DEV)
        v = buf[1:1 + f.numel()].view(f.shape)
        v.copy_(f)
        mis.append(v)
    for m in range(3):
        assert torch.equal(dfacto.mttkrp(ctx, plain, m, mis), dfacto.mttkrp(ctx, rel, m, mis))


@pytest.mark.parametrize("R,dtype", [(32, "f32"), (10, "f32"), (16, "bf16")])
def test_relabeled_als_gd_bitwise(pair, R, dtype):
    ctx, coo, plain, rel = pair
    F0 = gen.init_factors(coo.dims, R, seed=80 + R)
    res = []
    for t in (plain, rel):
        Fd, _ = factors_to_dev(F0, dtype)
        lam = torch.zeros(R, dtype=torch.float64, device=DEV)
        fit = torch.zeros(1, dtype=torch.float64, device=DEV)
        for _ in range(2):
            dfacto.als_iter(ctx, t, Fd, lam, fit)
        G = [torch.empty((d, R), device=DEV) for d in coo.dims]
        f = torch.zeros(1, dtype=torch.float64, device=DEV)
        dfacto.gd_grad(ctx, t, Fd, G, f)
        torch.cuda.synchronize()
        res.append((Fd, lam, fit, G, f))
    (Fa, la, fa, Ga, fva), (Fb, lb, fb, Gb, fvb) = res
    for x, y in zip((*Fa, la, fa, *Ga, fva), (*Fb, lb, fb, *Gb, fvb)):
        assert torch.equal(_bits(x), _bits(y))


@pytest.mark.parametrize("R,dtype", [(16, "f32"), (32, "bf16")])
def test_relabeled_group_member_bitwise(pair, R, dtype):
    """A relabeled tensor in a group gives the single-call results of the
    plain build (BF16 at R = 32: eight columns per lane for the relabeled
    member, four for the plain single call)."""
    ctx, coo, plain, rel = pair
    other = gen.zipf_distinct((900, 700, 500), 30_000, 1.1, seed=63)
    t2 = build(ctx, other)
    F0a = gen.init_factors(coo.dims, R, seed=64)
    F0b = gen.init_factors(other.dims, R, seed=65)
    Fa, _ = factors_to_dev(F0a, dtype)
    Fb, _ = factors_to_dev(F0b, dtype)
    lams = [torch.zeros(R, dtype=torch.float64, device=DEV) for _ in range(2)]
    fits = torch.zeros(2, dtype=torch.float64, device=DEV)
    g = dfacto.Group(ctx, [rel, t2], [Fa, Fb], lams, fits, graph=True)
    g.als(3)
    torch.cuda.synchronize()
    Fs, _ = factors_to_dev(F0a, dtype)
    lam = torch.zeros(R, dtype=torch.float64, device=DEV)
    fit = torch.zeros(1, dtype=torch.float64, device=DEV)
    for _ in range(3):
        dfacto.als_iter(ctx, plain, Fs, lam, fit)
    torch.cuda.synchronize()
    for x, y in zip(Fa, Fs):
        assert torch.equal(_bits(x), _bits(y))
    assert torch.equal(lams[0], lam) and fits[0].item() == fit.item()
    g.close()
    t2.close()


def test_relabeled_matches_oracle(pair):
    ctx, coo, plain, rel = pair
    R = 32
    F0 = gen.init_factors(coo.dims, R, seed=66)
    Fd, Fw = factors_to_dev(F0, "f32")
    for m in range(3):
        got = to_host64(dfacto.mttkrp(ctx, rel, m, Fd))
        ref = oracle.mttkrp(*coo.arrays64(), coo.dims, Fw, m)
        err = rel_fro(got, ref)
        say(f"  relabeled mode {m}: rel err {err:.2e}")
        assert err <= 1e-5


def test_relabel_order_follows_gather_counts(pair):
    """The relabel order of each mode's tables is the exact order of
    decreasing gather count, ties by row index: leaf rows counted by their
    nonzeros, mid rows by the fiber segment headers that gather them (a fiber
    of L nonzeros has ceil(L / 128) segments), counted here on the host."""
    ctx, coo, plain, rel = pair
    coords = (coo.i.astype(np.int64), coo.j.astype(np.int64), coo.k.astype(np.int64))
    for m in range(3):
        root, mid, leaf = coords[m], coords[(m + 2) % 3], coords[(m + 1) % 3]
        dl, dm = coo.dims[(m + 1) % 3], coo.dims[(m + 2) % 3]
        cnt_leaf = np.bincount(leaf, minlength=dl)
        fib, flen = np.unique(root * dm + mid, return_counts=True)
        cnt_mid = np.bincount(fib % dm, weights=-(-flen // 128), minlength=dm).astype(np.int64)
        for table, cnt in ((0, cnt_leaf), (1, cnt_mid)):
            want = np.lexsort((np.arange(len(cnt)), -cnt))
            got = dfacto.gather_order(ctx, rel, m, table)
            assert np.array_equal(got, want), (m, table)
    with pytest.raises(dfacto.DfactoError):
        dfacto.gather_order(ctx, plain, 0, 0)  # not relabeled


def test_relabel_by_size_and_flags(pair):
    """dfacto_build_flattenings relabels from 2^23 nonzeros on when there are
    at least 64 nonzeros per factor row, and contradictory flags or chunk
    lengths out of range are refused."""
    ctx, coo, plain, rel = pair
    from gpu_util import coo_to_dev
    i, j, k, v = coo_to_dev(coo)
    t = dfacto.build_flattenings(ctx, coo.dims, i, j, k, v)
    assert not t.info()["relabeled"]  # 400K nonzeros
    t.close()
    for dims, want in (((1000, 1000, 1000), True), ((200_000, 100_000, 50_000), False)):
        gi, gj, gk, gv = gen.zipf_distinct_torch(dims, 9_000_000, 1.1, seed=63, device=DEV)
        t = dfacto.build_flattenings(ctx, dims, gi, gj, gk, gv)
        assert t.info()["relabeled"] == want, dims  # 9M nonzeros: 3000 / 26 per row
        t.close()
        del gi, gj, gk, gv
    import ctypes
    lib = dfacto.load()
    d = (ctypes.c_int64 * 3)(*coo.dims)
    h = ctypes.c_void_p()
    st = lib.dfacto_build_flattenings_ex(ctx.handle, d, int(v.numel()), i.data_ptr(), j.data_ptr(),
                                         k.data_ptr(), v.data_ptr(), 3, 0, ctypes.byref(h))
    assert st == dfacto.E_INVALID and not h.value
    for bad in (100, 255, (1 << 20) + 1):  # chunk lengths out of range
        st = lib.dfacto_build_flattenings_ex(ctx.handle, d, int(v.numel()), i.data_ptr(),
                                             j.data_ptr(), k.data_ptr(), v.data_ptr(), 0, bad,
                                             ctypes.byref(h))
        assert st == dfacto.E_INVALID and not h.value
