"""Seeded synthetic inputs for the DFacTo hot path.

This module only draws coordinates, values and initial factors; it contains
none of the factorization arithmetic.  Both the HIP library's tests/benchmark
and the FP64 oracle consume exactly the arrays produced here.

Every generator is deterministic in its seed (numpy ``PCG64``).

Recipes (the paper's own datasets -- Amazon reviews, NELL, etc. of
Section 5, Table 1 -- are not available; these stand in for their shape,
size and skew):

* ``uniform_distinct``: ``nnz`` distinct linear indices drawn without
  replacement from ``[0, I*J*K)`` and split by mixed radix into (i, j, k);
  values N(0, 1) rounded to FP32.
* ``zipf_distinct``: per mode, rank r in 1..dim has probability
  proportional to r^-s (inverse-CDF draw over an FP64 cumulative table),
  and rank r maps to index ``perm_m[r-1]`` of a seeded permutation, so the
  heavy indices are scattered over the index range.  The three modes are
  drawn independently; draws continue until ``nnz`` *distinct* coordinates
  exist and the first draw of a coordinate supplies its value.  Values are
  |N(0,1)| rounded to FP32 (the paper's tensors hold positive counts).
* ``preferential_distinct``: the paper's synthetic model (Section 5):
  index i of a mode is drawn with probability proportional to the number of
  nonzeros already at i, plus an initial weight 1 per index (the model
  leaves unused indices at zero otherwise).  The draws of that urn are
  exchangeable with Dirichlet(1, ..., 1) weights, so each mode draws its
  weights once and then i.i.d. indices; draws continue until ``nnz``
  distinct coordinates exist, |N(0,1)| FP32 values.
* ``zipf_distinct_torch``: the same per-mode Zipf(s) draw for tensors too
  large to deduplicate on the host (the 1.2B-nonzero paper shape), in torch
  on a given device (``torch.Generator``, Philox on the GPU): draws continue
  in batches until at least ``nnz`` distinct coordinates exist, then a
  seeded uniform choice of exactly ``nnz`` of them is kept; values |N(0,1)|
  FP32.  Its stream differs from the numpy recipes and between devices.
* ``planted_dense`` / ``planted_sparse``: exact low-rank tensors
  sum_r a_r o b_r o c_r with every entry of the (union) support stored.
* ``init_factors``: U(0, 1) in FP64, drawn in the order A, B, C.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np


@dataclass
class Coo:
    """A 3-way sparse tensor in coordinate format (0-based indices)."""

    dims: tuple
    i: np.ndarray  # uint32
    j: np.ndarray  # uint32
    k: np.ndarray  # uint32
    val: np.ndarray  # float32 (what the device receives)

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])

    def val64(self) -> np.ndarray:
        """Values widened to FP64 for the oracle (same numbers as the device)."""
        return self.val.astype(np.float64)

    def arrays64(self):
        return self.i, self.j, self.k, self.val64()


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def uniform_distinct(dims, nnz: int, seed: int) -> Coo:
    I, J, K = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    lin = rng.choice(I * J * K, size=nnz, replace=False).astype(np.int64)
    i = (lin // (J * K)).astype(np.uint32)
    j = ((lin // K) % J).astype(np.uint32)
    k = (lin % K).astype(np.uint32)
    val = rng.standard_normal(nnz).astype(np.float32)
    return Coo((I, J, K), i, j, k, val)


def zipf_cdf(dim: int, s: float) -> np.ndarray:
    w = np.arange(1, dim + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)
    c /= c[-1]
    c[-1] = 1.0
    return c


def _draw_ranks(cdf: np.ndarray, u: np.ndarray, pool: ThreadPoolExecutor) -> np.ndarray:
    parts = np.array_split(u, max(1, 4 * pool._max_workers))
    out = list(pool.map(lambda c: np.searchsorted(cdf, c, side="right"), parts))
    r = np.concatenate(out)
    np.minimum(r, len(cdf) - 1, out=r)
    return r


def _first_occurrences(keys: np.ndarray, pool: ThreadPoolExecutor,
                       lo: np.ndarray | None = None) -> np.ndarray:
    """Sorted positions of the first occurrence of every distinct key (keys
    alone, or the pairs (keys, lo) when the coordinate needs two words)."""
    nb = 16
    h = keys if lo is None else (keys * np.uint64(0xD6E8FEB86659FD93)) ^ lo
    bucket = ((h * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(60)).astype(np.uint8)

    def one(b):
        pos = np.flatnonzero(bucket == b)
        if lo is None:
            kb = keys[pos]
            order = np.argsort(kb, kind="stable")
            ks = kb[order]
            first = np.ones(len(ks), dtype=bool)
            if len(ks) > 1:
                first[1:] = ks[1:] != ks[:-1]
        else:
            kh, kl = keys[pos], lo[pos]
            order = np.lexsort((kl, kh))  # stable: equal pairs keep draw order
            sh, sl = kh[order], kl[order]
            first = np.ones(len(order), dtype=bool)
            if len(order) > 1:
                first[1:] = (sh[1:] != sh[:-1]) | (sl[1:] != sl[:-1])
        return pos[order[first]]

    if len(keys) > 400_000_000:  # bound the memory of concurrent buckets
        parts = []
        for g in range(0, nb, 4):
            parts.extend(pool.map(one, range(g, g + 4)))
    else:
        parts = list(pool.map(one, range(nb)))
    return np.sort(np.concatenate(parts))


def zipf_distinct(dims, nnz: int, s: float, seed: int, values: str = "absnormal",
                  progress=None) -> Coo:
    I, J, K = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    cdfs = [zipf_cdf(d, s) for d in (I, J, K)]
    perms = [rng.permutation(d).astype(np.uint32) for d in (I, J, K)]
    return _distinct_from_cdfs((I, J, K), nnz, cdfs, perms, rng, values, progress, "zipf")


def preferential_cdf(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Cumulative weights of one mode of the preferential-attachment model
    with initial weight 1 per index: draw i is index i with probability
    proportional to (nonzeros already at i) + 1.  That Polya urn's draws are
    exchangeable with de Finetti measure Dirichlet(1, ..., 1), so drawing
    weights w ~ Dirichlet(1, ..., 1) (normalized Exp(1) variables) once and
    then i.i.d. indices from w gives the urn's law exactly."""
    w = rng.standard_exponential(dim)
    c = np.cumsum(w)
    c /= c[-1]
    c[-1] = 1.0
    return c


def preferential_distinct(dims, nnz: int, seed: int, values: str = "absnormal",
                          progress=None) -> Coo:
    I, J, K = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    cdfs = [preferential_cdf(d, rng) for d in (I, J, K)]
    return _distinct_from_cdfs((I, J, K), nnz, cdfs, None, rng, values, progress, "preferential")


def _distinct_from_cdfs(dims, nnz, cdfs, perms, rng, values, progress, label) -> Coo:
    """Draw (i, j, k) independently per mode from the cumulative tables
    (index = perms[m][rank] when perms is given) until nnz distinct
    coordinates exist; the first draw of a coordinate supplies its value."""
    I, J, K = dims
    if I * J * K < nnz:
        raise ValueError("more distinct nonzeros requested than cells")
    wide = float(I) * J * K >= 2.0 ** 63  # key = (i, j K + k) in two words
    if wide and float(J) * K >= 2.0 ** 63:
        raise ValueError("tensor too large for the coordinate key")
    pool = ThreadPoolExecutor(_workers())
    try:
        idx = [np.empty(0, np.uint32) for _ in range(3)]
        vals = np.empty(0, np.float32)
        draw = int(nnz * 1.25) + 1024
        while True:
            new = []
            for m in range(3):
                u = rng.random(draw)
                r = _draw_ranks(cdfs[m], u, pool)
                new.append(perms[m][r] if perms is not None else r.astype(np.uint32))
                del u, r
                if progress is not None:
                    progress(f"{label} draw: mode {m}, {draw:,} samples")
            if values == "absnormal":
                v = np.abs(rng.standard_normal(draw)).astype(np.float32)
            elif values == "normal":
                v = rng.standard_normal(draw).astype(np.float32)
            else:
                raise ValueError(values)
            idx = [np.concatenate([idx[m], new[m]]) for m in range(3)]
            vals = np.concatenate([vals, v])
            if wide:
                keys = idx[0].astype(np.uint64)
                lo = idx[1].astype(np.uint64) * np.uint64(K) + idx[2].astype(np.uint64)
                first = _first_occurrences(keys, pool, lo)
                del lo
            else:
                keys = (idx[0].astype(np.uint64) * np.uint64(J) + idx[1].astype(np.uint64)) \
                    * np.uint64(K) + idx[2].astype(np.uint64)
                first = _first_occurrences(keys, pool)
            if progress is not None:
                progress(f"{label} draw: {len(keys):,} coordinates, {len(first):,} distinct")
            if len(first) >= nnz:
                sel = first[:nnz]
                return Coo((I, J, K), idx[0][sel].copy(), idx[1][sel].copy(),
                           idx[2][sel].copy(), vals[sel].copy())
            # grow the next batch from the observed distinct yield
            got = len(first)
            rate = max(got / len(keys), 1e-3)
            draw = int((nnz - got) / rate * 1.2) + 1024
    finally:
        pool.shutdown()


def zipf_draws(dims, n: int, s: float, seed: int, progress=None) -> Coo:
    """n coordinates drawn independently per mode from Zipf(s) over a seeded
    permutation of each mode, |N(0,1)| values, duplicates kept (the
    flattening build sums them)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cdfs = [zipf_cdf(int(d), s) for d in dims]
    perms = [rng.permutation(int(d)).astype(np.uint32) for d in dims]
    pool = ThreadPoolExecutor(_workers())
    try:
        idx = []
        for m in range(3):
            u = rng.random(n)
            idx.append(perms[m][_draw_ranks(cdfs[m], u, pool)])
            del u
            if progress is not None:
                progress(f"zipf draws: mode {m}, {n:,} samples")
        val = np.abs(rng.standard_normal(n, dtype=np.float32))
    finally:
        pool.shutdown()
    return Coo(tuple(int(d) for d in dims), idx[0], idx[1], idx[2], val)


def zipf_distinct_torch(dims, nnz: int, s: float, seed: int, device="cpu",
                        batch: int = 1 << 27, max_key_bits: int = 63, progress=None):
    """nnz distinct coordinates with Zipf(s) marginals over a seeded
    permutation of each mode, generated with torch on ``device``.

    Coordinates are deduplicated as integer keys.  When I*J*K does not fit
    ``max_key_bits`` bits the coordinates are split into classes by
    i mod ncls and each class keys (i // ncls, j, k), so every key fits.
    Returns (i, j, k) as int32 tensors and |N(0,1)| FP32 values on
    ``device``, sorted by (class, key)."""
    import torch

    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    I, J, K = (int(d) for d in dims)
    if nnz > I * J * K:
        raise ValueError("more distinct coordinates than cells")
    cdfs = [torch.from_numpy(zipf_cdf(d, s)).to(dev) for d in (I, J, K)]
    perms = [torch.randperm(d, generator=g, device=dev) for d in (I, J, K)]
    JK = J * K
    lim = (1 << max_key_bits) - 1
    if JK - 1 > lim:
        raise ValueError("J*K exceeds the key range")
    ncls = 1
    while ((I + ncls - 1) // ncls) * JK - 1 > lim:
        ncls += 1
    uniq = [torch.empty(0, dtype=torch.int64, device=dev) for _ in range(ncls)]
    total, drawn = 0, 0
    while total < nnz:
        idx = []
        for m, d in enumerate((I, J, K)):
            u = torch.rand(batch, generator=g, device=dev, dtype=torch.float64)
            r = torch.searchsorted(cdfs[m], u, right=True).clamp_(max=d - 1)
            del u
            idx.append(perms[m][r])
            del r
        lo = idx[1] * K + idx[2]
        cls = idx[0] % ncls
        hi = idx[0] // ncls
        del idx
        for c in range(ncls):
            sel = cls == c
            uniq[c] = torch.unique(torch.cat([uniq[c], hi[sel] * JK + lo[sel]]))
            del sel
        del lo, cls, hi
        drawn += batch
        total = sum(int(x.numel()) for x in uniq)
        if progress is not None:
            progress(f"zipf draws: {drawn:,} drawn, {total:,} distinct")
    # a seeded uniform choice of exactly nnz of the distinct coordinates
    keep = torch.randperm(total, generator=g, device=dev)[:nnz].sort().values
    ii, jj, kk = [], [], []
    for c in range(ncls):
        key = uniq[c]
        uniq[c] = None
        ii.append(((key // JK) * ncls + c).to(torch.int32))
        rem = key % JK
        del key
        jj.append((rem // K).to(torch.int32))
        kk.append((rem % K).to(torch.int32))
        del rem
    out = []
    for parts in (ii, jj, kk):
        a = torch.cat(parts)
        parts.clear()
        out.append(a[keep])
        del a
    del keep
    val = torch.randn(nnz, generator=g, device=dev, dtype=torch.float32).abs_()
    return out[0], out[1], out[2], val


def planted_factors(dims, R: int, seed: int, density: float = 1.0):
    """N(0,1) factors; with density < 1 each column keeps that fraction of
    rows (chosen at random) and is zero elsewhere."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for d in dims:
        F = rng.standard_normal((int(d), R))
        if density < 1.0:
            keep = rng.random((int(d), R)) < density
            for r in range(R):  # never leave a column empty
                if not keep[:, r].any():
                    keep[rng.integers(0, int(d)), r] = True
            F = F * keep
        out.append(F)
    return out


def planted_dense(dims, R: int, seed: int) -> tuple:
    """Dense exact rank-R tensor with all I*J*K entries stored.
    Returns (Coo with FP32 values, factors, values in FP64)."""
    A, B, C = planted_factors(dims, R, seed)
    X = np.einsum("ir,jr,kr->ijk", A, B, C)
    I, J, K = X.shape
    ii, jj, kk = np.meshgrid(np.arange(I), np.arange(J), np.arange(K), indexing="ij")
    coo = Coo((I, J, K), ii.ravel().astype(np.uint32), jj.ravel().astype(np.uint32),
              kk.ravel().astype(np.uint32), X.ravel().astype(np.float32))
    return coo, (A, B, C), X.ravel().copy()


def planted_dense_noisy(dims, R: int, seed: int, noise: float) -> tuple:
    """Dense rank-R tensor plus Gaussian noise, all I*J*K entries stored:
    x = model + noise * rms(model) * N(0,1), so a rank-R fit leaves about
    noise^2 / (1 + noise^2) of ||X||^2 unexplained.  Returns (Coo with FP32
    values, factors)."""
    A, B, C = planted_factors(dims, R, seed)
    X = np.einsum("ir,jr,kr->ijk", A, B, C)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    X = X + noise * np.sqrt(np.mean(X * X)) * rng.standard_normal(X.shape)
    I, J, K = X.shape
    ii, jj, kk = np.meshgrid(np.arange(I), np.arange(J), np.arange(K), indexing="ij")
    coo = Coo((I, J, K), ii.ravel().astype(np.uint32), jj.ravel().astype(np.uint32),
              kk.ravel().astype(np.uint32), X.ravel().astype(np.float32))
    return coo, (A, B, C)


def planted_sparse(dims, R: int, seed: int, density: float = 0.2) -> tuple:
    """Exact rank-R tensor whose factor columns are ``density``-sparse; every
    entry of the union of the R rank-one supports is stored (zeros included
    where columns cancel).  Returns (Coo, factors, values in FP64)."""
    A, B, C = planted_factors(dims, R, seed, density)
    I, J, K = (int(d) for d in dims)
    cells = set()
    for r in range(R):
        ia, jb, kc = np.flatnonzero(A[:, r]), np.flatnonzero(B[:, r]), np.flatnonzero(C[:, r])
        g = np.stack(np.meshgrid(ia, jb, kc, indexing="ij"), -1).reshape(-1, 3)
        cells.update(map(tuple, g.tolist()))
    cells = np.array(sorted(cells), dtype=np.int64).reshape(-1, 3)
    x = np.einsum("er,er,er->e", A[cells[:, 0]], B[cells[:, 1]], C[cells[:, 2]])
    coo = Coo((I, J, K), cells[:, 0].astype(np.uint32), cells[:, 1].astype(np.uint32),
              cells[:, 2].astype(np.uint32), x.astype(np.float32))
    return coo, (A, B, C), x


def init_factors(dims, R: int, seed: int):
    """U(0,1) FP64 factors drawn in the order A, B, C."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.random((int(d), R)) for d in dims]


def round_factors(factors, dtype: str):
    """Factors as the device stores them ("f32" or "bf16"), widened back to
    FP64 so the oracle sees the same numbers.  BF16 rounding is
    round-to-nearest-even on the FP32 bit pattern."""
    out = []
    for F in factors:
        f32 = np.ascontiguousarray(F, dtype=np.float32)
        if dtype == "f32":
            out.append(f32.astype(np.float64))
        elif dtype == "bf16":
            out.append(bf16_to_f32(f32_to_bf16(f32)).astype(np.float64))
        else:
            raise ValueError(dtype)
    return out


def f32_to_bf16(x: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns (uint16), round to nearest even."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = ((b >> np.uint64(16)) & np.uint64(1)) + np.uint64(0x7FFF)
    return ((b + rounding) >> np.uint64(16)).astype(np.uint16)


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def small_uniform():
    """200 x 150 x 100, 20,000 distinct uniform coordinates, N(0,1), R = 8."""
    coo = uniform_distinct((200, 150, 100), 20_000, seed=1)
    return coo, 8, init_factors(coo.dims, 8, seed=1001)


def zipf_50m():
    """1M x 500K x 200K, 50M distinct Zipf(1.1) coordinates, |N(0,1)|, R = 32."""
    coo = zipf_distinct((1_000_000, 500_000, 200_000), 50_000_000, 1.1, seed=2)
    return coo, 32, init_factors(coo.dims, 32, seed=1002)


def batched_spec(t: int):
    """Shape of batched tensor t: dims log-uniform in [1e3, 1e5] per mode,
    nnz log-uniform in [1e4, 5e6] (capped at half the cells), R from
    {8, 16, 32}.  Returns (dims, nnz, R, data seed, init seed)."""
    rng = np.random.Generator(np.random.PCG64(4000 + t))
    dims = tuple(int(round(10 ** rng.uniform(3, 5))) for _ in range(3))
    nnz = int(round(10 ** rng.uniform(4, math.log10(5e6))))
    nnz = min(nnz, (dims[0] * dims[1] * dims[2]) // 2)
    R = int(rng.choice([8, 16, 32]))
    return dims, nnz, R, 4000 + t, 14000 + t


def batched_tensor(t: int):
    dims, nnz, R, s1, s2 = batched_spec(t)
    coo = zipf_distinct(dims, nnz, 1.1, seed=s1)
    return coo, R, init_factors(dims, R, seed=s2)
