"""Seeded generator checks (CPU only): determinism, distinctness, ranges and
the Zipf head frequency against its closed form p_1 = 1 / H_{dim,s}."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from paper_1406_4519_amd import gen


def test_uniform_distinct_deterministic_and_distinct():
    a = gen.uniform_distinct((200, 150, 100), 20_000, seed=1)
    b = gen.uniform_distinct((200, 150, 100), 20_000, seed=1)
    for x, y in ((a.i, b.i), (a.j, b.j), (a.k, b.k), (a.val, b.val)):
        np.testing.assert_array_equal(x, y)
    assert a.val.dtype == np.float32 and a.i.dtype == np.uint32
    lin = (a.i.astype(np.int64) * 150 + a.j) * 100 + a.k
    assert len(np.unique(lin)) == 20_000
    assert a.i.max() < 200 and a.j.max() < 150 and a.k.max() < 100
    c = gen.uniform_distinct((200, 150, 100), 20_000, seed=2)
    assert not np.array_equal(a.i, c.i)


def test_zipf_distinct_counts_and_determinism():
    dims = (5000, 3000, 2000)
    a = gen.zipf_distinct(dims, 200_000, 1.1, seed=5)
    b = gen.zipf_distinct(dims, 200_000, 1.1, seed=5)
    np.testing.assert_array_equal(a.i, b.i)
    np.testing.assert_array_equal(a.val, b.val)
    lin = (a.i.astype(np.int64) * dims[1] + a.j) * dims[2] + a.k
    assert len(np.unique(lin)) == 200_000
    assert (a.val >= 0).all()
    assert a.i.max() < dims[0] and a.j.max() < dims[1] and a.k.max() < dims[2]


def test_zipf_head_frequency():
    dim, s, n = 10_000, 1.1, 2_000_000
    cdf = gen.zipf_cdf(dim, s)
    rng = np.random.Generator(np.random.PCG64(9))
    with ThreadPoolExecutor(4) as pool:
        r = gen._draw_ranks(cdf, rng.random(n), pool)
    H = float(np.sum(np.arange(1, dim + 1, dtype=np.float64) ** -s))
    for rank in (1, 2, 10):
        p = rank ** -s / H
        got = float(np.mean(r == rank - 1))
        assert abs(got - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_bf16_rounding_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0], dtype=np.float32)
    y = gen.bf16_to_f32(gen.f32_to_bf16(x))
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to the even (1.0)
    np.testing.assert_array_equal(y, np.array([1.0, 1.0, 1.0 + 2 ** -6, -2.5, 0.0], np.float32))


def test_batched_specs_in_range():
    for t in range(16):
        dims, nnz, R, s1, s2 = gen.batched_spec(t)
        assert all(1000 <= d <= 100_000 for d in dims)
        assert 10_000 <= nnz <= 5_000_000 or nnz == (dims[0] * dims[1] * dims[2]) // 2
        assert R in (8, 16, 32)


def test_zipf_distinct_torch_counts_classes_and_determinism():
    """The torch recipe (used for the 1.2B-nonzero paper shape) gives exactly
    nnz distinct in-range coordinates, deterministically, with and without
    the split of the key space into classes."""
    import torch

    dims = (300, 200, 100)
    for bits in (63, 16):  # 16 bits: keys split over i mod 100 classes
        a = gen.zipf_distinct_torch(dims, 20_000, 1.1, seed=5, batch=4096, max_key_bits=bits)
        b = gen.zipf_distinct_torch(dims, 20_000, 1.1, seed=5, batch=4096, max_key_bits=bits)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        i, j, k, v = a
        assert i.dtype == torch.int32 and v.dtype == torch.float32 and i.numel() == 20_000
        assert 0 <= int(i.min()) and int(i.max()) < dims[0]
        assert 0 <= int(j.min()) and int(j.max()) < dims[1]
        assert 0 <= int(k.min()) and int(k.max()) < dims[2]
        lin = (i.long() * dims[1] + j.long()) * dims[2] + k.long()
        assert torch.unique(lin).numel() == 20_000
        assert bool((v >= 0).all())
    # skew: the most frequent mode-0 index holds far more than a uniform share
    counts = torch.bincount(a[0].long(), minlength=dims[0])
    assert int(counts.max()) > 5 * 20_000 / dims[0]


def test_preferential_attachment_matches_the_urn():
    """The preferential-attachment sampler (Dirichlet(1) weights, then i.i.d.
    draws) has the urn's law: the count at one index after n draws over I
    indices is Beta-Binomial(n, 1, I - 1), variance n (I-1)(n+I) / (I^2 (I+1)),
    ten times the variance of independent uniform draws here; a direct
    sequential urn (weight = nonzeros at the index + 1) agrees as well."""
    I, n, reps = 20, 200, 3000
    rng = np.random.default_rng(21)
    var_bb = n * (I - 1) * (n + I) / (I * I * (I + 1))
    counts = np.empty(reps)
    for t in range(reps):
        cdf = gen.preferential_cdf(I, rng)
        r = np.minimum(np.searchsorted(cdf, rng.random(n), side="right"), I - 1)
        counts[t] = np.sum(r == 0)
    assert abs(counts.mean() - n / I) < 0.1 * n / I
    assert abs(counts.var() - var_bb) < 0.15 * var_bb
    urn = np.empty(reps)
    for t in range(reps):
        w = np.ones(I)
        for _ in range(n):
            i = min(int(np.searchsorted(np.cumsum(w), rng.random() * w.sum(), side="right")), I - 1)
            w[i] += 1.0
        urn[t] = w[0] - 1.0
    assert abs(urn.var() - var_bb) < 0.15 * var_bb


def test_preferential_distinct_counts_and_determinism():
    dims = (2000, 2000, 2000)
    a = gen.preferential_distinct(dims, 50_000, seed=8)
    b = gen.preferential_distinct(dims, 50_000, seed=8)
    for x, y in ((a.i, b.i), (a.j, b.j), (a.k, b.k), (a.val, b.val)):
        np.testing.assert_array_equal(x, y)
    lin = (a.i.astype(np.int64) * dims[1] + a.j) * dims[2] + a.k
    assert len(np.unique(lin)) == 50_000
    assert a.i.max() < dims[0] and a.j.max() < dims[1] and a.k.max() < dims[2]
    assert (a.val >= 0).all()
