"""The oracle's threaded loops (oracle.config(threads)) against the serial
ones: every result bitwise equal.  Threads split only independent work
(disjoint output rows, Gram entries, solve rows, columns) and keep every
sum in its serial order, so any difference is a bug in that split."""
import numpy as np
import pytest

import oracle
from paper_1406_4519_amd import gen


@pytest.fixture(autouse=True)
def serial_after():
    yield
    oracle.config(1, False)


def _tensor(dup: bool):
    # above the threaded paths' thresholds: 200K nonzeros, 5000+ rows
    coo = gen.zipf_distinct((6000, 5000, 4500), 200_000, 1.1, seed=71)
    i, j, k, v = coo.arrays64()
    if dup:  # repeat 1000 coordinates with new values
        rng = np.random.default_rng(3)
        pick = rng.choice(len(v), 1000, replace=False)
        i, j, k = (np.concatenate([a, a[pick]]) for a in (i, j, k))
        v = np.concatenate([v, rng.standard_normal(1000)])
    return coo.dims, i, j, k, v


def _both(fn):
    oracle.config(1, False)
    a = fn()
    oracle.config(5, False)
    b = fn()
    return a, b


def _eq(a, b):
    if isinstance(a, (tuple, list)):
        assert len(a) == len(b)
        for x, y in zip(a, b):
            _eq(x, y)
    elif isinstance(a, dict):
        for key in a:
            _eq(a[key], b[key])
    else:
        assert np.array_equal(np.asarray(a), np.asarray(b)), (a, b)


@pytest.mark.parametrize("dup", [False, True])
@pytest.mark.parametrize("R", [3, 16])
def test_threads_mttkrp_inner_normsq(dup, R):
    dims, i, j, k, v = _tensor(dup)
    F = gen.init_factors(dims, R, seed=72)
    for m in range(3):
        _eq(*_both(lambda: oracle.mttkrp(i, j, k, v, dims, F, m)))
    _eq(*_both(lambda: oracle.inner(i, j, k, v, F)))
    _eq(*_both(lambda: oracle.normsq(i, j, k, v)))


@pytest.mark.parametrize("store", ["f64", "bf16"])
@pytest.mark.parametrize("reg", [0.0, 0.4])
def test_threads_als_iter(store, reg):
    dims, i, j, k, v = _tensor(True)
    F = gen.init_factors(dims, 12, seed=73)
    _eq(*_both(lambda: oracle.als_iter(i, j, k, v, dims, F, reg, store=store)))


def test_threads_als_pinv_and_gd():
    dims, i, j, k, v = _tensor(False)
    F = gen.init_factors(dims, 6, seed=74)
    F[1][:, 5] = F[1][:, 4]  # singular Gram: the pseudo-inverse path
    F[2][:, 5] = F[2][:, 4]
    a, b = _both(lambda: oracle.als_iter(i, j, k, v, dims, F))
    assert a[4]["pinv_mask"] & 1
    _eq(a, b)
    _eq(*_both(lambda: oracle.gd_grad(i, j, k, v, dims, F, 0.2)))


def test_distinct_normsq_is_the_plain_sum():
    """With distinct coordinates declared, ||X||^2 is the sum of squares in
    input order; it equals the merged sum up to the order of additions."""
    dims, i, j, k, v = _tensor(False)
    ref = oracle.normsq(i, j, k, v)
    oracle.config(4, True)
    got = oracle.normsq(i, j, k, v)
    assert abs(got - ref) <= 1e-12 * ref
    s = 0.0
    for x in v:
        s += x * x
    assert got == s
