"""Pins for the oracle's full GD iteration (Algorithm 5: gradients, a
backtracking line search, the simultaneous update) and its objective (CPU
only).  Independent references: the dense brute-force objective
1/2 ||X - [[A,B,C]]||^2 + 1/2 reg sum ||F||^2 over every (i, j, k), the
line-search decision recomputed from that dense objective, BF16 storage
rounding by bit manipulation, and descent on a planted exact tensor."""
import numpy as np
import pytest

import brute
import oracle
from paper_1406_4519_amd import gen


@pytest.mark.parametrize("reg", [0.0, 0.7])
def test_objective_matches_dense_brute_force(reg):
    rng = np.random.default_rng(11)
    dims = (6, 5, 4)
    i, j, k, val = brute.random_coo(rng, dims, 40, dup=5)
    F = [rng.standard_normal((d, 3)) for d in dims]
    X = brute.dense(dims, i, j, k, val)
    got = oracle.objective(i, j, k, val, dims, F, reg)
    np.testing.assert_allclose(got, brute.objective(X, F, reg), rtol=1e-12)


def _armijo_reference(X, F, g, reg, alpha0, shrink, c, max_trials):
    """First trial step passing the Armijo test on the dense objective, and
    the smallest distance of any tried step's test from its boundary."""
    f0 = brute.objective(X, F, reg)
    g2 = sum(float(np.sum(x * x)) for x in g)
    alpha, margin = alpha0, np.inf
    for t in range(max_trials):
        ft = brute.objective(X, [a - alpha * b for a, b in zip(F, g)], reg)
        bound = f0 - c * alpha * g2
        margin = min(margin, abs(ft - bound) / max(1.0, abs(f0)))
        if ft <= bound:
            return t + 1, alpha, margin
        alpha *= shrink
    return max_trials, 0.0, margin


@pytest.mark.parametrize("reg,alpha0", [(0.0, 1.0), (0.3, 4.0), (0.0, 0.01)])
def test_gd_step_line_search_decision(reg, alpha0):
    rng = np.random.default_rng(12)
    dims = (7, 6, 5)
    i, j, k, val = brute.random_coo(rng, dims, 60)
    F = [rng.standard_normal((d, 2)) for d in dims]
    X = brute.dense(dims, i, j, k, val)
    grads, _ = oracle.gd_grad(i, j, k, val, dims, F, reg)
    trials, alpha, margin = _armijo_reference(X, F, grads, reg, alpha0, 0.5, 1e-4, 30)
    assert margin > 1e-9, "a tried step sits on the Armijo boundary: choose another case"
    A, B, C, info = oracle.gd_step(i, j, k, val, dims, F, reg, alpha0=alpha0, shrink=0.5, c=1e-4,
                                   max_trials=30)
    assert info["accepted"] and info["trials"] == trials and info["alpha"] == alpha
    for got, f, g in zip((A, B, C), F, grads):
        np.testing.assert_allclose(got, f - alpha * g, rtol=0, atol=1e-12)
    np.testing.assert_allclose(info["f0"], brute.objective(X, F, reg), rtol=1e-12)
    np.testing.assert_allclose(info["f"], brute.objective(X, [A, B, C], reg), rtol=1e-12)
    np.testing.assert_allclose(info["gnorm2"], sum(float(np.sum(g * g)) for g in grads), rtol=1e-12)
    assert info["f"] < info["f0"]


def test_gd_step_leaves_factors_when_no_trial_passes():
    rng = np.random.default_rng(13)
    dims = (5, 4, 3)
    i, j, k, val = brute.random_coo(rng, dims, 20)
    F = [rng.standard_normal((d, 2)) for d in dims]
    A, B, C, info = oracle.gd_step(i, j, k, val, dims, F, alpha0=1e6, max_trials=1)
    assert not info["accepted"] and info["alpha"] == 0.0 and info["trials"] == 1
    assert info["f"] == info["f0"]
    for got, f in zip((A, B, C), F):
        np.testing.assert_array_equal(got, f)


def _bf16(x):
    """Round to FP32, then to BF16 (nearest, ties to even) by bit manipulation."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def test_gd_step_bf16_storage_rounds_the_update():
    rng = np.random.default_rng(14)
    dims = (6, 5, 4)
    i, j, k, val = brute.random_coo(rng, dims, 50)
    F = [_bf16(rng.standard_normal((d, 3))) for d in dims]
    grads, _ = oracle.gd_grad(i, j, k, val, dims, F)
    A, B, C, info = oracle.gd_step(i, j, k, val, dims, F, store="bf16")
    assert info["accepted"]
    for got, f, g in zip((A, B, C), F, grads):
        np.testing.assert_array_equal(got, _bf16(f - info["alpha"] * g))
        assert not np.any(got.astype(np.float32).view(np.uint32) & 0xFFFF)


def test_gd_steps_descend_on_planted_tensor():
    """From a perturbation of an exact rank-2 factorization, repeated steps
    decrease f monotonically and drive it far below its starting value."""
    coo, F, x64 = gen.planted_dense((6, 5, 4), 2, seed=15)
    rng = np.random.default_rng(16)
    G = [f + 0.05 * rng.standard_normal(f.shape) for f in F]
    f_start = oracle.objective(coo.i, coo.j, coo.k, x64, coo.dims, G)
    fs = []
    for _ in range(60):
        A, B, C, info = oracle.gd_step(coo.i, coo.j, coo.k, x64, coo.dims, G)
        assert info["accepted"] and info["f"] <= info["f0"]
        fs.append(info["f"])
        G = [A, B, C]
    assert fs[-1] < 1e-3 * f_start
