"""Pins for the oracle's joint matrix completion + tensor factorization
model (CPU only): the objective against a dense brute force, the gradient
against central finite differences of that objective, every ALS block
against per-row dense least squares solved by numpy (also with BF16 factor
storage), and monotone descent of the alternating updates."""
import numpy as np
import pytest

import brute
import oracle
from paper_1406_4519_amd import gen


def _problem(seed, dims=(6, 5, 4), nnz=40, ny=14, R=3):
    rng = np.random.default_rng(seed)
    i, j, k, val = brute.random_coo(rng, dims, nnz)
    lin = rng.choice(dims[0] * dims[1], size=ny, replace=False)
    yi, yj = (lin // dims[1]).astype(np.uint32), (lin % dims[1]).astype(np.uint32)
    yv = rng.standard_normal(ny)
    F = [rng.standard_normal((d, R)) for d in dims]
    return (i, j, k, val), (yi, yj, yv), F


def _dense_f(dims, x, y, F, mu, lam):
    X = brute.dense(dims, *x)
    A, B, C = F
    yi, yj, yv = y
    fy = 0.5 * float(np.sum((yv - np.einsum("er,er->e", A[yi], B[yj])) ** 2))
    D = X - brute.cp_full(F)
    return fy + mu * 0.5 * float(np.sum(D * D)) + 0.5 * lam * sum(float(np.sum(f * f)) for f in F)


@pytest.mark.parametrize("mu,lam", [(1.0, 0.0), (0.3, 0.5), (0.0, 0.2)])
def test_joint_objective_and_gradient(mu, lam):
    dims = (6, 5, 4)
    x, y, F = _problem(3, dims)
    g, f = oracle.joint_grad(*x, dims, *y, F, mu, lam)
    np.testing.assert_allclose(f, _dense_f(dims, x, y, F, mu, lam), rtol=1e-12)
    h = 1e-6
    for m in range(3):
        for idx in np.ndindex(F[m].shape):
            Fp = [a.copy() for a in F]
            Fm = [a.copy() for a in F]
            Fp[m][idx] += h
            Fm[m][idx] -= h
            fd = (_dense_f(dims, x, y, Fp, mu, lam) - _dense_f(dims, x, y, Fm, mu, lam)) / (2 * h)
            assert abs(fd - g[m][idx]) <= 1e-6 * max(1.0, abs(fd))


def _row_lstsq(X, y, F, mu, lam, n, row):
    """argmin over one row of factor n of the joint objective, as a stacked
    least-squares problem: ratings rows, sqrt(mu)-weighted tensor rows over
    every cell of that slice, sqrt(lam) ridge rows."""
    A, B, C = F
    R = A.shape[1]
    yi, yj, yv = y
    rows, rhs = [], []
    if n == 0:
        sel = yi == row
        rows.append(B[yj[sel]])
        rhs.append(yv[sel])
        rows.append(np.sqrt(mu) * np.einsum("jr,kr->jkr", B, C).reshape(-1, R))
        rhs.append(np.sqrt(mu) * X[row].reshape(-1))
    elif n == 1:
        sel = yj == row
        rows.append(A[yi[sel]])
        rhs.append(yv[sel])
        rows.append(np.sqrt(mu) * np.einsum("ir,kr->ikr", A, C).reshape(-1, R))
        rhs.append(np.sqrt(mu) * X[:, row, :].reshape(-1))
    else:
        rows.append(np.sqrt(mu) * np.einsum("ir,jr->ijr", A, B).reshape(-1, R))
        rhs.append(np.sqrt(mu) * X[:, :, row].reshape(-1))
    rows.append(np.sqrt(lam) * np.eye(R))
    rhs.append(np.zeros(R))
    sol, *_ = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)
    return sol


@pytest.mark.parametrize("mu,lam", [(1.0, 0.1), (0.25, 1.0)])
def test_joint_als_blocks_are_row_least_squares(mu, lam):
    dims = (6, 5, 4)
    x, y, F = _problem(4, dims)
    X = brute.dense(dims, *x)
    A, B, C, f = oracle.joint_als_iter(*x, dims, *y, F, mu, lam)
    # Gauss-Seidel: A from (B, C); B from (new A, C); C from (new A, new B)
    steps = [(0, [F[0], F[1], F[2]], A), (1, [A, F[1], F[2]], B), (2, [A, B, F[2]], C)]
    for n, cur, new in steps:
        for row in range(dims[n]):
            ref = _row_lstsq(X, y, cur, mu, lam, n, row)
            np.testing.assert_allclose(new[row], ref, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(f, _dense_f(dims, x, y, [A, B, C], mu, lam), rtol=1e-12)


def test_joint_als_bf16_storage_blocks():
    """store="bf16": every block is the same per-row least squares, from the
    factors as stored, and is then rounded to BF16 (through FP32,
    nearest-even) before the next block uses it.  Rounding by gen's
    independent converter."""
    dims = (6, 5, 4)
    x, y, F = _problem(6, dims)
    X = brute.dense(dims, *x)
    mu, lam = 0.7, 0.2

    def rnd(M):
        return gen.bf16_to_f32(gen.f32_to_bf16(M.astype(np.float32))).astype(np.float64)

    F = [rnd(f) for f in F]
    A, B, C, f = oracle.joint_als_iter(*x, dims, *y, F, mu, lam, store="bf16")
    for new in (A, B, C):
        np.testing.assert_array_equal(new, rnd(new))
    steps = [(0, [F[0], F[1], F[2]], A), (1, [A, F[1], F[2]], B), (2, [A, B, F[2]], C)]
    for n, cur, new in steps:
        ref = np.array([_row_lstsq(X, y, cur, mu, lam, n, row) for row in range(dims[n])])
        np.testing.assert_allclose(new, rnd(ref), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(f, _dense_f(dims, x, y, [A, B, C], mu, lam), rtol=1e-12)
    with pytest.raises(ValueError):
        oracle.joint_als_iter(*x, dims, *y, F, mu, lam, store="f16")


def test_joint_als_rows_equal_the_iteration():
    """joint_als_rows solves the listed rows exactly as joint_als_iter does:
    users from the initial factors, items from the updated A (bitwise, same
    arithmetic), in any order and with repeats."""
    dims = (7, 6, 5)
    x, y, F = _problem(7, dims, nnz=60, ny=20)
    A, B, C, _ = oracle.joint_als_iter(*x, dims, *y, F, 0.6, 0.3)
    users = np.array([3, 0, 6, 3])
    np.testing.assert_array_equal(oracle.joint_als_rows(*x, dims, *y, F, 0.6, 0.3, 0, users),
                                  A[users])
    items = np.arange(dims[1])[::-1]
    np.testing.assert_array_equal(
        oracle.joint_als_rows(*x, dims, *y, [A, F[1], F[2]], 0.6, 0.3, 1, items), B[items])
    with pytest.raises(ValueError):
        oracle.joint_als_rows(*x, dims, *y, F, 0.6, 0.3, 2, users)


def test_joint_als_descends():
    dims = (7, 6, 5)
    x, y, F = _problem(5, dims, nnz=60, ny=20)
    f_prev = _dense_f(dims, x, y, F, 0.5, 0.1)
    for _ in range(10):
        A, B, C, f = oracle.joint_als_iter(*x, dims, *y, F, 0.5, 0.1)
        assert f <= f_prev * (1 + 1e-12)
        f_prev = f
        F = [A, B, C]
