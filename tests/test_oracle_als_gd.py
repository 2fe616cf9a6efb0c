"""Pins for the oracle's CP-ALS iteration, fit and GD gradient (CPU only).

Independent references: dense least squares on the eq. (1) flattenings with
an explicit Khatri-Rao product (numpy lstsq), the Appendix A Gram identity,
least-squares optimality, dense brute-force fit and objective, central finite
differences, and recovery of planted exact low-rank tensors.
"""
import numpy as np
import pytest

import brute
import oracle
from paper_1406_4519_amd import gen


def _normalize(F):
    lam = np.linalg.norm(F, axis=0)
    out = F.copy()
    nz = lam > 0
    out[:, nz] /= lam[nz]
    return out, lam


def test_khatri_rao_gram_identity():
    """(A kr B)^T (A kr B) = A^T A * B^T B  (Appendix A)."""
    rng = np.random.default_rng(0)
    A, B = rng.standard_normal((7, 4)), rng.standard_normal((5, 4))
    K = brute.khatri_rao(A, B)
    np.testing.assert_allclose(K.T @ K, (A.T @ A) * (B.T @ B), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("reg", [0.0, 0.3])
def test_als_iteration_vs_dense_least_squares(reg):
    """Each mode update equals the (ridge) least-squares solution on the dense
    flattening with an explicit Khatri-Rao product, then unit-norm columns
    (Algorithm 2, eq. for the ridge solution in Appendix B)."""
    rng = np.random.default_rng(1)
    dims = (6, 5, 4)
    R = 3
    i, j, k, val = brute.random_coo(rng, dims, 60)
    F0 = [rng.random((d, R)) for d in dims]
    A1, B1, C1, lam, info = oracle.als_iter(i, j, k, val, dims, F0, reg)
    X = brute.dense(dims, i, j, k, val)
    A, B, C = (f.copy() for f in F0)

    def ridge(Xn, KR):
        lhs = KR.T @ KR + reg * np.eye(R)
        return np.linalg.solve(lhs, KR.T @ Xn.T).T

    A, _ = _normalize(ridge(brute.flatten(X, 0), brute.khatri_rao(C, B)))
    B, _ = _normalize(ridge(brute.flatten(X, 1), brute.khatri_rao(A, C)))
    C, lamC = _normalize(ridge(brute.flatten(X, 2), brute.khatri_rao(B, A)))
    np.testing.assert_allclose(A1, A, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(B1, B, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(C1, C, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(lam, lamC, rtol=1e-9)
    # fit of the weighted model against dense brute force
    Xh = brute.cp_full((A1, B1, C1), lam)
    fit = 1 - np.linalg.norm(X - Xh) / np.linalg.norm(X)
    np.testing.assert_allclose(info["fit"], fit, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(info["xhat_sq"], float(np.sum(Xh * Xh)), rtol=1e-9)
    np.testing.assert_allclose(info["inner_direct"], float(np.sum(X * Xh)), rtol=1e-9)
    assert info["pinv_mask"] == 0


def test_als_bf16_storage_vs_dense_least_squares():
    """store="bf16": the same dense least-squares steps, each new factor
    rounded to BF16 (through FP32, nearest-even) before the next mode uses it;
    lambda from the unrounded factor.  Rounding by gen's independent
    converter."""
    rng = np.random.default_rng(3)
    dims = (7, 6, 5)
    R = 3
    i, j, k, val = brute.random_coo(rng, dims, 90)
    F0 = [rng.random((d, R)) for d in dims]
    A1, B1, C1, lam, info = oracle.als_iter(i, j, k, val, dims, F0, 0.0, store="bf16")
    X = brute.dense(dims, i, j, k, val)

    def rnd(F):
        return gen.bf16_to_f32(gen.f32_to_bf16(F.astype(np.float32))).astype(np.float64)

    def ls(Xn, KR):
        return np.linalg.solve(KR.T @ KR, KR.T @ Xn.T).T

    A, B, C = (f.copy() for f in F0)
    A, _ = _normalize(ls(brute.flatten(X, 0), brute.khatri_rao(C, B)))
    A = rnd(A)
    B, _ = _normalize(ls(brute.flatten(X, 1), brute.khatri_rao(A, C)))
    B = rnd(B)
    C, lamC = _normalize(ls(brute.flatten(X, 2), brute.khatri_rao(B, A)))
    C = rnd(C)
    # every output is exactly a BF16 value
    for F in (A1, B1, C1):
        np.testing.assert_array_equal(F, rnd(F))
    np.testing.assert_allclose(A1, A, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(B1, B, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(C1, C, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(lam, lamC, rtol=1e-9)
    Xh = brute.cp_full((A1, B1, C1), lam)
    fit = 1 - np.linalg.norm(X - Xh) / np.linalg.norm(X)
    np.testing.assert_allclose(info["fit"], fit, rtol=1e-9, atol=1e-10)
    # and it differs from FP64 storage
    A2, B2, C2, _, _ = oracle.als_iter(i, j, k, val, dims, F0, 0.0)
    assert np.abs(C2 - C1).max() > 1e-6


def test_als_last_mode_is_least_squares_optimal():
    """Right after the mode-3 solve (before normalization), the gradient of
    the ridge objective with respect to C vanishes."""
    rng = np.random.default_rng(2)
    dims = (15, 12, 10)
    R = 4
    i, j, k, val = brute.random_coo(rng, dims, 300)
    F0 = [rng.random((d, R)) for d in dims]
    for reg in (0.0, 0.5):
        A, B, C, lam, info = oracle.als_iter(i, j, k, val, dims, F0, reg)
        Chat = C * lam[None, :]
        (gA, gB, gC), f = oracle.gd_grad(i, j, k, val, dims, (A, B, Chat), reg)
        scale = np.linalg.norm(oracle.mttkrp(i, j, k, val, dims, (A, B, Chat), 2))
        assert np.linalg.norm(gC) <= 1e-10 * max(scale, 1.0)


def test_als_residual_monotone():
    rng = np.random.default_rng(3)
    dims = (20, 18, 16)
    R = 5
    i, j, k, val = brute.random_coo(rng, dims, 800)
    F = [rng.random((d, R)) for d in dims]
    prev = -np.inf
    for _ in range(15):
        A, B, C, lam, info = oracle.als_iter(i, j, k, val, dims, F)
        F = [A, B, C]
        assert info["fit"] >= prev - 1e-12
        prev = info["fit"]


def test_als_singular_gram_uses_pseudo_inverse():
    """Two identical columns in B and C make C^T C * B^T B singular; the update
    must equal the minimum-norm least-squares solution (pseudo-inverse)."""
    rng = np.random.default_rng(4)
    dims = (6, 5, 4)
    R = 3
    i, j, k, val = brute.random_coo(rng, dims, 50)
    A0 = rng.random((dims[0], R))
    B0 = rng.random((dims[1], R))
    C0 = rng.random((dims[2], R))
    B0[:, 2] = B0[:, 1]
    C0[:, 2] = C0[:, 1]
    A1, B1, C1, lam, info = oracle.als_iter(i, j, k, val, dims, (A0, B0, C0))
    assert info["pinv_mask"] & 1
    X = brute.dense(dims, i, j, k, val)
    KR = brute.khatri_rao(C0, B0)
    Ahat = np.linalg.lstsq(KR, brute.flatten(X, 0).T, rcond=None)[0].T
    A, _ = _normalize(Ahat)
    np.testing.assert_allclose(A1, A, rtol=1e-8, atol=1e-10)


def test_als_empty_tensor():
    dims = (4, 3, 2)
    R = 2
    e = np.zeros(0, np.uint32)
    F0 = [np.ones((d, R)) for d in dims]
    A, B, C, lam, info = oracle.als_iter(e, e, e, np.zeros(0), dims, F0)
    assert info["fit"] == 0.0
    assert np.all(A == 0) and np.all(B == 0) and np.all(C == 0) and np.all(lam == 0)


def test_planted_dense_recovery():
    """Noiseless rank-5 60 x 50 x 40 tensor, every entry stored; ALS from a
    U(0,1) start reaches fit > 0.9999."""
    coo, F, x64 = gen.planted_dense((60, 50, 40), 5, seed=11)
    i, j, k = coo.i, coo.j, coo.k
    Fi = gen.init_factors(coo.dims, 5, seed=12)
    fit = 0.0
    for it in range(500):
        A, B, C, lam, info = oracle.als_iter(i, j, k, x64, coo.dims, Fi)
        Fi = [A, B, C]
        fit = info["fit"]
        if fit > 0.99999:
            break
    assert fit > 0.9999


def test_planted_sparse_recovery():
    """Exact rank-4 tensor with 40%-dense factor columns, every entry of the
    union support stored.  (ALS is a local method: at 20% density several
    seeds stall in local minima from a U(0,1) start, so 40% is used.)"""
    coo, F, x64 = gen.planted_sparse((40, 35, 30), 4, seed=22, density=0.4)
    Fi = gen.init_factors(coo.dims, 4, seed=22)
    fit = 0.0
    for it in range(500):
        A, B, C, lam, info = oracle.als_iter(coo.i, coo.j, coo.k, x64, coo.dims, Fi)
        Fi = [A, B, C]
        fit = info["fit"]
        if fit > 0.99999:
            break
    assert fit > 0.9999


# --------------------------------------------------------------------------
# GD gradient
# --------------------------------------------------------------------------

@pytest.mark.parametrize("reg", [0.0, 0.7])
def test_gd_gradient_finite_differences(reg):
    rng = np.random.default_rng(5)
    dims = (5, 4, 3)
    R = 2
    i, j, k, val = brute.random_coo(rng, dims, 25)
    F = [rng.standard_normal((d, R)) for d in dims]
    X = brute.dense(dims, i, j, k, val)
    grads, f = oracle.gd_grad(i, j, k, val, dims, F, reg)
    np.testing.assert_allclose(f, brute.objective(X, F, reg), rtol=1e-12)
    h = 1e-6
    for m in range(3):
        for idx in np.ndindex(F[m].shape):
            Fp = [x.copy() for x in F]
            Fm = [x.copy() for x in F]
            Fp[m][idx] += h
            Fm[m][idx] -= h
            fd = (brute.objective(X, Fp, reg) - brute.objective(X, Fm, reg)) / (2 * h)
            assert abs(fd - grads[m][idx]) <= 1e-6 * max(1.0, abs(fd))


def test_gd_gradient_zero_at_exact_factorization():
    coo, F, x64 = gen.planted_dense((8, 7, 6), 3, seed=31)
    grads, f = oracle.gd_grad(coo.i, coo.j, coo.k, x64, coo.dims, F, 0.0)
    for g in grads:
        assert np.max(np.abs(g)) < 1e-10
    assert abs(f) < 1e-18 + 1e-12 * float(np.sum(x64 ** 2))
