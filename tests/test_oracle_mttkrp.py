"""Pins for the oracle's MTTKRP and flattening (CPU only).

Each check ties the oracle to something other than itself: the paper's
printed worked examples (Appendix D and Appendix A.1), dense brute force
through eq. (1) and the Khatri-Rao definition, the rank-one closed form, an
inner-product invariant, a textbook sparse-dense product special case, and
linearity in duplicated coordinates.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import brute
import oracle
from conftest import GOLDEN


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Appendix D worked example: exact integers
# --------------------------------------------------------------------------

def _appendix_d():
    g = _golden("appendix_d_example.json")
    S = np.array(g["S"], dtype=np.uint32)
    val = np.array(g["values"], dtype=np.float64)
    B = np.array(g["B"], dtype=np.float64)
    C = np.array(g["C"], dtype=np.float64)
    A = np.zeros((g["dims"][0], 2))
    return g, S[:, 0], S[:, 1], S[:, 2], val, A, B, C


def test_appendix_d_index_reading():
    """The per-nonzero products printed for columns 1 and 2 fix the reading
    of S: columns are (i, j, k), 0-based."""
    g, i, j, k, val, A, B, C = _appendix_d()
    np.testing.assert_array_equal(val * B[j, 0] * C[k, 0], g["per_nonzero_col1"])
    np.testing.assert_array_equal(val * B[j, 1] * C[k, 1], g["per_nonzero_col2"])


def test_appendix_d_mttkrp_exact():
    g, i, j, k, val, A, B, C = _appendix_d()
    M = oracle.mttkrp(i, j, k, val, g["dims"], (A, B, C), 0)
    np.testing.assert_array_equal(M, np.array(g["M"], dtype=np.float64))


def test_appendix_d_stage1_values_exact():
    """Stage 1 of Algorithm 1: value(M^r) for r = 1, 2, laid out I x K
    (reading: M^r[i, k] = sum_j x_ijk b_jr)."""
    g, i, j, k, val, A, B, C = _appendix_d()
    P = oracle.fiber_partials(i, j, k, val, 0, B)
    fl = oracle.flatten(i, j, k, val, 0)
    assert len(fl["fib_mid"]) == g["mode0_fibers"] == P.shape[0]
    I, K = g["dims"][0], g["dims"][2]
    for r, key in ((0, "M_r1"), (1, "M_r2")):
        Mr = np.zeros((I, K))
        for rt in range(len(fl["root_id"])):
            for f in range(fl["root_ptr"][rt], fl["root_ptr"][rt + 1]):
                Mr[fl["root_id"][rt], fl["fib_mid"][f]] = P[f, r]
        np.testing.assert_array_equal(Mr, np.array(g[key], dtype=np.float64))
        # second product of Algorithm 1: n_r = M^r c_r
        np.testing.assert_array_equal(Mr @ C[:, r], np.array(g["M"])[:, r])


def test_appendix_d_flattenings_exact():
    g, i, j, k, val, A, B, C = _appendix_d()
    for n, key in ((0, "X1"), (1, "X2")):
        fl = oracle.flatten(i, j, k, val, n)
        dims = g["dims"]
        leaf_dim = dims[(1, 2, 0)[n]]
        X = np.zeros((dims[n], np.prod(dims) // dims[n]))
        for rt in range(len(fl["root_id"])):
            for f in range(fl["root_ptr"][rt], fl["root_ptr"][rt + 1]):
                for e in range(fl["fib_ptr"][f], fl["fib_ptr"][f + 1]):
                    X[fl["root_id"][rt], fl["leaf"][e] + fl["fib_mid"][f] * leaf_dim] = fl["val"][e]
        np.testing.assert_array_equal(X, np.array(g[key], dtype=np.float64))


# --------------------------------------------------------------------------
# Appendix A.1 flattening example: eq. (1) for all three modes
# --------------------------------------------------------------------------

def _flat_dense(fl, dims, n):
    leaf_dim = dims[(1, 2, 0)[n]]
    X = np.zeros((dims[n], np.prod(dims) // dims[n]))
    for rt in range(len(fl["root_id"])):
        for f in range(fl["root_ptr"][rt], fl["root_ptr"][rt + 1]):
            for e in range(fl["fib_ptr"][f], fl["fib_ptr"][f + 1]):
                X[fl["root_id"][rt], fl["leaf"][e] + fl["fib_mid"][f] * leaf_dim] = fl["val"][e]
    return X


def test_appendix_a1_flattenings_exact():
    g = _golden("appendix_a1_flattening.json")
    dims = g["dims"]
    slices = np.array(g["frontal_slices"], dtype=np.float64)  # [k][i][j]
    X = np.transpose(slices, (1, 2, 0))  # [i][j][k]
    i, j, k = np.nonzero(X)
    val = X[i, j, k]
    for n, key in enumerate(("X1", "X2", "X3")):
        fl = oracle.flatten(i.astype(np.uint32), j.astype(np.uint32), k.astype(np.uint32), val, n)
        np.testing.assert_array_equal(_flat_dense(fl, dims, n), np.array(g[key], dtype=np.float64))
        # the brute-force eq. (1) helper agrees with the printed matrices too
        np.testing.assert_array_equal(brute.flatten(X, n), np.array(g[key], dtype=np.float64))


# --------------------------------------------------------------------------
# brute force, closed forms, invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mttkrp_vs_dense_khatri_rao(seed):
    rng = np.random.default_rng(seed)
    dims = (5, 4, 6)
    R = 3
    i, j, k, val = brute.random_coo(rng, dims, 40, dup=5)
    F = [rng.standard_normal((d, R)) for d in dims]
    X = brute.dense(dims, i, j, k, val)
    for n in range(3):
        got = oracle.mttkrp(i, j, k, val, dims, F, n)
        np.testing.assert_allclose(got, brute.mttkrp(X, F, n), rtol=1e-12, atol=1e-12)


def test_mttkrp_rank_one_closed_form():
    """X = a o b o c stored densely: X1 (C kr B) = a ((b^T B) * (c^T C)),
    and cyclically for modes 2 and 3."""
    rng = np.random.default_rng(7)
    dims = (4, 5, 3)
    R = 4
    a, b, c = (rng.standard_normal(d) for d in dims)
    X = np.multiply.outer(np.multiply.outer(a, b), c)
    i, j, k = (x.ravel().astype(np.uint32) for x in np.meshgrid(*map(np.arange, dims), indexing="ij"))
    val = X.ravel()
    A, B, C = (rng.standard_normal((d, R)) for d in dims)
    exp = [np.outer(a, (b @ B) * (c @ C)), np.outer(b, (a @ A) * (c @ C)), np.outer(c, (a @ A) * (b @ B))]
    for n in range(3):
        got = oracle.mttkrp(i, j, k, val, dims, (A, B, C), n)
        np.testing.assert_allclose(got, exp[n], rtol=1e-12, atol=1e-12)


def test_mttkrp_inner_product_invariant():
    """<A, M_0> = <B, M_1> = <C, M_2> = <X, [[A, B, C]]>."""
    rng = np.random.default_rng(3)
    dims = (30, 20, 25)
    R = 5
    i, j, k, val = brute.random_coo(rng, dims, 400)
    F = [rng.standard_normal((d, R)) for d in dims]
    ref = oracle.inner(i, j, k, val, F)
    X = brute.dense(dims, i, j, k, val)
    np.testing.assert_allclose(ref, float(np.sum(X * brute.cp_full(F))), rtol=1e-12)
    for n in range(3):
        M = oracle.mttkrp(i, j, k, val, dims, F, n)
        np.testing.assert_allclose(float(np.sum(F[n] * M)), ref, rtol=1e-12)


def test_mttkrp_k1_is_spmm():
    """With K = 1 mode 0 becomes the sparse-dense product X[:, :, 0] B diag(c_0)."""
    rng = np.random.default_rng(4)
    I, J = 40, 30
    R = 6
    i, j, k, val = brute.random_coo(rng, (I, J, 1), 200)
    A, B, C = (rng.standard_normal((d, R)) for d in (I, J, 1))
    S = sp.csr_matrix((val, (i.astype(np.int64), j.astype(np.int64))), shape=(I, J))
    exp = (S @ B) * C[0][None, :]
    got = oracle.mttkrp(i, j, k, val, (I, J, 1), (A, B, C), 0)
    np.testing.assert_allclose(got, exp, rtol=1e-12, atol=1e-12)


def test_mttkrp_duplicate_split_invariance():
    """Splitting each nonzero into two duplicates leaves every output unchanged."""
    rng = np.random.default_rng(5)
    dims = (12, 9, 7)
    R = 4
    i, j, k, val = brute.random_coo(rng, dims, 120)
    w = rng.random(len(val))
    i2, j2, k2 = (np.concatenate([x, x]) for x in (i, j, k))
    v2 = np.concatenate([val * w, val * (1 - w)])
    F = [rng.standard_normal((d, R)) for d in dims]
    for n in range(3):
        np.testing.assert_allclose(oracle.mttkrp(i2, j2, k2, v2, dims, F, n),
                                   oracle.mttkrp(i, j, k, val, dims, F, n), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.normsq(i2, j2, k2, v2), float(np.sum(val ** 2)), rtol=1e-12)


def test_flatten_statistics_brute_force():
    """Fiber, root and distinct counts against Python sets."""
    rng = np.random.default_rng(6)
    dims = (20, 15, 10)
    i, j, k, val = brute.random_coo(rng, dims, 300, dup=30)
    trip = set(zip(i.tolist(), j.tolist(), k.tolist()))
    order = {0: (0, 2, 1), 1: (1, 0, 2), 2: (2, 1, 0)}
    for n in range(3):
        fl = oracle.flatten(i, j, k, val, n)
        ro, mi, le = order[n]
        assert fl["nnz"] == len(trip)
        assert len(fl["fib_mid"]) == len({(t[ro], t[mi]) for t in trip})
        assert len(fl["root_id"]) == len({t[ro] for t in trip})
        # lexicographic (root, mid, leaf) order
        keys = []
        for rt in range(len(fl["root_id"])):
            for f in range(fl["root_ptr"][rt], fl["root_ptr"][rt + 1]):
                for e in range(fl["fib_ptr"][f], fl["fib_ptr"][f + 1]):
                    keys.append((fl["root_id"][rt], fl["fib_mid"][f], fl["leaf"][e]))
        assert keys == sorted(set(keys)) and len(keys) == len(trip)
    X = brute.dense(dims, i, j, k, val)
    np.testing.assert_allclose(oracle.normsq(i, j, k, val), float(np.sum(X * X)), rtol=1e-12)
