"""Brute-force dense references used only to pin the oracle.

Everything here is built directly from the paper's definitions on tiny
tensors: the dense tensor, its flattenings by eq. (1) (Section 2.1), and the
Khatri-Rao product column by column as Kronecker products of columns
(Appendix A).  No code is shared with the oracle or with the HIP library.
"""
import numpy as np


def dense(dims, i, j, k, val):
    X = np.zeros(tuple(int(d) for d in dims), dtype=np.float64)
    np.add.at(X, (np.asarray(i, np.int64), np.asarray(j, np.int64), np.asarray(k, np.int64)),
              np.asarray(val, np.float64))
    return X


def flatten(X, n):
    """Paper mode n+1 flattening by eq. (1) (0-based):
    X1[i, j + k J], X2[j, k + i K], X3[k, i + j I]."""
    I, J, K = X.shape
    if n == 0:
        out = np.zeros((I, J * K))
        for i in range(I):
            for j in range(J):
                for k in range(K):
                    out[i, j + k * J] = X[i, j, k]
    elif n == 1:
        out = np.zeros((J, K * I))
        for i in range(I):
            for j in range(J):
                for k in range(K):
                    out[j, k + i * K] = X[i, j, k]
    else:
        out = np.zeros((K, I * J))
        for i in range(I):
            for j in range(J):
                for k in range(K):
                    out[k, i + j * I] = X[i, j, k]
    return out


def khatri_rao(A, B):
    """A kr B: column r is the Kronecker product of column r of A and of B."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    assert A.shape[1] == B.shape[1]
    return np.stack([np.kron(A[:, r], B[:, r]) for r in range(A.shape[1])], axis=1)


def mttkrp(X, factors, n):
    """X^{n+1} times the Khatri-Rao product used by Algorithm 2:
    X1 (C kr B), X2 (A kr C), X3 (B kr A)."""
    A, B, C = factors
    if n == 0:
        return flatten(X, 0) @ khatri_rao(C, B)
    if n == 1:
        return flatten(X, 1) @ khatri_rao(A, C)
    return flatten(X, 2) @ khatri_rao(B, A)


def cp_full(factors, lam=None):
    A, B, C = (np.asarray(f, np.float64) for f in factors)
    R = A.shape[1]
    lam = np.ones(R) if lam is None else np.asarray(lam, np.float64)
    X = np.zeros((A.shape[0], B.shape[0], C.shape[0]))
    for r in range(R):
        X += lam[r] * np.multiply.outer(np.multiply.outer(A[:, r], B[:, r]), C[:, r])
    return X


def objective(X, factors, reg=0.0):
    """f = 1/2 sum over all (i,j,k) of (x - xhat)^2 + 1/2 reg sum ||F||^2."""
    D = X - cp_full(factors)
    return 0.5 * float(np.sum(D * D)) + 0.5 * reg * sum(float(np.sum(np.asarray(F) ** 2))
                                                        for F in factors)


def random_coo(rng, dims, nnz, dup=0):
    I, J, K = dims
    lin = rng.choice(I * J * K, size=nnz, replace=False)
    i, j, k = lin // (J * K), (lin // K) % J, lin % K
    val = rng.standard_normal(nnz)
    if dup:
        pick = rng.integers(0, nnz, dup)
        i = np.concatenate([i, i[pick]])
        j = np.concatenate([j, j[pick]])
        k = np.concatenate([k, k[pick]])
        val = np.concatenate([val, rng.standard_normal(dup)])
    return (i.astype(np.uint32), j.astype(np.uint32), k.astype(np.uint32), val)
