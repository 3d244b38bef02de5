"""Brute-force checks that pin the oracle at tiny n.

* dense: assemble the n^3 x n^3 Kronecker sum A = A1 (x) I (x) I + I (x) A2 (x) I
  + I (x) I (x) A3 (Section 3.2), eigendecompose it as one dense symmetric
  matrix, form F(A) = Q f(mu) Q^T and solve F(A) u = y (no use of the 1D
  eigenbases or of the tensor structure);
* alpha = 1: beta A^-1 + (gamma/beta) A = A^-1 (beta I + (gamma/beta) A^2), so
  u solves the sparse system (beta I + (gamma/beta) A^2) u = A y, with no
  eigensolver at all.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from . import fd
from .solve import f_control
from .tensor import cp_full


def kron_sum_dense(prob) -> np.ndarray:
    n = prob.n
    I = np.eye(n)
    A = [fd.stiffness_dense(prob.a[l]) for l in range(3)]
    return (np.kron(np.kron(A[0], I), I) + np.kron(np.kron(I, A[1]), I)
            + np.kron(np.kron(I, I), A[2]))


def dense_solve(prob) -> np.ndarray:
    n = prob.n
    A = kron_sum_dense(prob)
    mu, Q = np.linalg.eigh(A)
    F = (Q * f_control(mu, prob.alpha, prob.beta, prob.gamma)[None, :]) @ Q.T
    y = cp_full(prob.w, prob.Y).reshape(-1)
    return np.linalg.solve(F, y).reshape(n, n, n)


def dense_operator_apply(prob, u: np.ndarray) -> np.ndarray:
    A = kron_sum_dense(prob)
    mu, Q = np.linalg.eigh(A)
    F = (Q * f_control(mu, prob.alpha, prob.beta, prob.gamma)[None, :]) @ Q.T
    return (F @ u.reshape(-1)).reshape(u.shape)


def sparse_alpha1_solve(prob) -> np.ndarray:
    if prob.alpha != 1.0:
        raise ValueError("identity holds for alpha = 1 only")
    n = prob.n
    I = sps.identity(n, format="csr")
    A1 = []
    for l in range(3):
        d, e = fd.stiffness_tridiag(prob.a[l])
        A1.append(sps.diags([e, d, e], [-1, 0, 1], format="csr"))
    A = (sps.kron(sps.kron(A1[0], I), I) + sps.kron(sps.kron(I, A1[1]), I)
         + sps.kron(sps.kron(I, I), A1[2])).tocsr()
    N = n ** 3
    M = prob.beta * sps.identity(N, format="csr") + (prob.gamma / prob.beta) * (A @ A)
    y = cp_full(prob.w, prob.Y).reshape(-1)
    u = spla.spsolve(M.tocsc(), A @ y)
    return u.reshape(n, n, n)


# ---- d = 2 ------------------------------------------------------------------

def kron_sum_dense_2d(prob) -> np.ndarray:
    n = prob.n
    I = np.eye(n)
    A = [fd.stiffness_dense(prob.a[l]) for l in range(2)]
    return np.kron(A[0], I) + np.kron(I, A[1])


def dense_solve_2d(prob) -> np.ndarray:
    """F(A) u = y with the n^2 x n^2 Kronecker sum eigendecomposed as one dense
    symmetric matrix."""
    n = prob.n
    mu, Q = np.linalg.eigh(kron_sum_dense_2d(prob))
    F = (Q * f_control(mu, prob.alpha, prob.beta, prob.gamma)[None, :]) @ Q.T
    y = (prob.Y[0] * prob.w[None, :]) @ prob.Y[1].T
    return np.linalg.solve(F, y.reshape(-1)).reshape(n, n)


def sparse_alpha1_solve_2d(prob) -> np.ndarray:
    """alpha = 1: (beta I + (gamma/beta) A^2) u = A y, no eigensolver."""
    if prob.alpha != 1.0:
        raise ValueError("identity holds for alpha = 1 only")
    n = prob.n
    I = sps.identity(n, format="csr")
    A1 = []
    for l in range(2):
        d, e = fd.stiffness_tridiag(prob.a[l])
        A1.append(sps.diags([e, d, e], [-1, 0, 1], format="csr"))
    A = (sps.kron(A1[0], I) + sps.kron(I, A1[1])).tocsr()
    M = prob.beta * sps.identity(n * n, format="csr") + (prob.gamma / prob.beta) * (A @ A)
    y = ((prob.Y[0] * prob.w[None, :]) @ prob.Y[1].T).reshape(-1)
    return spla.spsolve(M.tocsc(), A @ y).reshape(n, n)
