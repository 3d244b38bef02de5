"""1D finite-difference Sturm-Liouville matrices and their eigenpairs.

Paper Section 3.2 (finite difference scheme): the 1D operator
-d/dx a(x) d/dx with homogeneous Dirichlet conditions is discretised on n
interior nodes with the coefficient evaluated at the midpoints a_{i+-1/2}.
Reading used here (the paper's printed matrix carries an overall minus sign
and ad-hoc boundary rows):

    h = 1/(n+1),  A = (1/h^2) tridiag(-a_{i-1/2}, a_{i-1/2} + a_{i+1/2}, -a_{i+1/2}),

which is symmetric positive definite.  The inputs are the n+1 samples
a_{1/2}, ..., a_{n+1/2}.  The paper's literal boundary rows (diagonal
2 a_{3/2} and 2 a_{n-1/2}) are the same matrix built from the samples
returned by `paper_literal_samples`.

Section 3.3: the eigendecomposition A = V diag(lam) V^T with the columns of V
the orthonormal eigenvectors (the paper writes G^T Lambda G with G holding
eigenvectors in its columns; the transform into eigen-coordinates is V^T).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def stiffness_tridiag(a_mid: np.ndarray):
    """Diagonal and off-diagonal of A_l from the n+1 midpoint samples."""
    a_mid = np.asarray(a_mid, dtype=np.float64)
    n = a_mid.shape[0] - 1
    if n < 1:
        raise ValueError("need at least one interior node")
    h2 = 1.0 / float(n + 1) ** 2
    diag = (a_mid[:-1] + a_mid[1:]) / h2
    off = -a_mid[1:-1] / h2
    return diag, off


def stiffness_dense(a_mid: np.ndarray) -> np.ndarray:
    d, e = stiffness_tridiag(a_mid)
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def paper_literal_samples(a_mid: np.ndarray) -> np.ndarray:
    """Samples that reproduce the paper's printed boundary rows:
    a_{1/2} := a_{3/2} and a_{n+1/2} := a_{n-1/2}."""
    b = np.array(a_mid, dtype=np.float64, copy=True)
    b[0] = b[1]
    b[-1] = b[-2]
    return b


def eig1d(a_mid: np.ndarray):
    """(lam, V): ascending eigenvalues and orthonormal eigenvector columns
    of A_l (LAPACK tridiagonal solver via SciPy)."""
    d, e = stiffness_tridiag(a_mid)
    try:
        lam, V = scipy.linalg.eigh_tridiagonal(d, e, lapack_driver="stemr")
    except np.linalg.LinAlgError:
        # MRRR can fail on strongly graded matrices (a coefficient that
        # nearly vanishes); implicit QL/QR (LAPACK stev) always converges there
        lam, V = scipy.linalg.eigh_tridiagonal(d, e, lapack_driver="stev")
    return lam, np.asfortranarray(V)


def laplacian_closed_form(n: int, c: float = 1.0):
    """Eigenpairs of the constant-coefficient matrix (a = c): the textbook
    values lam_k = c (4/h^2) sin^2(k pi h / 2) and the DST-I vectors
    v_k(i) = sqrt(2h) sin(i k pi h), k, i = 1..n (Section 3.4, with the sign
    of the positive definite operator)."""
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1, dtype=np.float64)
    lam = c * 4.0 / h ** 2 * np.sin(k * np.pi * h / 2.0) ** 2
    i = np.arange(1, n + 1, dtype=np.float64)[:, None]
    V = np.sqrt(2.0 * h) * np.sin(i * k[None, :] * np.pi * h)
    return lam, V
