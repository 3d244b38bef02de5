"""Preconditioner case (A): the anisotropic Laplacian in the sine basis.

Test infrastructure only (CPU, FP64): nothing in the library imports it.

Section 3.5, case (A).  The constant-coefficient anisotropic operator
-sum_l b0_l d^2/dx_l^2 (eqn anisotropicL, eqn PrecClassA) discretised by the
finite-difference scheme of Section 3.2 with a_l = b0_l is the Kronecker sum

    B = b0_1 Delta (+) b0_2 Delta (+) b0_3 Delta,
    Delta = (1/h^2) tridiag(-1, 2, -1),  h = 1/(n+1),

and the preconditioner is the inverse of the weighted sum of its fractional
powers (eqn Precond_var)

    B0 = beta B^-alpha + (gamma/beta) B^alpha,   P = B0^-1.

Delta is diagonalised by the sine transform (eqn DiagLaplace): with the
orthonormal DST-I matrix S[i, k] = sqrt(2h) sin(i k pi h), i, k = 1..n
(symmetric, S S = I), Delta = S diag(mu) S with mu_k = (4/h^2) sin^2(k pi h/2)
(Section 3.4, the sign of the positive definite operator).  Hence P is
diagonal in the tensor sine basis with entries
1/f(b0_1 mu_i + b0_2 mu_j + b0_3 mu_k), f(s) = beta s^-alpha + (gamma/beta) s^alpha.

The constants are the mid-range of the coefficient (eqn modcoeff):
b0_l = (max a_l + min a_l)/2, here over the n+1 midpoint samples the
discretisation uses.  b0_l = 1 in every mode is the classical Laplacian the
paper's 3D tests precondition with (Section 4).
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .solve import f_control, mode_products


def dst1_matrix(n: int) -> np.ndarray:
    """Orthonormal DST-I matrix S[i, k] = sqrt(2/(n+1)) sin(pi i k/(n+1)),
    i, k = 1..n.  The integer product i k is reduced modulo 2(n+1) before the
    sine is taken, so large n lose no accuracy to argument reduction."""
    i = np.arange(1, n + 1, dtype=np.int64)
    m = np.outer(i, i) % (2 * (n + 1))
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * m / (n + 1))


def laplace_eigenvalues(n: int) -> np.ndarray:
    """mu_k = (4/h^2) sin^2(k pi h/2), k = 1..n, h = 1/(n+1): the eigenvalues
    of (1/h^2) tridiag(-1, 2, -1) for the sine vectors of `dst1_matrix`."""
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1, dtype=np.float64)
    return 4.0 / h ** 2 * np.sin(k * np.pi * h / 2.0) ** 2


def b0_midrange(a_mid: np.ndarray) -> float:
    """b0 = (max a + min a)/2 over the midpoint samples (eqn modcoeff)."""
    a = np.asarray(a_mid, dtype=np.float64)
    return 0.5 * (float(a.max()) + float(a.min()))


def b0_for(prob, b0: Optional[Sequence[float]] = None) -> np.ndarray:
    """Per-mode constants: the given ones where positive, else the mid-range."""
    out = np.array([b0_midrange(prob.a[l]) for l in range(3)])
    if b0 is not None:
        for l in range(3):
            if b0[l] > 0:
                out[l] = float(b0[l])
    return out


def symbol(prob, b0: Sequence[float]) -> np.ndarray:
    """P in the tensor sine basis: 1/f(b0_1 mu_i + b0_2 mu_j + b0_3 mu_k), n^3."""
    mu = laplace_eigenvalues(prob.n)
    s = (b0[0] * mu[:, None, None] + b0[1] * mu[None, :, None] + b0[2] * mu[None, None, :])
    return 1.0 / f_control(s, prob.alpha, prob.beta, prob.gamma)


def apply_full(prob, R: np.ndarray, b0: Sequence[float]) -> np.ndarray:
    """P R for a full grid tensor R (grid coordinates): sine transform in
    every mode, scale by the symbol, transform back (S is its own inverse)."""
    S = dst1_matrix(prob.n)
    Rt = mode_products(R, [S, S, S])
    return mode_products(symbol(prob, b0) * Rt, [S, S, S])


def apply_eig(prob, sp, Rh: np.ndarray, b0: Sequence[float]) -> np.ndarray:
    """P applied to a full tensor given in the eigen-coordinates of A
    (`solve.Spectral`): back to the grid with V_l, `apply_full`, forward
    with V_l^T."""
    R = mode_products(Rh, sp.V)
    Z = apply_full(prob, R, b0)
    return mode_products(Z, [V.T for V in sp.V])
