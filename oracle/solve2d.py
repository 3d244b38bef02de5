"""Exact solution of the two-dimensional control equation (the d = 2 variant).

Test infrastructure only (CPU, FP64): nothing in the library imports it.

Sections 2-3 with d = 2 (the 2D experiments of Section 4, Tables 4.1-4.3):
on (0,1)^2 with n interior nodes per mode, A = A_1 (+) A_2 (Kronecker sum of
the 1D finite-difference matrices of Section 3.2) and

    F(A) u = y,   F(A) = beta A^-alpha + (gamma/beta) A^alpha.

With A_l = V_l diag(lam_l) V_l^T, F(A) is diagonal in the tensor eigenbasis
with entries f(lam1_i + lam2_j), so for a design given as a sum of rank-1
matrices y = sum_s w_s Y1[:, s] Y2[:, s]^T:

    Y_hat = V_1^T y V_2,   U_hat = Y_hat / D,   u = V_1 U_hat V_2^T.

A full grid matrix T[i1, i2] has mode l on axis l - 1.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import fd
from .solve import f_control


class Spectral2D:
    """Eigenpairs of the two 1D matrices and the design in eigen-coordinates."""

    def __init__(self, prob, eig=None):
        """eig: optional [(lam, V), (lam, V)] of the same coefficients, reused."""
        self.prob = prob
        self.lam, self.V = [], []
        for l in range(2):
            lam, V = eig[l] if eig is not None else fd.eig1d(prob.a[l])
            self.lam.append(lam)
            self.V.append(V)
        self.Yh = [self.V[l].T @ prob.Y[l] for l in range(2)]

    def D(self) -> np.ndarray:
        p = self.prob
        s = self.lam[0][:, None] + self.lam[1][None, :]
        return f_control(s, p.alpha, p.beta, p.gamma)


def cp_full_2d(w, F: Sequence[np.ndarray]) -> np.ndarray:
    """sum_s w_s F1[:, s] F2[:, s]^T."""
    return (np.asarray(F[0]) * np.asarray(w, dtype=np.float64)[None, :]) @ np.asarray(F[1]).T


def solve_full_2d(prob, sp: Spectral2D = None) -> np.ndarray:
    sp = sp or Spectral2D(prob)
    Uh = cp_full_2d(prob.w, sp.Yh) / sp.D()
    return sp.V[0] @ Uh @ sp.V[1].T


def rel_error_2d(prob, w_u, U_u: Sequence[np.ndarray], sp: Spectral2D = None) -> dict:
    """Relative L2 error of u = sum_t w_t U1[:, t] U2[:, t]^T against the exact
    solution, and the relative residual ||y - F(A) u|| / ||y||, both in
    eigen-coordinates (orthogonal V_l keep the norms)."""
    sp = sp or Spectral2D(prob)
    D = sp.D()
    Yb = cp_full_2d(prob.w, sp.Yh)
    Ub = cp_full_2d(w_u, [sp.V[l].T @ np.asarray(U_u[l], dtype=np.float64) for l in range(2)])
    Ex = Yb / D
    return {"rel_l2": float(np.linalg.norm(Ub - Ex) / np.linalg.norm(Ex)),
            "rel_residual": float(np.linalg.norm(Yb - D * Ub) / np.linalg.norm(Yb)),
            "n": prob.n}
