"""Exact solution of the discrete control equation and error evaluators.

Paper Section 3.1: after eliminating state and adjoint, the control solves

    F(A) u = y,   F(A) = beta A^-alpha + (gamma/beta) A^alpha          (1)

with A = A_1 (+) A_2 (+) A_3 the Kronecker sum of the 1D matrices (Section
3.2) and the fractional powers defined spectrally (Section 2).  With
A_l = V_l diag(lam_l) V_l^T (Section 3.3), F(A) is diagonal in the tensor
eigenbasis with entries f(lam1_i + lam2_j + lam3_k),
f(s) = beta s^-alpha + (gamma/beta) s^alpha, so

    U_hat = Y_hat / D,   D[i,j,k] = f(lam1_i + lam2_j + lam3_k),
    Y_hat = Y x_1 V_1^T x_2 V_2^T x_3 V_3^T,   U = U_hat x_1 V_1 x_2 V_2 x_3 V_3.

Index convention: a full tensor T[i1, i2, i3] is stored in C order, so that
mode l of the tensor is the l-th array axis and kron(A_1, I, I) acts on i1.
The Euclidean norm replaces the L2 norm (Section 2).

Because every V_l is orthogonal, the relative L2 error of a candidate u given
in canonical format can be evaluated in eigen-coordinates, one i1-slab at a
time, without ever forming u on the grid.
"""
from __future__ import annotations

from typing import Iterable, Optional, Sequence

import numpy as np

from . import fd


def f_control(s, alpha: float, beta: float, gamma: float):
    """f(s) = beta s^-alpha + (gamma/beta) s^alpha (control equation (1))."""
    s = np.asarray(s, dtype=np.float64)
    return beta * s ** (-alpha) + (gamma / beta) * s ** alpha


def f_state(s, alpha: float, beta: float):
    """Symbol of the state map y = beta A^-alpha u (Section 3.1)."""
    s = np.asarray(s, dtype=np.float64)
    return beta * s ** (-alpha)


class Spectral:
    """Eigenpairs of the three 1D matrices and the design function in
    eigen-coordinates for one problem."""

    def __init__(self, prob):
        self.prob = prob
        self.lam = []
        self.V = []
        for l in range(3):
            lam, V = fd.eig1d(prob.a[l])
            self.lam.append(lam)
            self.V.append(V)
        # Y_hat_l = V_l^T Y_l
        self.Yh = [self.V[l].T @ prob.Y[l] for l in range(3)]

    def D_block(self, i0: int, i1: int) -> np.ndarray:
        p = self.prob
        s = (self.lam[0][i0:i1, None, None] + self.lam[1][None, :, None]
             + self.lam[2][None, None, :])
        return f_control(s, p.alpha, p.beta, p.gamma)

    def to_eig(self, U: Sequence[np.ndarray]):
        """Factors of a canonical tensor in eigen-coordinates: V_l^T U_l."""
        return [self.V[l].T @ np.asarray(U[l], dtype=np.float64) for l in range(3)]


def cp_block(w: np.ndarray, F: Sequence[np.ndarray], i0: int, i1: int,
             chunk: int = 1 << 22) -> np.ndarray:
    """Rows i0..i1 (mode 1) of the full tensor sum_s w_s F1[:,s] o F2[:,s] o F3[:,s].
    Formed as (b x S) @ (S x n2 n3) with the Khatri-Rao product built in
    column chunks to bound memory."""
    w = np.asarray(w, dtype=np.float64)
    A = F[0][i0:i1, :] * w[None, :]
    n2, n3 = F[1].shape[0], F[2].shape[0]
    S = w.shape[0]
    out = np.empty((i1 - i0, n2, n3))
    rows = max(1, min(n2, chunk // max(1, S * n3)))
    for j0 in range(0, n2, rows):
        j1 = min(n2, j0 + rows)
        kr = (F[1][j0:j1, None, :] * F[2][None, :, :]).reshape((j1 - j0) * n3, S)
        out[:, j0:j1, :] = (A @ kr.T).reshape(i1 - i0, j1 - j0, n3)
    return out


def solve_eig_block(sp: Spectral, i0: int, i1: int) -> np.ndarray:
    """Rows i0..i1 of U_hat = Y_hat / D (the exact solution in eigen-coordinates)."""
    return cp_block(sp.prob.w, sp.Yh, i0, i1) / sp.D_block(i0, i1)


def solve_full(prob, sp: Optional[Spectral] = None) -> np.ndarray:
    """Exact u on the full n^3 grid (small n only): divide, then three mode
    products with V_1, V_2, V_3."""
    sp = sp or Spectral(prob)
    n = prob.n
    Uh = solve_eig_block(sp, 0, n)
    return mode_products(Uh, sp.V)


def state_full(prob, U: np.ndarray, sp: Optional[Spectral] = None) -> np.ndarray:
    """State y = beta A^-alpha u for a full-grid control u (Section 3.1)."""
    sp = sp or Spectral(prob)
    Uh = mode_products(U, [V.T for V in sp.V])
    s = (sp.lam[0][:, None, None] + sp.lam[1][None, :, None] + sp.lam[2][None, None, :])
    return mode_products(Uh * f_state(s, prob.alpha, prob.beta), sp.V)


def mode_products(T: np.ndarray, M: Sequence[np.ndarray]) -> np.ndarray:
    """T x_1 M_1 x_2 M_2 x_3 M_3, i.e. out[a,b,c] = sum T[i,j,k] M1[a,i] M2[b,j] M3[c,k]."""
    out = np.tensordot(M[0], T, axes=(1, 0))
    out = np.tensordot(M[1], out, axes=(1, 1)).transpose(1, 0, 2)
    out = np.tensordot(M[2], out, axes=(1, 2)).transpose(1, 2, 0)
    return np.ascontiguousarray(out)


def full_from_factors(w, F) -> np.ndarray:
    n1 = F[0].shape[0]
    return cp_block(w, F, 0, n1)


class ErrorReport(dict):
    pass


def _slab_groups(idx, block):
    """Consecutive runs of at most `block` mode-1 slab indices."""
    groups = []
    k = 0
    while k < len(idx):
        j = k
        while j + 1 < len(idx) and idx[j + 1] == idx[j] + 1 and j + 1 - k < block:
            j += 1
        groups.append((idx[k], idx[j] + 1))
        k = j + 1
    return groups


def slab_rows(w: np.ndarray, F: Sequence[np.ndarray], i0: int, i1: int) -> np.ndarray:
    """Rows i0..i1 (mode 1) of sum_s w_s F1[:,s] o F2[:,s] o F3[:,s], slab by
    slab: slab i is F2 diag(w * F1[i,:]) F3^T, one BLAS product per slab (the
    same sum as cp_block, formed in another order)."""
    w = np.asarray(w, dtype=np.float64)
    A = F[0][i0:i1, :] * w[None, :]
    return np.matmul(F[1][None, :, :] * A[:, None, :], F[2].T[None, :, :])


def _parallel_sum(fn, groups, workers):
    """Sum the tuples fn(i0, i1) returns over the slab groups, on a thread
    pool (NumPy releases the GIL in its kernels) with single-threaded BLAS
    inside, in group order (the result does not depend on the scheduling)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:   # pragma: no cover
        threadpool_limits = None
    if workers <= 1 or len(groups) <= 1:
        parts = [fn(i0, i1) for i0, i1 in groups]
    else:
        import contextlib
        limit = threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext()
        with limit, ThreadPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(lambda g: fn(*g), groups))
    tot = [0.0] * len(parts[0]) if parts else []
    for p in parts:
        for k, v in enumerate(p):
            tot[k] += v
    return tot


def rel_error(prob, w_u: np.ndarray, U_u: Sequence[np.ndarray], sp: Optional[Spectral] = None,
              slabs: Optional[Iterable[int]] = None, block: int = 8,
              workers: Optional[int] = None) -> ErrorReport:
    """Relative L2 error of a canonical candidate u = sum_t w_t U1 o U2 o U3
    against the exact solution, and the exact-operator relative residual
    ||y - F(A) u|| / ||y||.

    Both are evaluated in eigen-coordinates (V orthogonal, so the norms are
    unchanged), i1-slab by i1-slab.  With `slabs` given, only those mode-1
    slabs enter both numerator and denominator (a sampled estimate); the
    report says how many slabs were used.  Slab groups are evaluated on a
    thread pool and summed in slab order."""
    sp = sp or Spectral(prob)
    n = prob.n
    Uh = sp.to_eig(U_u)
    w_u = np.asarray(w_u, dtype=np.float64)
    idx = sorted(set(int(i) for i in slabs)) if slabs is not None else list(range(n))

    def part(i0, i1):
        D = sp.D_block(i0, i1)
        Yb = slab_rows(prob.w, sp.Yh, i0, i1)
        Ub = slab_rows(w_u, Uh, i0, i1)
        Ex = Yb / D
        return (float(np.sum((Ub - Ex) ** 2)), float(np.sum(Ex ** 2)),
                float(np.sum((Yb - D * Ub) ** 2)), float(np.sum(Yb ** 2)))

    num, den, rnum, rden = _parallel_sum(part, _slab_groups(idx, block), workers)
    rep = ErrorReport(rel_l2=float(np.sqrt(num / den)) if den > 0 else float("nan"),
                      rel_residual=float(np.sqrt(rnum / rden)) if rden > 0 else float("nan"),
                      slabs=len(idx), n=n)
    return rep


# ---- state recovery and the cost functional (Section 3.1) -----------------
#
# The state equation y = beta A^-alpha u (eqn `State`) is diagonal in the
# tensor eigenbasis with the symbol f_state(s) = beta s^-alpha.  The discrete
# cost functional of Section 3.1 with the finite-difference mass matrix M = I
# is J(y, u) = 1/2 ||y - y_Omega||^2 + gamma/2 ||u||^2 (Euclidean norms,
# Section 2); the control equation (1) is its stationarity condition after
# eliminating y, so J is smallest at the exact control.

def cost_full(prob, u: np.ndarray, y: np.ndarray) -> float:
    """J(y, u) on the full grid."""
    from .tensor import cp_full
    yom = cp_full(prob.w, prob.Y)
    return 0.5 * float(np.sum((y - yom) ** 2)) + 0.5 * prob.gamma * float(np.sum(u * u))


def cost_from_factors(prob, w_u, U_u: Sequence[np.ndarray], w_y, Y_y: Sequence[np.ndarray]) -> float:
    """J(y, u) for canonical u and y, from canonical inner products only
    (Appendix 1): ||y - y_Omega||^2 = <y,y> - 2 <y,y_Omega> + <y_Omega,y_Omega>."""
    from .tensor import cp_inner
    yy = cp_inner(w_y, Y_y, w_y, Y_y)
    yo = cp_inner(w_y, Y_y, prob.w, prob.Y)
    oo = cp_inner(prob.w, prob.Y, prob.w, prob.Y)
    uu = cp_inner(w_u, U_u, w_u, U_u)
    return 0.5 * (yy - 2.0 * yo + oo) + 0.5 * prob.gamma * uu


def state_rel_error(prob, w_y: np.ndarray, Y_y: Sequence[np.ndarray],
                    sp: Optional[Spectral] = None, slabs: Optional[Iterable[int]] = None,
                    block: int = 8, workers: Optional[int] = None) -> ErrorReport:
    """Relative L2 error of a canonical candidate state y against the exact
    state beta A^-alpha u* of the exact control u* (eigen-coordinates, slab by
    slab; with `slabs` a sampled estimate)."""
    sp = sp or Spectral(prob)
    n = prob.n
    Yy = sp.to_eig(Y_y)
    w_y = np.asarray(w_y, dtype=np.float64)
    idx = sorted(set(int(i) for i in slabs)) if slabs is not None else list(range(n))

    def part(i0, i1):
        D = sp.D_block(i0, i1)
        s = (sp.lam[0][i0:i1, None, None] + sp.lam[1][None, :, None]
             + sp.lam[2][None, None, :])
        Ex = f_state(s, prob.alpha, prob.beta) * slab_rows(prob.w, sp.Yh, i0, i1) / D
        Yb = slab_rows(w_y, Yy, i0, i1)
        return float(np.sum((Yb - Ex) ** 2)), float(np.sum(Ex ** 2))

    num, den = _parallel_sum(part, _slab_groups(idx, block), workers)
    return ErrorReport(rel_l2=float(np.sqrt(num / den)) if den > 0 else float("nan"),
                       slabs=len(idx), n=n)


def optimal_cost(prob, sp: Optional[Spectral] = None) -> float:
    """J at the exact control, evaluated on the full grid in eigen-coordinates
    (small and moderate n)."""
    sp = sp or Spectral(prob)
    n = prob.n
    s = (sp.lam[0][:, None, None] + sp.lam[1][None, :, None] + sp.lam[2][None, None, :])
    Yh = cp_block(prob.w, sp.Yh, 0, n)
    Uh = Yh / f_control(s, prob.alpha, prob.beta, prob.gamma)
    Yst = f_state(s, prob.alpha, prob.beta) * Uh
    return 0.5 * float(np.sum((Yst - Yh) ** 2)) + 0.5 * prob.gamma * float(np.sum(Uh * Uh))

