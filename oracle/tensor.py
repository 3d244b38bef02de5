"""Canonical and Tucker tensor formats, written out from their definitions
(paper Appendix 1).  Full-grid operations: meant for small n.

Canonical tensor:  T = sum_k xi_k u_k^(1) o u_k^(2) o u_k^(3)
Tucker tensor:     T = beta x_1 V^(1) x_2 V^(2) x_3 V^(3), V^(l) orthonormal.
Scalar product:    <A, B> = sum_k sum_m c_k b_m prod_l <u_k^(l), v_m^(l)>
Hadamard product:  A (.) B = sum_k sum_m c_k b_m (u_k^(1) . v_m^(1)) o ... ,
                   term (k, m) stored at column k * R_B + m.
HOSVD: the mode-l basis is the leading left singular vectors of the mode-l
unfolding T_(l); the truncated tensor is T x_l (V_l V_l^T) for all l.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def cp_full(w, F: Sequence[np.ndarray]) -> np.ndarray:
    return np.einsum("s,is,js,ks->ijk", np.asarray(w, dtype=np.float64), F[0], F[1], F[2])


def cp_inner(wa, A: Sequence[np.ndarray], wb, B: Sequence[np.ndarray]) -> float:
    G = np.ones((len(wa), len(wb)))
    for l in range(3):
        G = G * (A[l].T @ B[l])
    return float(np.asarray(wa) @ G @ np.asarray(wb))


def cp_hadamard(wa, A: Sequence[np.ndarray], wb, B: Sequence[np.ndarray]):
    wa = np.asarray(wa, dtype=np.float64)
    wb = np.asarray(wb, dtype=np.float64)
    w = (wa[:, None] * wb[None, :]).reshape(-1)
    F = []
    for l in range(3):
        n = A[l].shape[0]
        F.append((A[l][:, :, None] * B[l][:, None, :]).reshape(n, -1))
    return w, F


def unfold(T: np.ndarray, mode: int) -> np.ndarray:
    return np.moveaxis(T, mode, 0).reshape(T.shape[mode], -1)


def mode_spectra(T: np.ndarray):
    """Singular values of the three unfoldings."""
    return [np.linalg.svd(unfold(T, l), compute_uv=False) for l in range(3)]


def hosvd_truncate(T: np.ndarray, tol: float) -> Tuple[np.ndarray, Tuple[int, int, int], list]:
    """HOSVD truncation with the per-mode rank rule

        r_l = min { r : sum_{i > r} sigma_{l,i}^2 <= tol^2 ||T||^2 / 3 },

    so that ||T - T_r|| <= tol ||T|| (the HOSVD error is bounded by the sum of
    the three discarded tails).  Returns the truncated tensor, the ranks and
    the orthonormal bases."""
    nrm2 = float(np.sum(T * T))
    ranks = []
    bases = []
    for l in range(3):
        Ul, s, _ = np.linalg.svd(unfold(T, l), full_matrices=False)
        tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])
        # tail[r] = sum_{i >= r} s_i^2 (0-based) = energy dropped when keeping r
        r = int(np.argmax(tail <= tol * tol * nrm2 / 3.0))
        ranks.append(r)
        bases.append(Ul[:, :r])
    out = T
    for l in range(3):
        P = bases[l] @ bases[l].T
        out = np.moveaxis(np.tensordot(P, np.moveaxis(out, l, 0), axes=(1, 0)), 0, l)
    return out, tuple(ranks), bases


def tucker_full(core: np.ndarray, bases: Sequence[np.ndarray]) -> np.ndarray:
    return np.einsum("abc,ia,jb,kc->ijk", core, bases[0], bases[1], bases[2])
