"""Seeded synthetic inputs for the fractional control equation.

This module only draws numbers and samples the closed-form input functions
(coefficients a_l and Gaussian-bump design functions y_Omega).  It holds none of
the method's arithmetic, so that both the CPU oracle and the GPU path can
consume the very same inputs.

Grid convention: n interior nodes per mode, h = 1/(n+1), nodes x_i = i*h
(i = 1..n); the coefficient a_l is sampled at the n+1 midpoints (i+1/2)*h,
i = 0..n (finite-difference scheme of Section 3.2 of the paper).

The paper's own design functions (box- and H-type shapes, Section 4) are given
only as figures, so smooth Gaussian bumps stand in for them.

Draw order (numpy.random.default_rng(seed)):
  * configs with per-mode random coefficients draw the three coefficient
    parameters first, in mode order;
  * then, for each rank term s: the weight w_s, then (centre, width) for
    mode 1, 2, 3.
The batched workload draws, per problem: n, rank, alpha, the three
coefficient parameters, then the rank terms as above.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

__all__ = [
    "Problem",
    "nodes",
    "midpoints",
    "gaussian_bumps",
    "workload_small",
    "workload_quadratic",
    "workload_sine",
    "workload_batched",
    "workload_batched_uniform",
    "workload_paper_shaped",
    "eigvec_rhs_problem",
    "workload_paper_2d",
    "workload_quadratic_2d",
]


@dataclasses.dataclass
class Problem:
    """One instance of (beta A^-alpha + (gamma/beta) A^alpha) u = y.

    a     : list of three float64 arrays of length n+1 (midpoint samples)
    w     : float64 weights of the canonical design function, length S
    Y     : list of three float64 arrays n x S (Fortran order), factor columns
    """

    name: str
    n: int
    a: List[np.ndarray]
    alpha: float
    beta: float
    gamma: float
    eps: float
    w: np.ndarray
    Y: List[np.ndarray]

    @property
    def rank(self) -> int:
        return int(self.w.shape[0])


def nodes(n: int) -> np.ndarray:
    """Interior nodes x_i = i/(n+1), i = 1..n."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def midpoints(n: int) -> np.ndarray:
    """Midpoints (i+1/2)/(n+1), i = 0..n, where a_l is sampled."""
    return (np.arange(0, n + 1, dtype=np.float64) + 0.5) / (n + 1)


def gaussian_bumps(n: int, centres: Sequence[float], widths: Sequence[float]) -> np.ndarray:
    """n x S Fortran-ordered matrix of exp(-(x-mu)^2 / (2 sigma^2)) at the nodes."""
    x = nodes(n)[:, None]
    mu = np.asarray(centres, dtype=np.float64)[None, :]
    sg = np.asarray(widths, dtype=np.float64)[None, :]
    return np.asfortranarray(np.exp(-((x - mu) ** 2) / (2.0 * sg * sg)))


def _draw_bumps(rng: np.random.Generator, n: int, rank: int):
    w = np.empty(rank)
    mu = np.empty((3, rank))
    sg = np.empty((3, rank))
    for s in range(rank):
        w[s] = rng.uniform(0.5, 1.5)
        for l in range(3):
            mu[l, s] = rng.uniform(0.2, 0.8)
            sg[l, s] = rng.uniform(0.05, 0.2)
    Y = [gaussian_bumps(n, mu[l], sg[l]) for l in range(3)]
    return w, Y


def workload_small(n: int = 32) -> Problem:
    """n=32, a_l = 1 + 0.5 sin(2 pi x) in every mode, alpha=0.5, beta=1e-2,
    gamma=1, rank-1 design g(x1) g(x2) g(x3), g = Gaussian at 0.5, sigma 0.1."""
    xm = midpoints(n)
    a = [1.0 + 0.5 * np.sin(2.0 * np.pi * xm) for _ in range(3)]
    g = gaussian_bumps(n, [0.5], [0.1])
    return Problem("small_n32", n, a, 0.5, 1e-2, 1.0, 1e-6, np.ones(1), [g.copy(), g.copy(), g.copy()])


def workload_quadratic(alpha: float = 0.5, n: int = 256, seed: int = 2, rank: int = 5,
                       beta: float = 1e-3) -> Problem:
    """a_l = 1 + c_l x^2, c_l ~ U[0.5, 2]; rank-5 Gaussian-bump design."""
    rng = np.random.default_rng(seed)
    c = [rng.uniform(0.5, 2.0) for _ in range(3)]
    xm = midpoints(n)
    a = [1.0 + c[l] * xm * xm for l in range(3)]
    w, Y = _draw_bumps(rng, n, rank)
    return Problem(f"quadratic_n{n}_a{alpha:g}", n, a, float(alpha), beta, 1.0, 1e-6, w, Y)


def workload_sine(n: int = 1024, seed: int = 3, rank: int = 10, alpha: float = 0.5,
                  beta: float = 1e-4) -> Problem:
    """a_l = 1 + 0.9 sin(4 pi x + phi_l), phi_l ~ U[0, 2 pi); rank-10 bumps.

    The same seed at a smaller n gives the same phases and bumps on the
    coarser grid (the subproblem used for full-grid checks)."""
    rng = np.random.default_rng(seed)
    phi = [rng.uniform(0.0, 2.0 * np.pi) for _ in range(3)]
    xm = midpoints(n)
    a = [1.0 + 0.9 * np.sin(4.0 * np.pi * xm + phi[l]) for l in range(3)]
    w, Y = _draw_bumps(rng, n, rank)
    return Problem(f"sine_n{n}", n, a, float(alpha), beta, 1.0, 1e-6, w, Y)


def workload_batched(count: int = 64, seed: int = 5,
                     sizes: Sequence[int] = (64, 128, 256, 512, 1024, 2048),
                     beta: float = 1e-3) -> List[Problem]:
    """Independent problems of uneven size and rank: n from `sizes`,
    rank ~ randint[1, 10], alpha ~ U[0.2, 0.8], coefficients as in the
    quadratic workload, bumps as above."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        rank = int(rng.integers(1, 11))
        alpha = float(rng.uniform(0.2, 0.8))
        c = [rng.uniform(0.5, 2.0) for _ in range(3)]
        xm = midpoints(n)
        a = [1.0 + c[l] * xm * xm for l in range(3)]
        w, Y = _draw_bumps(rng, n, rank)
        out.append(Problem(f"batched{p}_n{n}", n, a, alpha, beta, 1.0, 1e-6, w, Y))
    return out


def workload_batched_uniform(count: int = 64, n: int = 1024, seed0: int = 100) -> List[Problem]:
    """`count` problems at one size, distributed like the sine workload,
    seeds seed0 .. seed0+count-1."""
    return [workload_sine(n=n, seed=seed0 + p) for p in range(count)]


def workload_paper_shaped(n: int, alpha: float) -> Problem:
    """Coefficients of the paper's 3D tests with the shifted second
    coefficient (sin x cos x + 0.1), beta = gamma = 1, and a rank-1 box
    indicator on [0.25, 0.75]^3 standing in for the unavailable H-shape."""
    xm = midpoints(n)
    a = [np.sin(100.0 * np.pi * xm) + 1.1,
         np.sin(xm) * np.cos(xm) + 0.1,
         np.cos(5.0 * np.pi * xm) + 2.0]
    x = nodes(n)
    box = ((x >= 0.25) & (x <= 0.75)).astype(np.float64)[:, None]
    return Problem(f"paper_n{n}_a{alpha:g}", n, a, float(alpha), 1.0, 1.0, 1e-6, np.ones(1),
                   [np.asfortranarray(box.copy()) for _ in range(3)])


def eigvec_rhs_problem(base: Problem, vecs: Sequence[np.ndarray]) -> Problem:
    """Same operator as `base`, with the rank-1 design v1 (x) v2 (x) v3."""
    Y = [np.asfortranarray(np.asarray(v, dtype=np.float64).reshape(-1, 1)) for v in vecs]
    return dataclasses.replace(base, name=base.name + "_eigvec", w=np.ones(1), Y=Y)


# ---- d = 2 (two-entry lists a and Y) ----------------------------------------

def workload_paper_2d(n: int, alpha: float, gamma: float = 1.0) -> Problem:
    """The paper's 2D tests: a_1 = sin(100 pi x) + 1.1, a_2 = sin x cos x,
    beta = 1, a rank-1 box indicator on [0.25, 0.75]^2 standing in for the
    box-type design."""
    xm = midpoints(n)
    a = [np.sin(100.0 * np.pi * xm) + 1.1, np.sin(xm) * np.cos(xm)]
    x = nodes(n)
    box = ((x >= 0.25) & (x <= 0.75)).astype(np.float64)[:, None]
    return Problem(f"paper2d_n{n}_a{alpha:g}", n, a, float(alpha), 1.0, float(gamma), 1e-6,
                   np.ones(1), [np.asfortranarray(box.copy()) for _ in range(2)])


def workload_quadratic_2d(alpha: float = 0.5, n: int = 256, seed: int = 2, rank: int = 5,
                          beta: float = 1e-3) -> Problem:
    """The quadratic-coefficient family in two modes: the same draws as
    `workload_quadratic` (three coefficient parameters, then per rank term a
    weight and three bumps), of which the first two modes are used."""
    p = workload_quadratic(alpha=alpha, n=n, seed=seed, rank=rank, beta=beta)
    return dataclasses.replace(p, name=f"quadratic2d_n{n}_a{alpha:g}", a=p.a[:2], Y=p.Y[:2])
